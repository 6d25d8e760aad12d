"""Python binding of libozaki: emulated-FP64 (Ozaki scheme) GEMM, two-site
H_eff.psi and a Davidson step on MI355X (gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libozaki.so.  PyTorch supplies device memory (``data_ptr``) and
streams.  The library must have been built (``python -m
paper_2510_04795_amd._build``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libozaki.so")

OZ_OK, OZ_CONVERGED, OZ_STAGNATED, OZ_MAX_ITER = 0, 1, 2, 3
OZ_STATIC_WORKSPACE_BYTES = 96 << 20
OZ_FLAG_NONFINITE = 1
OZ_EXP_NONFINITE = -(2 ** 31)
OZ_HEFF_LAUNCH_RESIDENT = -2
OZ_HEFF_LAUNCH_PAIRED_TERMS = -3
PHASES = {1: "slice", 2: "pair", 3: "fp64", 4: "heff_L", 5: "heff_R", 6: "heff_aux"}
STATUS = {0: "running", 1: "converged", 2: "stagnated", 3: "max_iter"}

if not os.path.exists(LIB_PATH):
    raise ImportError("libozaki.so is not built: run `python -m paper_2510_04795_amd._build` "
                      "(expected at %s)" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)
_i32, _i64, _dbl, _ptr, _sz = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class HeffTriple(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("lo", ctypes.c_int32), ("li", ctypes.c_int32),
                ("ri", ctypes.c_int32), ("ro", ctypes.c_int32), ("alpha", ctypes.c_double)]


class HeffLayout(ctypes.Structure):
    _fields_ = [("n_left", ctypes.c_int32), ("n_right", ctypes.c_int32), ("phys", ctypes.c_int32),
                ("left_dim", _ptr), ("right_dim", _ptr),
                ("n_psi_blocks", ctypes.c_int32), ("psi_lr", _ptr), ("psi_offset", _ptr),
                ("n_L_blocks", ctypes.c_int32), ("L_key", _ptr), ("L_offset", _ptr),
                ("n_R_blocks", ctypes.c_int32), ("R_key", _ptr), ("R_offset", _ptr)]


class DavidsonInfo(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("resnorm", ctypes.c_double), ("iter", ctypes.c_int32),
                ("m", ctypes.c_int32), ("status", ctypes.c_int32)]


class RdmEigInfo(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("status", ctypes.c_int32), ("off", ctypes.c_double),
                ("trace", ctypes.c_double)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("ozaki_status_string", ctypes.c_char_p, [_i32])
_sig("ozaki_last_error", ctypes.c_char_p, [])
_sig("ozaki_version", _i32, [])
_sig("ozaki_ctx_create", _i32, [ctypes.POINTER(_ptr), _i32])
_sig("ozaki_ctx_destroy", _i32, [_ptr])
_sig("ozaki_ctx_flags", _i32, [_ptr, ctypes.POINTER(ctypes.c_uint32)])
_sig("ozaki_ctx_set_timing", _i32, [_ptr, _i32])
_sig("ozaki_ctx_phase_times", _i32, [_ptr, _ptr, _ptr, _i32])
_sig("ozaki_pair_variants", _i32, [_i32, _i32, _ptr, _ptr, _i32])
_sig("ozaki_ctx_set_variant", _i32, [_ptr, _i32, _i32, _i32])
_sig("ozaki_ctx_get_variant", _i32, [_ptr, _i32, _i32])
_sig("ozaki_ctx_set_autotune", _i32, [_ptr, _i32])
_sig("ozaki_dgemm_tune", _i32, [_ptr, ctypes.c_char, ctypes.c_char, _i64, _i64, _i64, _ptr, _i64, _ptr,
                                _i64, _ptr, _i64, _i32, _i32, _ptr, _sz, _ptr, _ptr])
_sig("heff_plan_variants", _i32, [_ptr, _ptr, _ptr])
_sig("heff_plan_launches", _i32, [_ptr, _ptr, _ptr])
_sig("ozaki_ctx_set_heff_launch", _i32, [_ptr, _i32])
_sig("ozaki_ctx_set_heff_budget", _i32, [_ptr, _sz])
_sig("ozaki_ctx_set_heff_phase", _i32, [_ptr, _i32, _i32, _i32, _i32])
_sig("ozaki_slices_for_bits", _i32, [_i32])
_sig("ozaki_pair_count", _i32, [_i32, _i32])
_sig("ozaki_max_exact_k", _i64, [_i32, _i32])
_sig("ozaki_dgemm_workspace_bytes", _sz, [_i64, _i64, _i64, _i32, _i32])
_sig("ozaki_dgemm", _i32, [_ptr, ctypes.c_char, ctypes.c_char, _i64, _i64, _i64, _dbl, _ptr, _i64,
                           _ptr, _i64, _dbl, _ptr, _i64, _i32, _i32, _ptr, _sz, _ptr])
_sig("ozaki_dgemm_static", _i32, [_ptr, ctypes.c_char, ctypes.c_char, _i64, _i64, _i64, _dbl, _ptr, _i64,
                                  _ptr, _i64, _dbl, _ptr, _i64, _i32, _i32, _ptr])
_sig("ozaki_dgemm_auto_workspace_bytes", _sz, [_i64, _i64, _i64])
_sig("ozaki_choose_slices", _i32, [_ptr, ctypes.c_char, ctypes.c_char, _i64, _i64, _i64, _ptr, _i64, _ptr,
                                   _i64, _ptr, _sz, _ptr, _ptr, _ptr, _ptr])
_sig("ozaki_dgemm_auto", _i32, [_ptr, ctypes.c_char, ctypes.c_char, _i64, _i64, _i64, _dbl, _ptr, _i64,
                                _ptr, _i64, _dbl, _ptr, _i64, _i32, _i32, _ptr, _sz, _ptr, _ptr, _ptr])
_sig("ozaki_split", _i32, [_ptr, _i32, _i64, _i64, _ptr, _i64, _i32, _ptr, _ptr, _ptr])
_sig("ozaki_pair_products", _i32, [_ptr, _i64, _i64, _i64, _i32, _i32, _ptr, _ptr, _ptr, _ptr])
_sig("heff_plan_create", _i32, [_ptr, ctypes.POINTER(_ptr), ctypes.POINTER(HeffLayout), _ptr, _ptr,
                                _i32, ctypes.POINTER(HeffTriple), _ptr, _i32, _i32, _ptr])
_sig("heff_apply", _i32, [_ptr, _ptr, _ptr, _ptr])
_sig("heff_plan_set_graphs", _i32, [_ptr, _i32])
_sig("heff_plan_graph_count", _i32, [_ptr])
_sig("heff_vector_length", _i64, [_ptr])
_sig("heff_plan_chunks", _i32, [_ptr])
_sig("heff_plan_phase", _i32, [_ptr, _i32, _ptr, _ptr, _ptr])
_sig("heff_plan_bytes", _i64, [_ptr, _ptr])
_sig("heff_flops", _dbl, [_ptr])
_sig("heff_plan_destroy", _i32, [_ptr])
_sig("davidson_create", _i32, [_ptr, ctypes.POINTER(_ptr), _ptr, _ptr, _ptr, _i32, _dbl, _i32, _ptr])
_sig("davidson_step", _i32, [_ptr, ctypes.POINTER(DavidsonInfo), _ptr])
_sig("davidson_get_vector", _i32, [_ptr, _ptr, _ptr])
_sig("davidson_set_graphs", _i32, [_ptr, _i32])
_sig("davidson_graph_count", _i32, [_ptr])
_sig("davidson_destroy", _i32, [_ptr])
_sig("lanczos_create", _i32, [_ptr, ctypes.POINTER(_ptr), _ptr, _ptr, _i32, _dbl, _i32, _ptr])
_sig("lanczos_step", _i32, [_ptr, ctypes.POINTER(DavidsonInfo), _ptr])
_sig("lanczos_get_vector", _i32, [_ptr, _ptr, _ptr])
_sig("lanczos_destroy", _i32, [_ptr])
_sig("rdm_eig_create", _i32, [_ptr, ctypes.POINTER(_ptr), _i64, _i32, _i32])
_sig("rdm_eig_solve", _i32, [_ptr, _ptr, _i64, _i64, _ptr, _ptr, _i64, _dbl, _i32,
                             ctypes.POINTER(RdmEigInfo), _ptr])
_sig("rdm_eig_destroy", _i32, [_ptr])
_sig("ozaki_renormalize_workspace_bytes", _sz, [_i64, _i64, _i32, _i32])
_sig("ozaki_renormalize", _i32, [_ptr, _i64, _i64, _ptr, _i64, _i32, ctypes.POINTER(_ptr), _i64,
                                 ctypes.POINTER(_ptr), _i64, _i32, _i32, _ptr, _sz, _ptr])

EXPORTED = [
    "ozaki_status_string", "ozaki_last_error", "ozaki_version", "ozaki_ctx_create",
    "ozaki_ctx_destroy", "ozaki_ctx_flags", "ozaki_ctx_set_timing", "ozaki_ctx_phase_times",
    "ozaki_pair_variants", "ozaki_ctx_set_variant", "ozaki_ctx_get_variant",
    "ozaki_ctx_set_autotune", "ozaki_ctx_set_heff_launch", "ozaki_ctx_set_heff_budget",
    "ozaki_ctx_set_heff_phase", "ozaki_dgemm_tune", "heff_plan_variants",
    "heff_plan_launches", "ozaki_slices_for_bits", "ozaki_pair_count",
    "ozaki_max_exact_k", "ozaki_dgemm_workspace_bytes", "ozaki_dgemm", "ozaki_dgemm_static", "ozaki_split",
    "ozaki_choose_slices", "ozaki_dgemm_auto_workspace_bytes", "ozaki_dgemm_auto",
    "ozaki_pair_products", "heff_plan_create", "heff_apply", "heff_plan_set_graphs",
    "heff_plan_graph_count", "heff_vector_length", "heff_plan_chunks", "heff_plan_bytes",
    "heff_plan_phase", "heff_flops",
    "heff_plan_destroy", "davidson_create", "davidson_step", "davidson_get_vector",
    "davidson_set_graphs", "davidson_graph_count", "davidson_destroy", "lanczos_create", "lanczos_step", "lanczos_get_vector", "lanczos_destroy",
    "rdm_eig_create", "rdm_eig_solve", "rdm_eig_destroy", "ozaki_renormalize_workspace_bytes",
    "ozaki_renormalize",
]


class OzakiError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.ozaki_last_error().decode() or _lib.ozaki_status_string(status).decode()
        super().__init__("%s: %s (status %d)" % (where, msg, status))
        self.status = status


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise OzakiError(rc, where)
    return rc


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("%s must be a float64 CUDA tensor" % name)
    return t


def _dev_vec(t: torch.Tensor, n: int, name: str) -> torch.Tensor:
    """A float64 CUDA vector the library reads or writes n elements of."""
    _dev_f64(t, name)
    if t.numel() != n or not t.is_contiguous():
        raise ValueError("%s must be contiguous with %d elements" % (name, n))
    return t


def _dev_out(t: torch.Tensor, rows: int, cols: int, name: str) -> torch.Tensor:
    """A float64 CUDA matrix of rows x cols the library writes."""
    _dev_f64(t, name)
    if tuple(t.shape) != (rows, cols):
        raise ValueError("%s must be %d x %d, not %s" % (name, rows, cols, tuple(t.shape)))
    return t


def _ld(t: torch.Tensor, name: str) -> int:
    """Leading dimension of a row-major 2-D view (unit column stride)."""
    if t.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    if t.numel() == 0:
        return max(t.size(1), 1)
    if t.size(1) > 1 and t.stride(1) != 1:
        raise ValueError("%s must be a row-major 2-D tensor with unit column stride" % name)
    return max(t.stride(0), t.size(1), 1)


def pair_variants(slices: int, ndiag: int = 0):
    """[(variant, tile_m, tile_n)] of the built tile variants for (slices, ndiag)."""
    import numpy as np
    tm = np.zeros(16, dtype=np.int32)
    tn = np.zeros(16, dtype=np.int32)
    n = _check(_lib.ozaki_pair_variants(slices, ndiag, tm.ctypes.data, tn.ctypes.data, 16),
               "ozaki_pair_variants")
    return [(v, int(tm[v]), int(tn[v])) for v in range(n) if tm[v] > 0]


def slices_for_bits(bits: int) -> int:
    return _check(_lib.ozaki_slices_for_bits(bits), "ozaki_slices_for_bits")


def pair_count(slices: int, ndiag: int = 0) -> int:
    return _check(_lib.ozaki_pair_count(slices, ndiag), "ozaki_pair_count")


def max_exact_k(slices: int, ndiag: int = 0) -> int:
    return _check(_lib.ozaki_max_exact_k(slices, ndiag), "ozaki_max_exact_k")


def workspace_bytes(M: int, N: int, K: int, slices: int, ndiag: int = 0) -> int:
    return int(_lib.ozaki_dgemm_workspace_bytes(M, N, K, slices, ndiag))


class Context:
    """An ozaki_ctx bound to one device."""

    def __init__(self, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        h = _ptr()
        _check(_lib.ozaki_ctx_create(ctypes.byref(h), device), "ozaki_ctx_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _lib.ozaki_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def flags(self) -> int:
        v = ctypes.c_uint32(0)
        _check(_lib.ozaki_ctx_flags(self.handle, ctypes.byref(v)), "ozaki_ctx_flags")
        return int(v.value)

    def set_timing(self, enable: bool = True):
        _check(_lib.ozaki_ctx_set_timing(self.handle, int(bool(enable))), "ozaki_ctx_set_timing")

    def phase_times(self, max_phases: int = 8192):
        """[(phase name, ms)] recorded since the last call (waits for the events)."""
        import numpy as np
        ph = np.zeros(max_phases, dtype=np.int32)
        ms = np.zeros(max_phases, dtype=np.float64)
        n = _check(_lib.ozaki_ctx_phase_times(self.handle, ph.ctypes.data, ms.ctypes.data,
                                              max_phases), "ozaki_ctx_phase_times")
        return [(PHASES.get(int(p), str(int(p))), float(t)) for p, t in zip(ph[:n], ms[:n])]

    def set_variant(self, slices: int, ndiag: int = 0, variant: int = -1):
        _check(_lib.ozaki_ctx_set_variant(self.handle, slices, ndiag, variant), "ozaki_ctx_set_variant")

    def get_variant(self, slices: int, ndiag: int = 0) -> int:
        return _check(_lib.ozaki_ctx_get_variant(self.handle, slices, ndiag), "ozaki_ctx_get_variant")

    def set_autotune(self, enable: bool = True):
        _check(_lib.ozaki_ctx_set_autotune(self.handle, int(bool(enable))), "ozaki_ctx_set_autotune")

    def set_heff_launch(self, mode: int = -1):
        """Launch of later heff plans' grouped phases: 0 one workgroup per
        tile, k > 0 streamed on k compute units (capped at the device's),
        OZ_HEFF_LAUNCH_RESIDENT the resident kernel for the first phase
        where it is built for the tile variant, OZ_HEFF_LAUNCH_PAIRED_TERMS
        the paired-term kernel for the second phase where built, -1 timed
        choice (default)."""
        _check(_lib.ozaki_ctx_set_heff_launch(self.handle, int(mode)), "ozaki_ctx_set_heff_launch")

    def set_heff_phase(self, phase: int, variant: int = -1, order: int = 0, launch: int = 0):
        """Fix grouped phase `phase` (0 first product, 1 second) of later
        emulated heff plans: tile variant (-1 clears), order (0 XCD parts,
        1 longest tile first, 2 whole outputs per XCD, heaviest first to the
        least loaded), launch (0 per tile, k > 0 streamed on k CUs,
        OZ_HEFF_LAUNCH_RESIDENT resident, first phase only,
        OZ_HEFF_LAUNCH_PAIRED_TERMS paired terms, second phase only).
        With both phases fixed a plan times nothing."""
        _check(_lib.ozaki_ctx_set_heff_phase(self.handle, int(phase), int(variant), int(order), int(launch)),
               "ozaki_ctx_set_heff_phase")

    def set_heff_budget(self, nbytes: int = 0):
        """Device bytes later heff plans may use for their intermediates T
        (0 = the library default of 8 GiB); the triple list runs in chunks
        that fit, with bit-identical results."""
        _check(_lib.ozaki_ctx_set_heff_budget(self.handle, int(nbytes)), "ozaki_ctx_set_heff_budget")

    def tune(self, A, B, slices: int, ndiag: int = 0, C=None, transa="N", transb="N",
             workspace=None, stream=None):
        """Time every tile variant on this GEMM and keep the fastest; returns
        (variant, {variant: ms})."""
        import numpy as np
        _dev_f64(A, "A")
        _dev_f64(B, "B")
        M, N, K = self._dims(A, B, transa, transb)
        if C is None:
            C = torch.empty((M, N), dtype=torch.float64, device=A.device)
        _dev_out(C, M, N, "C")
        if workspace is None:
            workspace = self.workspace(M, N, K, slices, ndiag)
        ms = np.full(16, -1.0, dtype=np.float64)
        v = _check(_lib.ozaki_dgemm_tune(self.handle, transa.upper().encode(), transb.upper().encode(),
                                         M, N, K, A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"),
                                         C.data_ptr(), _ld(C, "C"), slices, ndiag,
                                         workspace.data_ptr(),
                                         workspace.numel() * workspace.element_size(),
                                         _stream(stream), ms.ctypes.data), "ozaki_dgemm_tune")
        return v, {i: float(t) for i, t in enumerate(ms) if t >= 0}

    # ---- GEMM -----------------------------------------------------------
    def workspace(self, M, N, K, slices, ndiag=0) -> torch.Tensor | None:
        n = workspace_bytes(M, N, K, slices, ndiag)
        if n == 0:
            return None
        return torch.empty(n, dtype=torch.uint8, device="cuda:%d" % self.device)

    def dgemm(self, A, B, slices: int = 6, ndiag: int = 0, alpha: float = 1.0, beta: float = 0.0,
              C=None, transa: str = "N", transb: str = "N", workspace=None, stream=None):
        """C = alpha op(A) op(B) + beta C; slices = 0 runs the native FP64 MFMA GEMM."""
        _dev_f64(A, "A")
        _dev_f64(B, "B")
        ta, tb = transa.upper() == "T", transb.upper() == "T"
        M = A.size(1) if ta else A.size(0)
        K = A.size(0) if ta else A.size(1)
        N = B.size(0) if tb else B.size(1)
        if (B.size(1) if tb else B.size(0)) != K:
            raise ValueError("inner dimensions differ")
        if C is None:
            C = torch.empty((M, N), dtype=torch.float64, device=A.device)
            if beta != 0.0:
                raise ValueError("beta != 0 needs C")
        _dev_out(C, M, N, "C")
        if workspace is None:
            workspace = self.workspace(M, N, K, slices, ndiag)
        wptr = workspace.data_ptr() if workspace is not None else None
        wlen = workspace.numel() * workspace.element_size() if workspace is not None else 0
        _check(_lib.ozaki_dgemm(self.handle, transa.upper().encode(), transb.upper().encode(), M, N,
                                K, alpha, A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"),
                                beta, C.data_ptr(), _ld(C, "C"), slices, ndiag, wptr, wlen,
                                _stream(stream)), "ozaki_dgemm")
        return C

    def dgemm_static(self, A, B, C, slices: int = 6, ndiag: int = 0, alpha: float = 1.0, beta: float = 0.0,
                     transa: str = "N", transb: str = "N", stream=None):
        """ozaki_dgemm_static: as dgemm, with the library's static per-GPU
        workspace; C (the output) is passed in, nothing is allocated."""
        _dev_f64(A, "A")
        _dev_f64(B, "B")
        _dev_f64(C, "C")
        ta, tb = transa.upper() == "T", transb.upper() == "T"
        M = A.size(1) if ta else A.size(0)
        K = A.size(0) if ta else A.size(1)
        N = B.size(0) if tb else B.size(1)
        if (B.size(1) if tb else B.size(0)) != K or tuple(C.shape) != (M, N):
            raise ValueError("operand shapes do not match")
        _check(_lib.ozaki_dgemm_static(self.handle, transa.upper().encode(), transb.upper().encode(), M, N,
                                       K, alpha, A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"),
                                       beta, C.data_ptr(), _ld(C, "C"), slices, ndiag, _stream(stream)),
               "ozaki_dgemm_static")
        return C

    def renormalize(self, U, ops, slices: int = 6, ndiag: int = 0, outs=None, workspace=None, stream=None):
        """O'_k = U^T O_k U for every O_k in ops (two GEMMs each, emulated or
        native FP64 by ``slices``); returns the list of D x D results."""
        _dev_f64(U, "U")
        n, D = U.shape
        ops = list(ops)
        for o in ops:
            _dev_f64(o, "ops[k]")
            if tuple(o.shape) != (n, n):
                raise ValueError("every operator must be %d x %d" % (n, n))
        if outs is None:
            outs = [torch.empty((D, D), dtype=torch.float64, device=U.device) for _ in ops]
        outs = list(outs)
        if len(outs) != len(ops):
            raise ValueError("one output per operator: %d outputs for %d operators" % (len(outs), len(ops)))
        for o in outs:
            _dev_out(o, D, D, "outs[k]")
        ldo = _ld(ops[0], "ops[0]") if ops else max(n, 1)
        ldout = _ld(outs[0], "outs[0]") if outs else max(D, 1)
        if any(_ld(o, "ops[k]") != ldo for o in ops) or any(_ld(o, "outs[k]") != ldout for o in outs):
            raise ValueError("all operators (and all outputs) must share one leading dimension")
        if workspace is None:
            nb = _lib.ozaki_renormalize_workspace_bytes(n, D, slices, ndiag)
            workspace = torch.empty(max(nb, 1), dtype=torch.uint8, device=U.device)
        po = (_ptr * max(len(ops), 1))(*[o.data_ptr() for o in ops])
        pr = (_ptr * max(len(outs), 1))(*[o.data_ptr() for o in outs])
        _check(_lib.ozaki_renormalize(self.handle, n, D, U.data_ptr(), _ld(U, "U"), len(ops), po, ldo, pr,
                                      ldout, slices, ndiag, workspace.data_ptr(),
                                      workspace.numel() * workspace.element_size(), _stream(stream)),
               "ozaki_renormalize")
        return outs

    # ---- emulation modes --------------------------------------------------
    def auto_workspace(self, M, N, K) -> torch.Tensor | None:
        n = int(_lib.ozaki_dgemm_auto_workspace_bytes(M, N, K))
        if n == 0:
            return None
        return torch.empty(n, dtype=torch.uint8, device="cuda:%d" % self.device)

    @staticmethod
    def _dims(A, B, transa, transb):
        ta, tb = transa.upper() == "T", transb.upper() == "T"
        M = A.size(1) if ta else A.size(0)
        K = A.size(0) if ta else A.size(1)
        N = B.size(0) if tb else B.size(1)
        if (B.size(1) if tb else B.size(0)) != K:
            raise ValueError("inner dimensions differ")
        return M, N, K

    def choose_slices(self, A, B, transa: str = "N", transb: str = "N", workspace=None, stream=None):
        """(slices, ndiag, {rho_a, rho_b, predicted, native}) of the automatic choice."""
        import numpy as np
        _dev_f64(A, "A")
        _dev_f64(B, "B")
        M, N, K = self._dims(A, B, transa, transb)
        if workspace is None:
            workspace = self.auto_workspace(M, N, K)
        s_out, g_out = ctypes.c_int32(), ctypes.c_int32()
        st = np.zeros(4, dtype=np.float64)
        _check(_lib.ozaki_choose_slices(self.handle, transa.upper().encode(), transb.upper().encode(), M, N, K,
                                        A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"),
                                        workspace.data_ptr() if workspace is not None else None,
                                        workspace.numel() if workspace is not None else 0, _stream(stream),
                                        ctypes.byref(s_out), ctypes.byref(g_out), st.ctypes.data),
               "ozaki_choose_slices")
        return s_out.value, g_out.value, {"rho_a": float(st[0]), "rho_b": float(st[1]),
                                          "predicted": float(st[2]), "native": float(st[3])}

    def dgemm_auto(self, A, B, bits: int = 0, performant: bool = False, alpha: float = 1.0,
                   beta: float = 0.0, C=None, transa: str = "N", transb: str = "N", workspace=None,
                   stream=None):
        """C = alpha op(A) op(B) + beta C with the width (bits; 0 = automatic) and the path
        (performant: timed per shape) chosen by the library; returns (C, slices, ndiag)
        of the path taken (0, 0 = native FP64)."""
        _dev_f64(A, "A")
        _dev_f64(B, "B")
        M, N, K = self._dims(A, B, transa, transb)
        if C is None:
            if beta != 0.0:
                raise ValueError("beta != 0 needs C")
            C = torch.empty((M, N), dtype=torch.float64, device=A.device)
        _dev_out(C, M, N, "C")
        if workspace is None:
            workspace = self.auto_workspace(M, N, K)
        s_out, g_out = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.ozaki_dgemm_auto(self.handle, transa.upper().encode(), transb.upper().encode(), M, N, K,
                                     alpha, A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"), beta,
                                     C.data_ptr(), _ld(C, "C"), int(bits), int(performant),
                                     workspace.data_ptr() if workspace is not None else None,
                                     workspace.numel() if workspace is not None else 0, _stream(stream),
                                     ctypes.byref(s_out), ctypes.byref(g_out)), "ozaki_dgemm_auto")
        return C, s_out.value, g_out.value

    # ---- steps on their own (tests) --------------------------------------
    def split(self, X, slices: int, by_columns: bool = False, stream=None):
        """(digits int8 [S][groups][len], exps int32 [groups]) of X's slices."""
        _dev_f64(X, "X")
        rows, cols = X.shape
        groups, length = (cols, rows) if by_columns else (rows, cols)
        digits = torch.empty((slices, groups, length), dtype=torch.int8, device=X.device)
        exps = torch.empty(groups, dtype=torch.int32, device=X.device)
        _check(_lib.ozaki_split(self.handle, int(by_columns), rows, cols, X.data_ptr(), _ld(X, "X"),
                                slices, digits.data_ptr(), exps.data_ptr(), _stream(stream)),
               "ozaki_split")
        return digits, exps

    def pair_products(self, Adig, BTdig, slices: int, ndiag: int = 0, stream=None):
        """int32 Q[g][i][j] = sum over kept pairs on diagonal g of Adig[s] BTdig[t]^T."""
        S, M, K = Adig.shape
        _, N, _ = BTdig.shape
        G = slices if ndiag == 0 else ndiag
        Q = torch.empty((G, M, N), dtype=torch.int32, device=Adig.device)
        Adig = Adig.contiguous()
        BTdig = BTdig.contiguous()
        _check(_lib.ozaki_pair_products(self.handle, M, N, K, slices, ndiag, Adig.data_ptr(),
                                        BTdig.data_ptr(), Q.data_ptr(), _stream(stream)),
               "ozaki_pair_products")
        return Q


# ---- effective Hamiltonian ----------------------------------------------------
class HeffPlan:
    """A planned H_eff.psi (dense or block-sparse); see heff_plan_create in ozaki.h.

    The layout arrays are host data; L_data, R_data (and diag) are flat float64
    CUDA tensors that must outlive the plan.
    """

    def __init__(self, ctx: Context, layout: dict, L_data, R_data, triples, diag=None,
                 slices: int = 6, ndiag: int = 0, stream=None):
        import numpy as np
        self.ctx = ctx
        self._keep = [L_data, R_data, diag]
        arr = {}

        def a32(x):
            v = np.ascontiguousarray(np.asarray(x, dtype=np.int32))
            arr[id(v)] = v
            return v.ctypes.data

        def a64(x):
            v = np.ascontiguousarray(np.asarray(x, dtype=np.int64))
            arr[id(v)] = v
            return v.ctypes.data

        lay = HeffLayout(
            n_left=len(layout["left_dim"]), n_right=len(layout["right_dim"]), phys=layout["phys"],
            left_dim=a32(layout["left_dim"]), right_dim=a32(layout["right_dim"]),
            n_psi_blocks=len(layout["psi_offset"]), psi_lr=a32(layout["psi_lr"]),
            psi_offset=a64(layout["psi_offset"]),
            n_L_blocks=len(layout["L_offset"]), L_key=a32(layout["L_key"]),
            L_offset=a64(layout["L_offset"]),
            n_R_blocks=len(layout["R_offset"]), R_key=a32(layout["R_key"]),
            R_offset=a64(layout["R_offset"]))
        tri = (HeffTriple * max(1, len(triples)))()
        for n, (op, lo, li, ri, ro, al) in enumerate(triples):
            tri[n] = HeffTriple(op, lo, li, ri, ro, al)
        h = _ptr()
        _check(_lib.heff_plan_create(ctx.handle, ctypes.byref(h), ctypes.byref(lay),
                                     _dev_f64(L_data, "L").data_ptr(),
                                     _dev_f64(R_data, "R").data_ptr(), len(triples), tri,
                                     diag.data_ptr() if diag is not None else None, slices, ndiag,
                                     _stream(stream)), "heff_plan_create")
        self.handle = h
        self.n = int(_lib.heff_vector_length(h))
        if diag is not None:
            try:
                _dev_vec(diag, self.n, "diag")
            except (TypeError, ValueError):
                self.close()
                raise
        self.flops = float(_lib.heff_flops(h))
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.heff_plan_variants(h, ctypes.byref(a), ctypes.byref(b)), "heff_plan_variants")
        self.variants = (a.value, b.value)
        _check(_lib.heff_plan_launches(h, ctypes.byref(a), ctypes.byref(b)), "heff_plan_launches")
        self.launches = (a.value, b.value)

    def apply(self, psi, sigma=None, stream=None):
        _dev_vec(psi, self.n, "psi")
        if sigma is None:
            sigma = torch.empty_like(psi)
        else:
            _dev_vec(sigma, self.n, "sigma")
        _check(_lib.heff_apply(self.handle, psi.data_ptr(), sigma.data_ptr(), _stream(stream)),
               "heff_apply")
        return sigma

    def set_graphs(self, enable: bool = True):
        """Replay captured HIP graphs in apply (default) or issue the launches directly."""
        _check(_lib.heff_plan_set_graphs(self.handle, int(bool(enable))), "heff_plan_set_graphs")

    @property
    def graph_count(self) -> int:
        return _check(_lib.heff_plan_graph_count(self.handle), "heff_plan_graph_count")

    def phase(self, phase: int):
        """(variant, order, launch) of grouped phase `phase` (0 or 1)."""
        v, o, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.heff_plan_phase(self.handle, int(phase), ctypes.byref(v), ctypes.byref(o), ctypes.byref(l)),
               "heff_plan_phase")
        return v.value, o.value, l.value

    @property
    def chunks(self) -> int:
        return _check(_lib.heff_plan_chunks(self.handle), "heff_plan_chunks")

    @property
    def bytes(self):
        """(device bytes of the plan, of which the intermediates T)."""
        t = ctypes.c_int64(0)
        total = _check(_lib.heff_plan_bytes(self.handle, ctypes.byref(t)), "heff_plan_bytes")
        return total, t.value

    def close(self):
        if getattr(self, "handle", None):
            _lib.heff_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Davidson:
    """Device-resident Davidson iteration for the lowest eigenpair of a HeffPlan."""

    def __init__(self, ctx: Context, plan: HeffPlan, hdiag, x0, m_max: int = 32,
                 tol: float = 1e-8, max_iter: int = 300, stream=None):
        self.ctx = ctx
        self.plan = plan
        h = _ptr()
        _check(_lib.davidson_create(ctx.handle, ctypes.byref(h), plan.handle,
                                    _dev_vec(hdiag, plan.n, "hdiag").data_ptr(),
                                    _dev_vec(x0, plan.n, "x0").data_ptr(), m_max, tol, max_iter,
                                    _stream(stream)), "davidson_create")
        self.handle = h

    def step(self, stream=None) -> DavidsonInfo:
        info = DavidsonInfo()
        _check(_lib.davidson_step(self.handle, ctypes.byref(info), _stream(stream)), "davidson_step")
        return info

    def vector(self, out=None, stream=None):
        if out is None:
            out = torch.empty(self.plan.n, dtype=torch.float64, device="cuda:%d" % self.ctx.device)
        _dev_vec(out, self.plan.n, "out")
        _check(_lib.davidson_get_vector(self.handle, out.data_ptr(), _stream(stream)),
               "davidson_get_vector")
        return out

    def set_graphs(self, enable: bool):
        _check(_lib.davidson_set_graphs(self.handle, 1 if enable else 0), "davidson_set_graphs")

    @property
    def graph_count(self) -> int:
        return _check(_lib.davidson_graph_count(self.handle), "davidson_graph_count")

    def run(self, stream=None):
        """Iterate until a terminal status; returns (theta, status, iterations, residual)."""
        while True:
            info = self.step(stream)
            if info.status != OZ_OK:
                return info.theta, STATUS[info.status], info.iter, info.resnorm

    def close(self):
        if getattr(self, "handle", None):
            _lib.davidson_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Lanczos:
    """Device-resident Lanczos iteration (full reorthogonalisation, explicit
    restart) for the lowest eigenpair of a HeffPlan; same step interface as
    Davidson."""

    def __init__(self, ctx: Context, plan: HeffPlan, x0, m_max: int = 32, tol: float = 1e-8,
                 max_iter: int = 300, stream=None):
        self.ctx = ctx
        self.plan = plan
        h = _ptr()
        _check(_lib.lanczos_create(ctx.handle, ctypes.byref(h), plan.handle, _dev_vec(x0, plan.n, "x0").data_ptr(),
                                   m_max, tol, max_iter, _stream(stream)), "lanczos_create")
        self.handle = h

    def step(self, stream=None) -> DavidsonInfo:
        info = DavidsonInfo()
        _check(_lib.lanczos_step(self.handle, ctypes.byref(info), _stream(stream)), "lanczos_step")
        return info

    def vector(self, out=None, stream=None):
        if out is None:
            out = torch.empty(self.plan.n, dtype=torch.float64, device="cuda:%d" % self.ctx.device)
        _dev_vec(out, self.plan.n, "out")
        _check(_lib.lanczos_get_vector(self.handle, out.data_ptr(), _stream(stream)), "lanczos_get_vector")
        return out

    def run(self, stream=None):
        """Iterate until a terminal status; returns (theta, status, iterations, residual)."""
        while True:
            info = self.step(stream)
            if info.status != OZ_OK:
                return info.theta, STATUS[info.status], info.iter, info.resnorm

    def close(self):
        if getattr(self, "handle", None):
            _lib.lanczos_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RdmEig:
    """Eigenpairs of a symmetric positive semidefinite matrix (a reduced
    density matrix) by two-sided block Jacobi on the device; the GEMMs run
    emulated (slices >= 2) or in native FP64 (slices = 0)."""

    def __init__(self, ctx: Context, n: int, slices: int = 0, ndiag: int = 0):
        self.ctx = ctx
        self.n = n
        h = _ptr()
        _check(_lib.rdm_eig_create(ctx.handle, ctypes.byref(h), n, slices, ndiag), "rdm_eig_create")
        self.handle = h

    def solve(self, A, nev: int | None = None, tol: float = 0.0, max_sweeps: int = 30, stream=None):
        """Returns (evals [nev], Z [n, nev] with the eigenvectors as columns, info)."""
        _dev_f64(A, "A")
        if tuple(A.shape) != (self.n, self.n):
            raise ValueError("A must be %d x %d" % (self.n, self.n))
        nev = self.n if nev is None else nev
        evals = torch.empty(max(nev, 1), dtype=torch.float64, device=A.device)[:nev]
        Z = torch.empty((self.n, max(nev, 1)), dtype=torch.float64, device=A.device)
        info = RdmEigInfo()
        _check(_lib.rdm_eig_solve(self.handle, A.data_ptr(), _ld(A, "A"), nev, evals.data_ptr(), Z.data_ptr(),
                                  Z.stride(0), tol, max_sweeps, ctypes.byref(info), _stream(stream)),
               "rdm_eig_solve")
        return evals, Z[:, :nev], info

    def close(self):
        if getattr(self, "handle", None):
            _lib.rdm_eig_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def truncate(ctx: Context, psi, D: int, slices: int = 0, ndiag: int = 0, eig: RdmEig | None = None,
             max_sweeps: int = 30):
    """DMRG truncation of a two-site tensor psi (m x k, row-major): rho =
    psi psi^T by ozaki_dgemm, its D dominant eigenpairs by RdmEig, both in
    the arithmetic (slices, ndiag).  Returns (U [m, D], kept eigenvalues,
    discarded weight = trace(rho) - sum of the kept ones, info)."""
    _dev_f64(psi, "psi")
    m = psi.size(0)
    rho = ctx.dgemm(psi, psi, slices=slices, ndiag=ndiag, transb="T")
    own = eig is None
    if own:
        eig = RdmEig(ctx, m, slices, ndiag)
    try:
        evals, U, info = eig.solve(rho, D, max_sweeps=max_sweeps)
    finally:
        if own:
            eig.close()
    return U, evals, info.trace - sum(evals.tolist()), info
