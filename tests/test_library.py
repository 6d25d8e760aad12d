"""The C-ABI library loads, exports every declared entry point and its host
logic (parameter rules, workspace sizes, argument checks) behaves without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ozaki.h")
LIB = os.path.join(ROOT, "paper_2510_04795_amd", "libozaki.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("ozaki_", "heff_", "davidson_", "lanczos_", "rdm_"))))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libozaki.so is not built (python -m paper_2510_04795_amd._build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("ozaki_dgemm", "heff_plan_create", "heff_apply", "davidson_step",
                 "ozaki_split", "ozaki_pair_products"):
        assert must in names
    assert len(names) >= 20


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2510_04795_amd import ozaki
    assert sorted(ozaki.EXPORTED) == declared_functions()


def test_parameter_rules(lib):
    lib.ozaki_slices_for_bits.restype = ctypes.c_int
    for bits, S in [(15, 2), (23, 3), (31, 4), (39, 5), (47, 6), (55, 7), (63, 8)]:
        assert lib.ozaki_slices_for_bits(bits) == S
    assert lib.ozaki_slices_for_bits(0) < 0
    assert lib.ozaki_pair_count(7, 13) == 49
    assert lib.ozaki_pair_count(6, 0) == 21 and lib.ozaki_pair_count(6, 7) == 26
    lib.ozaki_max_exact_k.restype = ctypes.c_int64
    # every int8 x int8 product is at most 2^14; S pairs share the widest diagonal
    for S in range(2, 9):
        k = lib.ozaki_max_exact_k(S, 0)
        assert k * S * 2 ** 14 <= 2 ** 31 - 1 < (k + 1) * S * 2 ** 14


def test_workspace_sizes(lib):
    lib.ozaki_dgemm_workspace_bytes.restype = ctypes.c_size_t
    lib.ozaki_dgemm_workspace_bytes.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_int] * 2
    assert lib.ozaki_dgemm_workspace_bytes(100, 100, 100, 0, 0) == 0
    w = lib.ozaki_dgemm_workspace_bytes(8192, 8192, 8192, 6, 0)
    assert w >= 2 * 6 * 8192 * 8192          # int8 slices of both operands
    assert w < 2 * 6 * 8192 * 8192 + 64 << 20
    big = lib.ozaki_dgemm_workspace_bytes(64, 64, 40000, 8, 0)
    assert big >= 8 * 8 * 64 * 64            # int64 carries of the chunked inner dimension


def test_errors_without_device(lib):
    from paper_2510_04795_amd import ozaki
    rc = ozaki._lib.ozaki_dgemm(None, b"N", b"N", 4, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4,
                                6, 0, None, 0, None)
    assert rc == -1 and b"ctx" in ozaki._lib.ozaki_last_error()
    assert ozaki._lib.ozaki_status_string(-2) == b"workspace missing or too small"
    import torch
    if not torch.cuda.is_available():
        h = ctypes.c_void_p()
        assert ozaki._lib.ozaki_ctx_create(ctypes.byref(h), 0) == -3


def test_new_entry_points_reject_bad_arguments_on_the_host():
    """The Lanczos, RDM eigensolver and renormalisation entry points check
    their handles and sizes before touching a device."""
    from paper_2510_04795_amd import ozaki
    L = ozaki._lib
    h = ctypes.c_void_p()
    assert L.lanczos_create(None, ctypes.byref(h), None, None, 32, 1e-8, 300, None) == -1
    assert L.lanczos_step(None, None, None) == -1
    assert L.lanczos_get_vector(None, None, None) == -1
    assert L.lanczos_destroy(None) == 0
    assert L.rdm_eig_create(None, ctypes.byref(h), 16, 0, 0) == -1
    assert b"ctx" in L.ozaki_last_error()
    assert L.rdm_eig_solve(None, None, 16, 4, None, None, 4, 0.0, 10, None, None) == -1
    assert L.rdm_eig_destroy(None) == 0
    assert L.ozaki_ctx_set_heff_launch(None, 0) == -1
    assert L.heff_plan_launches(None, None, None) == -1
    assert L.ozaki_renormalize(None, 100, 20, None, 20, 1, None, 100, None, 20, 0, 0, None, 0, None) == -1
    # workspace: the intermediate T (n x D doubles, 256-byte aligned), plus the GEMM workspace when emulated
    t = (100 * 20 * 8 + 255) // 256 * 256
    assert L.ozaki_renormalize_workspace_bytes(100, 20, 0, 0) == t
    w6 = L.ozaki_renormalize_workspace_bytes(100, 20, 6, 0)
    assert w6 == t + max(L.ozaki_dgemm_workspace_bytes(100, 20, 100, 6, 0),
                         L.ozaki_dgemm_workspace_bytes(20, 20, 100, 6, 0))
