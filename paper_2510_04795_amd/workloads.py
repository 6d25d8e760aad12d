"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and arranges them; it contains none of
the emulated-FP64 arithmetic.  Both the GPU path and the CPU oracle are fed
from here, so the two never share any code that computes the method itself.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and draws its
objects in a fixed order, so a (config, seed) pair always produces the same
bytes.  The element distribution N(0,1)*2^u with u an integer drawn uniformly
from [-U, U] mimics the wide dynamic range of DMRG operator blocks.

Workloads (the paper's molecular integrals are not available; these stand in
for them with the same shapes):

* ``gemm_pair``      - square GEMM operands (512^3 plain FP64 GEMM, and the
  2048/4096/8192 emulated-GEMM sweep with U = 10 or 30).
* ``heff_dense``     - dense two-site problem: Kop symmetric D x D operator
  pairs (L_k, R_k) and a two-site tensor psi of shape (D, d^2 = 16, D), the
  local dimension d = 4 of a spatial orbital (Theory of TNS/DMRG, Eq. mps).
* ``heff_sparse``    - symmetry-sector block-sparse problem: 40 sectors with
  log-normal sizes, a random psi sparsity pattern and ~2000 (L, psi, R)
  triples, standing in for SU(2)/U(1) multiplet blocks.
* ``davidson_problem`` - a symmetric H_eff = sum_k L_k (x) R_k + diagonal
  shift scaled to a spectral norm of about 10 Ha, with its diagonal and a
  start vector, for the Krylov eigensolver step.
* ``two_site_psi``   - a two-site tensor reshaped to a matrix (D d) x (d D)
  with a planted Schmidt spectrum (exponentially decaying, unit norm), for
  the reduced-density-matrix truncation step.
* ``block_operators`` - symmetric block operators of the enlarged block for
  the renormalisation step.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "wide_normal", "symmetrize", "gemm_pair", "heff_dense", "heff_sparse",
    "HeffSparse", "davidson_problem", "DavidsonProblem",
]


def wide_normal(rng: np.random.Generator, shape, U: int) -> np.ndarray:
    """N(0,1) * 2^u with u uniform over the integers in [-U, U], per element.

    The normals are drawn before the exponents.
    """
    x = rng.standard_normal(shape)
    u = rng.integers(-U, U, size=shape, endpoint=True)
    return np.ldexp(x, u)


def symmetrize(x: np.ndarray) -> np.ndarray:
    """Mirror the upper triangle of the trailing two axes onto the lower one."""
    up = np.triu(x)
    return up + np.swapaxes(np.triu(x, 1), -1, -2)


def gemm_pair(n: int, U: int = 10, seed: int = 0, m: int | None = None,
              k: int | None = None):
    """A (m x k) then B (k x n), both wide_normal(U) from one rng."""
    m = n if m is None else m
    k = n if k is None else k
    rng = np.random.default_rng(seed)
    A = wide_normal(rng, (m, k), U)
    B = wide_normal(rng, (k, n), U)
    return A, B


def heff_dense(D: int, kop: int = 64, phys: int = 16, U: int = 8, seed: int = 0):
    """Operators L[k], R[k] (symmetric D x D) for k < kop, then psi (D, phys, D).

    Drawn in the order L_0, R_0, L_1, R_1, ..., psi.
    """
    rng = np.random.default_rng(seed)
    L = np.empty((kop, D, D))
    R = np.empty((kop, D, D))
    for k in range(kop):
        L[k] = symmetrize(wide_normal(rng, (D, D), U))
        R[k] = symmetrize(wide_normal(rng, (D, D), U))
    psi = wide_normal(rng, (D, phys, D), U)
    return L, R, psi


@dataclasses.dataclass
class HeffSparse:
    """Block-sparse two-site problem with phys = 1 (blocks of sector pairs).

    dims[q]           sector size (shared by the left and right bond)
    psi_blocks        sorted list of (l, r) sector pairs present in psi/sigma
    psi[(l, r)]       dims[l] x dims[r] block
    L[(op, lo, li)]   dims[lo] x dims[li] block of left operator op
    R[(op, ro, ri)]   dims[ro] x dims[ri] block of right operator op
    triples           list of (op, lo, li, ri, ro, alpha):
                      sigma[lo, ro] += alpha * L[op][lo, li] psi[li, ri] R[op][ro, ri]^T
    """
    dims: np.ndarray
    psi_blocks: list
    psi: dict
    L: dict
    R: dict
    triples: list

    def flops(self) -> int:
        d = self.dims
        return int(sum(2 * (d[lo] * d[li] * d[ri] + d[lo] * d[ri] * d[ro])
                       for (_, lo, li, ri, ro, _) in self.triples))


def heff_sparse(n_sectors: int = 40, n_triples: int = 2000, kop: int = 64,
                median: float = 200.0, sigma_log: float = 0.8, lo_hi=(16, 1500),
                density: float = 0.12, reach: int = 2, U: int = 12,
                seed: int = 0) -> HeffSparse:
    """Sector sizes, psi mask, distinct triples, then psi, L and R blocks.

    Sector sizes: clip(rint(exp(ln(median) + sigma_log * N(0,1))), lo, hi).
    psi mask: uniform(0,1) < density over sector pairs (sigma uses the same
    pattern).  Triples: op uniform in [0, kop); the source (li, ri) uniform
    over mask blocks; the target (lo, ro) uniform over mask blocks with
    |lo - li| <= reach and |ro - ri| <= reach; alpha = 1.  Draws continue
    until n_triples distinct triples exist (or the candidate set is used up).
    Blocks are then drawn as wide_normal(U) in sorted key order: psi blocks,
    L blocks, R blocks.
    """
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(n_sectors)
    dims = np.clip(np.rint(np.exp(math.log(median) + sigma_log * z)), lo_hi[0],
                   lo_hi[1]).astype(np.int64)
    mask = rng.random((n_sectors, n_sectors)) < density
    blocks = [tuple(map(int, b)) for b in np.argwhere(mask)]
    blocks.sort()
    near = {}
    for (li, ri) in blocks:
        near[(li, ri)] = [(lo, ro) for (lo, ro) in blocks
                          if abs(lo - li) <= reach and abs(ro - ri) <= reach]
    capacity = kop * sum(len(v) for v in near.values())
    target = min(n_triples, capacity)
    seen = set()
    triples = []
    while len(triples) < target:
        op = int(rng.integers(0, kop))
        li, ri = blocks[int(rng.integers(0, len(blocks)))]
        cand = near[(li, ri)]
        lo, ro = cand[int(rng.integers(0, len(cand)))]
        key = (op, lo, li, ri, ro)
        if key in seen:
            continue
        seen.add(key)
        triples.append((op, lo, li, ri, ro, 1.0))
    psi = {}
    for (l, r) in blocks:
        psi[(l, r)] = wide_normal(rng, (int(dims[l]), int(dims[r])), U)
    Lkeys = sorted({(op, lo, li) for (op, lo, li, ri, ro, _) in triples})
    Rkeys = sorted({(op, ro, ri) for (op, lo, li, ri, ro, _) in triples})
    L = {key: wide_normal(rng, (int(dims[key[1]]), int(dims[key[2]])), U) for key in Lkeys}
    R = {key: wide_normal(rng, (int(dims[key[1]]), int(dims[key[2]])), U) for key in Rkeys}
    return HeffSparse(dims=dims, psi_blocks=blocks, psi=psi, L=L, R=R, triples=triples)


@dataclasses.dataclass
class DavidsonProblem:
    """H = sum_k L[k] (x) R[k] + diag(delta) acting on psi (D x D), n = D^2.

    hdiag is the diagonal of H (an input of the diagonal preconditioner) and
    x0 the normalised start vector, both laid out like psi (row-major D x D).
    """
    L: np.ndarray
    R: np.ndarray
    delta: np.ndarray
    hdiag: np.ndarray
    x0: np.ndarray
    scale: float


def _heff_apply_fp64(L, R, X):
    # plain FP64 sum_k L_k X R_k^T, used only to estimate the norm for scaling
    out = np.zeros_like(X)
    for k in range(L.shape[0]):
        out += L[k] @ X @ R[k].T
    return out


def davidson_problem(D: int, kop: int = 32, norm: float = 10.0, well: float = -30.0,
                     power_iters: int = 60, seed: int = 0) -> DavidsonProblem:
    """Random symmetric operator pairs scaled to a total spectral norm ~ ``norm``.

    L_k, R_k = sym(N(0,1)^{D x D}) / (2 sqrt(D)) (GOE-like, norm ~ 1 each);
    nu = ||sum_k L_k (x) R_k||_2 by ``power_iters`` FP64 power iterations from
    a seed-0 start; every L_k and R_k is multiplied by sqrt(norm / nu).  The
    shift is delta[0, 0] = ``well`` (a planted reference state, like a
    Hartree-Fock determinant) and zero elsewhere.  The start vector is
    e_{argmin hdiag} + 0.1 * rhat with rhat a normalised N(0,1) vector drawn
    from seed 1, then normalised.
    """
    rng = np.random.default_rng(seed)
    c = 1.0 / (2.0 * math.sqrt(D))
    L = np.empty((kop, D, D))
    R = np.empty((kop, D, D))
    for k in range(kop):
        L[k] = symmetrize(rng.standard_normal((D, D))) * c
        R[k] = symmetrize(rng.standard_normal((D, D))) * c
    v = np.random.default_rng(0).standard_normal((D, D))
    v /= np.linalg.norm(v)
    nu = 1.0
    for _ in range(power_iters):
        w = _heff_apply_fp64(L, R, v)
        nu = float(np.linalg.norm(w))
        v = w / nu
    s = math.sqrt(norm / nu)
    L *= s
    R *= s
    delta = np.zeros((D, D))
    delta[0, 0] = well
    dL = np.einsum("kii->ki", L)
    dR = np.einsum("kii->ki", R)
    hdiag = np.einsum("ki,kj->ij", dL, dR) + delta
    r = np.random.default_rng(1).standard_normal(D * D)
    r /= np.linalg.norm(r)
    x0 = 0.1 * r
    x0[int(np.argmin(hdiag))] += 1.0
    x0 /= np.linalg.norm(x0)
    return DavidsonProblem(L=L, R=R, delta=delta, hdiag=hdiag,
                           x0=x0.reshape(D, D), scale=s)


# ----------------------------------------------------------------------------
# Flat layouts for the library's H_eff plan (data arrangement only)
# ----------------------------------------------------------------------------
def flatten_dense(L: np.ndarray, R: np.ndarray, psi: np.ndarray):
    """Layout dict, flat L, flat R, flat psi and triples of a dense two-site
    problem: one left and one right sector of size D, phys = psi.shape[1],
    triples (k, 0, 0, 0, 0, 1) for every operator pair k."""
    kop, D, _ = L.shape
    p = psi.shape[1]
    layout = {"left_dim": [D], "right_dim": [psi.shape[2]], "phys": p,
              "psi_lr": [0, 0], "psi_offset": [0],
              "L_key": [x for k in range(kop) for x in (k, 0, 0)],
              "L_offset": [k * D * D for k in range(kop)],
              "R_key": [x for k in range(kop) for x in (k, 0, 0)],
              "R_offset": [k * R.shape[1] * R.shape[2] for k in range(kop)]}
    triples = [(k, 0, 0, 0, 0, 1.0) for k in range(kop)]
    return layout, np.ascontiguousarray(L).ravel(), np.ascontiguousarray(R).ravel(), \
        np.ascontiguousarray(psi).ravel(), triples


def flatten_sparse(prob: "HeffSparse"):
    """Layout dict, flat L, flat R, flat psi and triples of a block-sparse
    problem (phys = 1); blocks are stored in sorted key order."""
    dims = [int(d) for d in prob.dims]
    psi_off, off = [], 0
    for (l, r) in prob.psi_blocks:
        psi_off.append(off)
        off += dims[l] * dims[r]
    psi_flat = np.concatenate([prob.psi[b].ravel() for b in prob.psi_blocks]) if prob.psi_blocks else np.zeros(0)
    Lk = sorted(prob.L)
    Rk = sorted(prob.R)
    L_off, o = [], 0
    for k in Lk:
        L_off.append(o)
        o += prob.L[k].size
    R_off, o = [], 0
    for k in Rk:
        R_off.append(o)
        o += prob.R[k].size
    layout = {"left_dim": dims, "right_dim": dims, "phys": 1,
              "psi_lr": [x for b in prob.psi_blocks for x in b], "psi_offset": psi_off,
              "L_key": [x for k in Lk for x in k], "L_offset": L_off,
              "R_key": [x for k in Rk for x in k], "R_offset": R_off}
    L_flat = np.concatenate([prob.L[k].ravel() for k in Lk]) if Lk else np.zeros(0)
    R_flat = np.concatenate([prob.R[k].ravel() for k in Rk]) if Rk else np.zeros(0)
    return layout, L_flat, R_flat, psi_flat, list(prob.triples)


def unflatten_sparse(prob: "HeffSparse", flat: np.ndarray) -> dict:
    """Blocks of a flat sigma laid out like flatten_sparse's psi."""
    out, off = {}, 0
    for (l, r) in prob.psi_blocks:
        n = int(prob.dims[l]) * int(prob.dims[r])
        out[(l, r)] = flat[off:off + n].reshape(int(prob.dims[l]), int(prob.dims[r]))
        off += n
    return out


@dataclasses.dataclass
class TwoSitePsi:
    psi: np.ndarray       # m x k, row-major
    schmidt: np.ndarray   # planted Schmidt values, decreasing, sum of squares 1
    left: np.ndarray      # m x r orthonormal left Schmidt vectors (columns)


def _orthonormal_columns(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    q, r = np.linalg.qr(rng.standard_normal((rows, cols)))
    return q * np.sign(np.diag(r))


def two_site_psi(m: int, k: int | None = None, tau: float | None = None, seed: int = 0) -> TwoSitePsi:
    """psi = X diag(s) Y^T with X (m x r), Y (k x r) Haar-like orthonormal
    columns (QR of N(0,1) matrices, drawn in that order) and r = min(m, k);
    s_i^2 proportional to exp(-i / tau) (default tau = m / 64, so the weight
    beyond the leading quarter of the spectrum is about e^-16), normalised to
    unit Frobenius norm.  The eigenvalues of rho = psi psi^T are s_i^2."""
    k = m if k is None else k
    r = min(m, k)
    tau = m / 64.0 if tau is None else tau
    rng = np.random.default_rng(seed)
    X = _orthonormal_columns(rng, m, r)
    Y = _orthonormal_columns(rng, k, r)
    w = np.exp(-np.arange(r) / tau)
    s = np.sqrt(w / w.sum())
    return TwoSitePsi(psi=np.ascontiguousarray((X * s) @ Y.T), schmidt=s, left=X)


def block_operators(n: int, count: int, seed: int = 0) -> np.ndarray:
    """count symmetric n x n operators sym(N(0,1)) / sqrt(n) (spectral norm ~ 2)."""
    rng = np.random.default_rng(seed)
    out = np.empty((count, n, n))
    for c in range(count):
        out[c] = symmetrize(rng.standard_normal((n, n))) / math.sqrt(n)
    return out
