"""GPU truncation and renormalisation: the block-Jacobi RDM eigensolver
against LAPACK's eigh (eigenvalues, residuals, orthogonality, kept subspace)
in native and emulated arithmetic, the truncation of a planted two-site
tensor, and ozaki_renormalize bit-exact against the oracle's GEMM
composition (emulated) or within the FP64 GEMM bound (native)."""
import numpy as np
import pytest

import oracle
from paper_2510_04795_amd import workloads as wl
from tests.helpers import assert_bitexact

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def oz():
    import torch
    from paper_2510_04795_amd import ozaki
    torch.cuda.init()
    ctx = ozaki.Context(0)
    yield ozaki, ctx, torch
    ctx.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def u_eff(S):
    return U64 if S == 0 else max(U64, 2.0 ** (1 - 8 * S))


def solve(oz, A, S=0, nev=None, **kw):
    ozaki, ctx, torch = oz
    eig = ozaki.RdmEig(ctx, A.shape[0], S)
    try:
        w, Z, info = eig.solve(dev(torch, A), nev, **kw)
        return w.cpu().numpy(), Z.cpu().numpy(), info
    finally:
        eig.close()


def check_eigenpairs(A, w, Z, S, slack=1.0):
    """Eigenvalues against LAPACK, residual and orthogonality, all within
    64 sqrt(n) u |A|_2 (u of the arithmetic in use)."""
    n = A.shape[0]
    nev = w.size
    ref = oracle.rdm_eigh(A, nev)[0]
    norm = max(np.linalg.norm(A, 2), np.finfo(float).tiny)
    tol = slack * 64 * np.sqrt(n) * u_eff(S)
    assert np.all(np.diff(w) <= 0), "eigenvalues not in decreasing order"
    assert np.max(np.abs(w - ref)) <= tol * norm, np.max(np.abs(w - ref)) / norm
    res = np.linalg.norm(A @ Z - Z * w, axis=0)
    assert np.max(res) <= tol * norm, np.max(res) / norm
    assert np.max(np.abs(Z.T @ Z - np.eye(nev))) <= tol, np.max(np.abs(Z.T @ Z - np.eye(nev)))


def wishart(n, r=None, seed=0):
    B = np.random.default_rng(seed).standard_normal((n, n if r is None else r))
    return B @ B.T / n


@pytest.mark.parametrize("n", [1, 40, 200, 513])
def test_fp64_wishart(oz, n):
    A = wishart(n, seed=n)
    w, Z, info = solve(oz, A)
    assert info.status == 1 and info.sweeps >= 1
    check_eigenpairs(A, w, Z, 0)
    assert abs(info.trace - np.trace(A)) <= 1e-12 * abs(np.trace(A))


@pytest.mark.parametrize("n", [64, 300])
def test_fp64_planted_rdm(oz, n):
    """An RDM whose spectrum decays to e^-64: the clustered tail of tiny
    eigenvalues converges slowly (linear phase of cyclic Jacobi), but the
    kept quarter must be resolved to FP64 accuracy within the sweep limit."""
    t = wl.two_site_psi(n, tau=n / 64.0, seed=1)
    A = t.psi @ t.psi.T
    w, Z, info = solve(oz, A, nev=n // 4)
    assert info.status in (1, 3)
    check_eigenpairs(A, w, Z, 0)
    assert np.max(np.abs(w - t.schmidt[: n // 4] ** 2)) <= 64 * np.sqrt(n) * U64 * w[0]


@pytest.mark.parametrize("S", [7, 5, 4, 3])
def test_emulated_accuracy_follows_slices(oz, S):
    """With the Gram and rotation GEMMs emulated, the eigenpairs keep the
    accuracy of the emulation's 8S - 1 bits."""
    A = wishart(256, seed=2)
    w, Z, info = solve(oz, A, S)
    assert info.status in (1, 2)
    check_eigenpairs(A, w, Z, S)


@pytest.mark.parametrize("seed", range(8))
def test_random_symmetric(oz, seed):
    """Seeded random symmetric matrices: sizes 2..300 (off the 32-row
    blocks), positive semidefinite of full or deficient rank, or indefinite;
    a random number of wanted eigenpairs; FP64 or S = 4..7.  Eigenvalues,
    residuals and orthogonality within the bound of the arithmetic."""
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(2, 301))
    kind = int(rng.integers(0, 3))
    if kind == 0:
        A = wishart(n, seed=800 + seed)
    elif kind == 1:
        A = wishart(n, r=int(rng.integers(1, n + 1)), seed=800 + seed)
    else:
        X = np.random.default_rng(800 + seed).standard_normal((n, n))
        A = (X + X.T) / 2
    nev = int(rng.integers(1, n + 1))
    S = int(rng.choice([0, 4, 5, 6, 7]))
    w, Z, info = solve(oz, A, S, nev=nev)
    assert info.status in (1, 2, 3), (seed, n, kind, nev, S, info.status)
    check_eigenpairs(A, w, Z, S)


def test_edge_matrices(oz):
    # zero matrix: all eigenvalues 0, orthonormal eigenvectors
    w, Z, info = solve(oz, np.zeros((50, 50)))
    assert np.all(w == 0) and np.max(np.abs(Z.T @ Z - np.eye(50))) < 1e-14
    # identity (one eigenvalue of multiplicity n)
    w, Z, _ = solve(oz, np.eye(70))
    assert np.max(np.abs(w - 1)) < 1e-14 and np.max(np.abs(Z.T @ Z - np.eye(70))) < 1e-14
    # diagonal with distinct entries: unit eigenvectors, sorted values
    d = np.random.default_rng(3).permutation(np.arange(1.0, 91.0))
    w, Z, info = solve(oz, np.diag(d))
    assert np.array_equal(w, np.sort(d)[::-1])
    assert np.array_equal(np.abs(Z), np.eye(90)[:, np.argsort(-d)])
    # rank-deficient: the nonzero part is resolved, the rest is ~0
    A = wishart(120, r=30, seed=4)
    w, Z, info = solve(oz, A)
    check_eigenpairs(A, w, Z, 0)
    assert np.max(np.abs(w[30:])) < 1e-13 * w[0]
    # nev = 0 and nev < n
    w, Z, _ = solve(oz, A, nev=0)
    assert w.size == 0 and Z.shape == (120, 0)
    w5, Z5, _ = solve(oz, A, nev=5)
    check_eigenpairs(A, w5, Z5, 0)


def test_errors(oz):
    ozaki, ctx, torch = oz
    for n in (0, 8193):
        with pytest.raises(ozaki.OzakiError):
            ozaki.RdmEig(ctx, n)
    with pytest.raises(ozaki.OzakiError):
        ozaki.RdmEig(ctx, 64, slices=1)
    eig = ozaki.RdmEig(ctx, 16)
    A = np.eye(16)
    A[3, 5] = np.nan
    with pytest.raises(ozaki.OzakiError):
        eig.solve(dev(torch, A))
    with pytest.raises(ozaki.OzakiError):
        eig.solve(dev(torch, np.eye(16)), 17)
    with pytest.raises(ozaki.OzakiError):
        eig.solve(dev(torch, np.eye(16)), max_sweeps=0)
    # the plan is still usable after rejected calls
    w, Z, info = eig.solve(dev(torch, np.diag(np.arange(16.0))))
    assert np.array_equal(w.cpu().numpy(), np.arange(15.0, -1.0, -1.0))
    eig.close()


def test_two_calls_share_a_plan(oz):
    ozaki, ctx, torch = oz
    eig = ozaki.RdmEig(ctx, 100, 6)
    for seed in (5, 6):
        A = wishart(100, seed=seed)
        w, Z, info = eig.solve(dev(torch, A))
        check_eigenpairs(A, w.cpu().numpy(), Z.cpu().numpy(), 6)
    eig.close()


@pytest.mark.parametrize("S", [0, 5])
def test_truncate_matches_oracle(oz, S):
    """rho is bit-exact with the oracle's (emulated) or within the FP64 GEMM
    bound; the kept subspace, eigenvalues and discarded weight agree."""
    ozaki, ctx, torch = oz
    t = wl.two_site_psi(160, 144, tau=8.0, seed=7)
    D = 40
    psi = dev(torch, t.psi)
    rho = ctx.dgemm(psi, psi, slices=S, transb="T").cpu().numpy()
    if S:
        assert_bitexact(rho, oracle.ozaki_dgemm(t.psi, t.psi, S, transb="T"), "rho")
    else:
        ap = np.abs(t.psi)
        gam = 144 * U64 / (1 - 144 * U64)
        assert np.all(np.abs(rho - t.psi @ t.psi.T) <= 2 * gam * (ap @ ap.T))
    U, w, dw, info = ozaki.truncate(ctx, psi, D, slices=S)
    U_ref, w_ref, dw_ref = oracle.truncate(t.psi, D, S=S)
    tol = 64 * np.sqrt(160) * u_eff(S)
    assert np.max(np.abs(w.cpu().numpy() - w_ref)) <= tol * w_ref[0]
    assert abs(dw - dw_ref) <= tol
    sv = np.linalg.svd(U_ref.T @ U.cpu().numpy(), compute_uv=False)
    assert np.all(np.abs(sv - 1) < 1e-8)


@pytest.mark.parametrize("S", [3, 6])
def test_renormalize_bitexact(oz, S):
    ozaki, ctx, torch = oz
    n, D = 200, 64
    ops = wl.block_operators(n, 3, seed=8)
    t = wl.two_site_psi(n, tau=10.0, seed=9)
    U = oracle.truncate(t.psi, D)[0]
    out = ctx.renormalize(dev(torch, U), [dev(torch, o) for o in ops], slices=S)
    for got, want in zip(out, oracle.renormalize(U, ops, S=S)):
        assert_bitexact(got.cpu().numpy(), want, "renormalize S=%d" % S)


@pytest.mark.parametrize("seed", range(6))
def test_renormalize_random_bitexact(oz, seed):
    """Seeded random renormalisations: n = 1..260, D = 1..n, 1 to 4
    operators with entries spread over 2^-6..2^6, a general (not orthonormal)
    U, S = 2..8 with every built ndiag: the oracle's bits."""
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(1, 261))
    D = int(rng.integers(1, n + 1))
    k = int(rng.integers(1, 5))
    S = int(rng.integers(2, 9))
    G = int(rng.choice(sorted({S, S + 1, 2 * S - 1})))

    def spread(shape):
        return np.ldexp(rng.standard_normal(shape), rng.integers(-6, 7, size=shape))

    U = spread((n, D))
    ops = [spread((n, n)) for _ in range(k)]
    out = ctx.renormalize(dev(torch, U), [dev(torch, o) for o in ops], slices=S, ndiag=G)
    for i, (got, want) in enumerate(zip(out, oracle.renormalize(U, ops, S=S, G=G))):
        assert_bitexact(got.cpu().numpy(), want, "seed %d n=%d D=%d S=%d G=%d operator %d" % (seed, n, D, S, G, i))


def test_renormalize_fp64_and_errors(oz):
    ozaki, ctx, torch = oz
    n, D = 130, 33
    ops = wl.block_operators(n, 2, seed=10)
    U = np.linalg.qr(np.random.default_rng(11).standard_normal((n, D)))[0]
    out = ctx.renormalize(dev(torch, U), [dev(torch, o) for o in ops], slices=0)
    gam = n * U64 / (1 - n * U64)
    for O, got in zip(ops, out):
        bound = 3 * gam * (np.abs(U).T @ np.abs(O) @ np.abs(U))
        assert np.all(np.abs(got.cpu().numpy() - U.T @ O @ U) <= bound)
    with pytest.raises(ValueError):
        ctx.renormalize(dev(torch, U), [dev(torch, np.zeros((n, n + 1)))])
    with pytest.raises(ozaki.OzakiError):
        ctx.renormalize(dev(torch, np.zeros((n, n + 1))), [dev(torch, ops[0])])
    assert ctx.renormalize(dev(torch, U), [], slices=4) == []


@pytest.mark.parametrize("S", [0, 7])
def test_large_rdm(oz, S):
    """n = 2048 (a two-site tensor of D = 512, d = 4): the dominant quarter
    of the spectrum against the planted values."""
    t = wl.two_site_psi(2048, seed=12)
    A = t.psi @ t.psi.T
    w, Z, info = solve(oz, A, S, nev=512)
    assert info.status in (1, 2, 3), info.status
    assert np.max(np.abs(w - t.schmidt[:512] ** 2)) <= 64 * np.sqrt(2048) * u_eff(S) * w[0]
    res = np.linalg.norm(A @ Z - Z * w, axis=0)
    assert np.max(res) <= 64 * np.sqrt(2048) * u_eff(S) * w[0]
