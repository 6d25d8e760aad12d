"""GPU parity of the emulated-FP64 GEMM against the CPU oracle.

Steps 1-2 (exponents, slices) and step 3 (int32 diagonal sums) must agree bit
for bit; the whole emulated GEMM must agree bit for bit as well (both sides
run the same FP64 recombination order).  The native FP64 MFMA path is held to
the textbook gamma_K |A||B| bound against the double-double reference.
Shapes span several tiles with ragged edges.
"""
import numpy as np
import pytest

import oracle
from paper_2510_04795_amd import workloads as wl
from tests.helpers import assert_bitexact

pytestmark = pytest.mark.gpu

SG = [(S, G) for S in range(2, 9) for G in sorted({S, S + 1, 2 * S - 1})]


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


def edge_matrix(rng, rows, cols, U):
    X = wl.wide_normal(rng, (rows, cols), U)
    X[min(1, rows - 1), :] = 0.0                  # a zero row
    X[rows // 2, cols // 3] = 5e-324              # a subnormal
    X[-1, 0] = 127 / 128 * 2.0 ** 40              # at the exponent bump boundary
    X[-1, -1] = -(127 / 128 + 2.0 ** -52) * 2.0 ** 40
    return X


@pytest.mark.parametrize("S", range(2, 9))
@pytest.mark.parametrize("by_columns", [False, True])
def test_split_bitexact(oz, S, by_columns):
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(S * 10 + by_columns)
    for (rows, cols, U) in [(77, 45, 10), (33, 130, 30), (1, 1, 5)]:
        X = edge_matrix(rng, rows, cols, U) if rows > 2 else wl.wide_normal(rng, (rows, cols), U)
        d, e = ctx.split(dev(torch, X), S, by_columns=by_columns)
        rd, re_, rb = oracle.split(X, S, by_columns=by_columns)
        if by_columns:
            rd = np.transpose(rd, (0, 2, 1))
        assert np.array_equal(e.cpu().numpy(), np.where(rb == 1, ozaki.OZ_EXP_NONFINITE, re_))
        assert np.array_equal(d.cpu().numpy(), rd)


@pytest.mark.parametrize("seed", range(8))
def test_split_and_pair_products_random(oz, seed):
    """Seeded random shapes (1..260 around the 32-wide groups and K blocks),
    spreads U = 0..60 with scattered zeros and subnormals, both orientations,
    S = 2..8 and every built ndiag: the oracle's exponents, digits and int32
    diagonal sums."""
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(1100 + seed)
    M, N, K = (int(x) for x in rng.integers(1, 261, size=3))
    S = int(rng.integers(2, 9))
    G = int(rng.choice(sorted({S, S + 1, 2 * S - 1})))
    U = int(rng.integers(0, 61))

    def draw(shape):
        X = wl.wide_normal(rng, shape, U)
        X[rng.random(shape) < 0.05] = 0.0
        X[rng.random(shape) < 0.02] *= 2.0 ** -1060
        return X

    A, B = draw((M, K)), draw((K, N))
    what = "seed %d %dx%dx%d S=%d G=%d U=%d" % (seed, M, K, N, S, G, U)
    for X, by_columns in ((A, False), (B, True)):
        d, e = ctx.split(dev(torch, X), S, by_columns=by_columns)
        rd, re_, rb = oracle.split(X, S, by_columns=by_columns)
        if by_columns:
            rd = np.transpose(rd, (0, 2, 1))
        assert np.array_equal(e.cpu().numpy(), np.where(rb == 1, ozaki.OZ_EXP_NONFINITE, re_)), what
        assert np.array_equal(d.cpu().numpy(), rd), what
    Ad, _, _ = oracle.split(A, S)
    Bd, _, _ = oracle.split(B, S, by_columns=True)
    if K <= ozaki.max_exact_k(S, G):
        Q = ctx.pair_products(dev(torch, Ad), dev(torch, np.transpose(Bd, (0, 2, 1))), S, G)
        assert np.array_equal(Q.cpu().numpy().astype(np.int64), oracle.pair_products(Ad, Bd, G)), what


def test_split_nonfinite_flag(oz):
    ozaki, ctx, torch = oz
    ctx.flags()
    X = np.ones((5, 7))
    X[2, 3] = np.nan
    X[4, 0] = -np.inf
    d, e = ctx.split(dev(torch, X), 6)
    e = e.cpu().numpy()
    assert e[2] == ozaki.OZ_EXP_NONFINITE and e[4] == ozaki.OZ_EXP_NONFINITE and e[0] == 1
    assert np.all(d.cpu().numpy()[:, [2, 4], :] == 0)
    assert ctx.flags() & ozaki.OZ_FLAG_NONFINITE
    assert ctx.flags() == 0


@pytest.mark.parametrize("S,G", SG)
def test_pair_products_bitexact(oz, S, G):
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(100 + S * 16 + G)
    M, N, K = 150, 97, 333
    A = wl.wide_normal(rng, (M, K), 20)
    B = wl.wide_normal(rng, (K, N), 20)
    Ad, _, _ = oracle.split(A, S)
    Bd, _, _ = oracle.split(B, S, by_columns=True)
    Q = ctx.pair_products(dev(torch, Ad), dev(torch, np.transpose(Bd, (0, 2, 1))), S, G)
    ref = oracle.pair_products(Ad, Bd, G)
    assert np.abs(ref).max() < 2 ** 31
    assert np.array_equal(Q.cpu().numpy().astype(np.int64), ref)


@pytest.mark.parametrize("S,G", SG)
def test_dgemm_bitexact(oz, S, G):
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(200 + S * 16 + G)
    M, N, K = 200, 131, 300
    A = wl.wide_normal(rng, (M, K), 10)
    B = wl.wide_normal(rng, (K, N), 10)
    C = ctx.dgemm(dev(torch, A), dev(torch, B), slices=S, ndiag=G).cpu().numpy()
    assert_bitexact(C, oracle.ozaki_dgemm(A, B, S, G), "S=%d G=%d" % (S, G))


@pytest.mark.parametrize("transa,transb", [("N", "T"), ("T", "N"), ("T", "T")])
def test_dgemm_transposes_alpha_beta(oz, transa, transb):
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(7)
    M, N, K = 96, 160, 70
    A = wl.wide_normal(rng, (M, K), 30)
    B = wl.wide_normal(rng, (K, N), 30)
    As = A.T.copy() if transa == "T" else A
    Bs = B.T.copy() if transb == "T" else B
    C0 = rng.standard_normal((M, N))
    for (alpha, beta) in [(1.0, 0.0), (-2.5, 0.75), (0.0, 1.0)]:
        got = ctx.dgemm(dev(torch, As), dev(torch, Bs), slices=6, alpha=alpha, beta=beta,
                        C=dev(torch, C0), transa=transa, transb=transb).cpu().numpy()
        ref = oracle.ozaki_dgemm(As, Bs, 6, 6, alpha=alpha, beta=beta, C=C0, transa=transa,
                                 transb=transb)
        assert_bitexact(got, ref, "%s%s a=%g b=%g" % (transa, transb, alpha, beta))


def test_dgemm_leading_dimensions(oz):
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(8)
    big = wl.wide_normal(rng, (90, 120), 10)
    A, B = big[:70, :50], big[5:55, 60:117]
    Ad, Bd = dev(torch, big)[:70, :50], dev(torch, big)[5:55, 60:117]
    Cbuf = torch.zeros((70, 80), dtype=torch.float64, device="cuda")
    ctx.dgemm(Ad, Bd, slices=7, C=Cbuf[:, 10:67])
    assert_bitexact(Cbuf[:, 10:67].cpu().numpy(), oracle.ozaki_dgemm(A.copy(), B.copy(), 7), "ld")
    assert np.all(Cbuf[:, :10].cpu().numpy() == 0) and np.all(Cbuf[:, 67:].cpu().numpy() == 0)


def test_dgemm_nonfinite_and_degenerate(oz):
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(9)
    A = rng.standard_normal((40, 33))
    B = rng.standard_normal((33, 50))
    A[3, 7] = np.nan
    B[10, 44] = np.inf
    ctx.flags()
    got = ctx.dgemm(dev(torch, A), dev(torch, B), slices=5).cpu().numpy()
    assert_bitexact(got, oracle.ozaki_dgemm(A, B, 5), "nan")
    assert ctx.flags() & ozaki.OZ_FLAG_NONFINITE
    C0 = rng.standard_normal((4, 6))
    got = ctx.dgemm(dev(torch, np.zeros((4, 0))), dev(torch, np.zeros((0, 6))), slices=6,
                    alpha=3.0, beta=0.5, C=dev(torch, C0)).cpu().numpy()
    assert_bitexact(got, 0.5 * C0, "K=0")
    one = ctx.dgemm(dev(torch, np.array([[3.0]])), dev(torch, np.array([[-0.5]])), slices=4)
    assert one.item() == -1.5


def test_dgemm_chunked_inner_dimension(oz):
    """K above the exact int32 range: chunks carried in int64, same result."""
    ozaki, ctx, torch = oz
    S = 8
    K = 40000
    assert K > ozaki.max_exact_k(S)
    rng = np.random.default_rng(10)
    A = wl.wide_normal(rng, (37, K), 6)
    B = wl.wide_normal(rng, (K, 29), 6)
    got = ctx.dgemm(dev(torch, A), dev(torch, B), slices=S).cpu().numpy()
    assert_bitexact(got, oracle.ozaki_dgemm(A, B, S), "chunked")


def test_dgemm_argument_errors(oz):
    ozaki, ctx, torch = oz
    A = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(ozaki.OzakiError):
        ctx.dgemm(A, A, slices=9)
    with pytest.raises(ozaki.OzakiError):
        ctx.dgemm(A, A, slices=6, ndiag=8)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ozaki.OzakiError) as ei:
        ctx.dgemm(A, A, slices=6, workspace=small)
    assert ei.value.status == -2


@pytest.mark.parametrize("transa,transb", [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")])
def test_fp64_mfma_within_gamma_bound(oz, transa, transb):
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(11)
    M, N, K = 130, 70, 257
    A = wl.wide_normal(rng, (M, K), 10)
    B = wl.wide_normal(rng, (K, N), 10)
    As = A.T.copy() if transa == "T" else A
    Bs = B.T.copy() if transb == "T" else B
    got = ctx.dgemm(dev(torch, As), dev(torch, Bs), slices=0, transa=transa,
                    transb=transb).cpu().numpy()
    hi, lo = oracle.dgemm_dd(A, B)
    u = 2.0 ** -53
    gam = K * u / (1 - K * u)
    err = np.abs((got - hi) - lo)
    assert np.all(err <= gam * (np.abs(A) @ np.abs(B)) * (1 + 1e-12))


@pytest.mark.parametrize("transa,transb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_fp64_mfma_large_tiles_within_gamma_bound(oz, transa, transb):
    """An extent large enough for the 128 x 128 FP64 tiles (ragged in every
    dimension, alpha and beta), sampled rows against the double-double sum."""
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(12)
    M, N, K = 3001, 2950, 333
    A = wl.wide_normal(rng, (M, K), 10)
    B = wl.wide_normal(rng, (K, N), 10)
    C0 = rng.standard_normal((M, N))
    As = A.T.copy() if transa == "T" else A
    Bs = B.T.copy() if transb == "T" else B
    C = dev(torch, C0)
    ctx.dgemm(dev(torch, As), dev(torch, Bs), slices=0, transa=transa, transb=transb,
              alpha=-1.5, beta=0.5, C=C)
    rows = np.array([0, 127, 128, 1500, 2999, 3000])
    got = C.cpu().numpy()[rows]
    hi, lo = oracle.dgemm_dd(A[rows], B)
    u = 2.0 ** -53
    gam = (K + 2) * u / (1 - (K + 2) * u)
    ref = -1.5 * hi + 0.5 * C0[rows]
    mag = 1.5 * (np.abs(A[rows]) @ np.abs(B)) + 0.5 * np.abs(C0[rows])
    err = np.abs(got - ref - (-1.5 * lo))
    assert np.all(err <= gam * mag * (1 + 1e-12) + 4 * u * np.abs(ref))


@pytest.mark.parametrize("S,variant", [(6, -1), (7, 4), (7, 0), (6, 0)])
def test_dgemm_full_size_sampled_rows(oz, S, variant):
    """n = 8192: S = 6 with the default tile, and S = G = 7 on the 64 x 128
    tile (three-stage ring) and on the 64 x 64 tile (two-stage ring, the
    launch the benchmark's tuning takes for its equal-error line), S = 6 on
    the 64 x 64 tile (three-stage ring); checked on sampled rows (exponents
    are per row of A and per column of B, so rows are independent)."""
    ozaki, ctx, torch = oz
    n = 8192
    A, B = wl.gemm_pair(n, U=10, seed=0)
    ctx.set_variant(S, 0, variant)
    try:
        Cd = ctx.dgemm(dev(torch, A), dev(torch, B), slices=S)
    finally:
        ctx.set_variant(S, 0, -1)
    rows = np.random.default_rng(1).choice(n, size=6, replace=False)
    got = Cd[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = oracle.ozaki_dgemm(A[rows], B, S)
    assert_bitexact(got, ref, "n=8192 rows S=%d" % S)


@pytest.mark.parametrize("S,G", [(2, 3), (4, 4), (5, 6), (6, 6), (7, 7), (7, 8), (8, 8), (7, 13)])
def test_every_tile_variant_bitexact(oz, S, G):
    """Tile variants change only the schedule: all give the oracle's bits."""
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(300 + S * 16 + G)
    A = wl.wide_normal(rng, (150, 270), 12)
    B = wl.wide_normal(rng, (270, 199), 12)
    ref = oracle.ozaki_dgemm(A, B, S, G)
    variants = ozaki.pair_variants(S, G)
    assert variants and all(tm % 64 == 0 and tn % 64 == 0 for (_, tm, tn) in variants)
    try:
        for (v, tm, tn) in variants:
            ctx.set_variant(S, G, v)
            assert ctx.get_variant(S, G) == v
            got = ctx.dgemm(dev(torch, A), dev(torch, B), slices=S, ndiag=G).cpu().numpy()
            assert_bitexact(got, ref, "variant %d (%dx%d)" % (v, tm, tn))
    finally:
        ctx.set_variant(S, G, -1)


def test_tune_picks_a_built_variant(oz):
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(12)
    A = dev(torch, wl.wide_normal(rng, (512, 512), 10))
    B = dev(torch, wl.wide_normal(rng, (512, 512), 10))
    v, times = ctx.tune(A, B, slices=6)
    assert v in [x[0] for x in ozaki.pair_variants(6)]
    assert set(times) == set(x[0] for x in ozaki.pair_variants(6))
    assert ctx.get_variant(6) == v
    ctx.set_variant(6, 0, -1)
    with pytest.raises(ozaki.OzakiError):
        ctx.set_variant(8, 15, 3)   # 2x2 blocks of 15 accumulator sets are not built


@pytest.mark.parametrize("S,G", [(2, 3), (5, 5), (8, 15)])
def test_dgemm_vector_shapes_zero_rows_and_extreme_exponents(oz, S, G):
    """M = 1 and N = 1 products, a zero row of A and a zero column of B,
    subnormal entries and entries near 2^900 and 2^-1000 in the same operands: the
    emulated GEMM stays bit-exact with the oracle."""
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(40 + S)
    A = rng.standard_normal((37, 301)) * np.ldexp(1.0, rng.integers(-20, 20, size=(37, 301)))
    B = rng.standard_normal((301, 45)) * np.ldexp(1.0, rng.integers(-20, 20, size=(301, 45)))
    A[5] = 0.0
    B[:, 7] = 0.0
    A[9, :4] = [5e-324, -1e-310, 2.2e-308, 1e-300]
    A[11] = np.ldexp(A[11], 900)
    B[:, 13] = np.ldexp(B[:, 13], -1000)
    for (a, b) in [(A, B), (A[:1], B), (A, B[:, :1]), (A[:1], B[:, :1])]:
        got = ctx.dgemm(dev(torch, a), dev(torch, b), slices=S, ndiag=G).cpu().numpy()
        assert_bitexact(got, oracle.ozaki_dgemm(a, b, S, G), "shape %s x %s" % (a.shape, b.shape))


@pytest.mark.parametrize("seed", range(12))
def test_random_shapes_every_variant(oz, seed):
    """Seeded random products: shapes from 1 to 300 drawn near multiples of
    32 and 64 (tile edges one inside and one past a block), random
    transposes, alpha and beta, and (S, G) from every built combination,
    under every tile variant: the oracle's bits."""
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(5000 + seed)

    def dim():
        base = int(rng.choice([1, 32, 64, 96, 128, 160, 192, 256, 288]))
        return max(1, base + int(rng.integers(-1, 2)) * int(rng.integers(0, 2)) + int(rng.integers(0, 3)))

    S, G = SG[int(rng.integers(0, len(SG)))]
    M, N, K = dim(), dim(), dim()
    transa, transb = ("N", "T")[int(rng.integers(0, 2))], ("N", "T")[int(rng.integers(0, 2))]
    alpha, beta = float(rng.choice([1.0, -1.5, 0.5])), float(rng.choice([0.0, 1.0, -0.25]))
    A = wl.wide_normal(rng, (M, K), int(rng.integers(0, 31)))
    B = wl.wide_normal(rng, (K, N), int(rng.integers(0, 31)))
    As = A.T.copy() if transa == "T" else A
    Bs = B.T.copy() if transb == "T" else B
    C0 = rng.standard_normal((M, N))
    ref = oracle.ozaki_dgemm(As, Bs, S, G, alpha=alpha, beta=beta, C=C0, transa=transa, transb=transb)
    try:
        for (v, tm, tn) in ozaki.pair_variants(S, G):
            ctx.set_variant(S, G, v)
            got = ctx.dgemm(dev(torch, As), dev(torch, Bs), slices=S, ndiag=G, alpha=alpha, beta=beta,
                            C=dev(torch, C0), transa=transa, transb=transb).cpu().numpy()
            assert_bitexact(got, ref, "seed %d S=%d G=%d %dx%dx%d %s%s a=%g b=%g variant %d"
                            % (seed, S, G, M, N, K, transa, transb, alpha, beta, v))
    finally:
        ctx.set_variant(S, G, -1)


def test_binding_checks_output_shapes(oz):
    """A C of another shape than op(A) op(B), or outputs that do not match
    the operators, are refused by the binding before the library could
    write past them; a strided C of the right shape is accepted."""
    ozaki, ctx, torch = oz
    A, B = wl.gemm_pair(40, U=4, seed=3, m=24, k=32)
    dA, dB = dev(torch, A), dev(torch, B)
    for bad in [(23, 40), (24, 39), (40, 24)]:
        C = torch.zeros(bad, dtype=torch.float64, device="cuda")
        with pytest.raises(ValueError):
            ctx.dgemm(dA, dB, slices=6, C=C)
        with pytest.raises(ValueError):
            ctx.dgemm_auto(dA, dB, C=C)
        with pytest.raises(ValueError):
            ctx.tune(dA, dB, slices=6, C=C)
    with pytest.raises(TypeError):
        ctx.dgemm(dA, dB, slices=6, C=torch.zeros((24, 40), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        ctx.tune(dA, dev(torch, B[:31]), slices=6)
    buf = torch.zeros((24, 50), dtype=torch.float64, device="cuda")
    got = ctx.dgemm(dA, dB, slices=6, C=buf[:, 5:45]).cpu().numpy()
    assert_bitexact(got, oracle.ozaki_dgemm(A, B, 6), "strided C")
    U = dev(torch, np.linalg.qr(np.random.default_rng(0).standard_normal((40, 40)))[0][:, :8])
    ops = [dev(torch, A[:, :24].T @ A[:, :24] / 40.0 + np.eye(24)) for _ in range(2)]
    U24 = U[:24].contiguous()
    with pytest.raises(ValueError):
        ctx.renormalize(U24, ops, outs=[torch.empty((8, 8), dtype=torch.float64, device="cuda")])
    with pytest.raises(ValueError):
        ctx.renormalize(U24, ops, outs=[torch.empty((8, 7), dtype=torch.float64, device="cuda") for _ in ops])

