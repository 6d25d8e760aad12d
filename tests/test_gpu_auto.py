"""GPU tests of the emulation modes: automatic slice count (device statistics
and choice against the oracle's), eager width from a mantissa bit count,
performant dispatch (path taken, results exact for the emulated path and
within the FP64 bound for the native one)."""
import numpy as np
import pytest

import oracle
from paper_2510_04795_amd import workloads as wl
from tests.helpers import assert_bitexact

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("U", [0, 10, 30])
@pytest.mark.parametrize("transa,transb", [("N", "N"), ("T", "N"), ("N", "T")])
def test_choose_slices_matches_oracle(oz, U, transa, transb):
    ozaki, ctx, torch = oz
    A, B = wl.gemm_pair(200, U=U, seed=20 + U, m=190, k=170)
    As = A.T.copy() if transa == "T" else A
    Bs = B.T.copy() if transb == "T" else B
    S, G, st = ctx.choose_slices(dev(torch, As), dev(torch, Bs), transa=transa, transb=transb)
    ra, rb = oracle.rho(A), oracle.rho(B, by_columns=True)
    assert st["rho_a"] == pytest.approx(ra, rel=1e-12)
    assert st["rho_b"] == pytest.approx(rb, rel=1e-12)
    assert (S, G) == oracle.choose_slices(A, B)
    assert st["native"] == oracle.predicted_native_error(170)
    assert st["predicted"] <= st["native"]


def test_choose_slices_edge_cases(oz):
    ozaki, ctx, torch = oz
    A = np.zeros((40, 30))
    B = np.random.default_rng(1).standard_normal((30, 20))
    assert ctx.choose_slices(dev(torch, A), dev(torch, B))[:2] == (2, 2)
    A = np.random.default_rng(2).standard_normal((40, 30))
    A[3, 4] = np.inf
    assert ctx.choose_slices(dev(torch, A), dev(torch, B))[:2] == (7, 7)
    assert ctx.choose_slices(dev(torch, np.zeros((0, 30))), dev(torch, B))[:2] == (2, 2)


def test_dgemm_auto_bits_is_eager(oz):
    ozaki, ctx, torch = oz
    A, B = wl.gemm_pair(160, U=10, seed=31, m=150, k=140)
    dA, dB = dev(torch, A), dev(torch, B)
    for bits, S in [(53, 7), (47, 6), (63, 8), (7, 2)]:
        C, s, g = ctx.dgemm_auto(dA, dB, bits=bits)
        assert (s, g) == (S, S)
        assert_bitexact(C.cpu().numpy(), oracle.ozaki_dgemm(A, B, S, S), "bits=%d" % bits)


def test_dgemm_auto_automatic_width(oz):
    ozaki, ctx, torch = oz
    A, B = wl.gemm_pair(256, U=30, seed=32, m=230, k=250)
    C0 = np.random.default_rng(3).standard_normal((230, 256))
    dA, dB = dev(torch, A), dev(torch, B)
    C = dev(torch, C0)
    _, s, g = ctx.dgemm_auto(dA, dB, bits=0, alpha=0.5, beta=-2.0, C=C)
    assert (s, g) == oracle.choose_slices(A, B)
    want = oracle.ozaki_dgemm(A, B, s, g, alpha=0.5, beta=-2.0, C=C0)
    assert_bitexact(C.cpu().numpy(), want, "automatic width")


@pytest.mark.parametrize("seed", range(8))
def test_automatic_width_random(oz, seed):
    """Seeded random products (sizes 1..300, entries spread 2^-U..2^U with
    U = 0..40, rows and columns rescaled by up to 2^+-20, random transposes):
    the library's (S, G) and rho equal the oracle's, and the automatic-width
    GEMM gives the oracle's bits at that width."""
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(1000 + seed)
    m, k, n = (int(x) for x in rng.integers(1, 301, size=3))
    U = int(rng.integers(0, 41))
    A = np.ldexp(rng.standard_normal((m, k)), rng.integers(-U, U + 1, size=(m, k)))
    B = np.ldexp(rng.standard_normal((k, n)), rng.integers(-U, U + 1, size=(k, n)))
    if rng.random() < 0.5:
        A = np.ldexp(A, rng.integers(-20, 21, size=(m, 1)))
        B = np.ldexp(B, rng.integers(-20, 21, size=(1, n)))
    ta, tb = ("T" if rng.random() < 0.5 else "N"), ("T" if rng.random() < 0.5 else "N")
    As = A.T.copy() if ta == "T" else A
    Bs = B.T.copy() if tb == "T" else B
    S, G, st = ctx.choose_slices(dev(torch, As), dev(torch, Bs), transa=ta, transb=tb)
    what = "seed %d %dx%dx%d U=%d %s%s" % (seed, m, k, n, U, ta, tb)
    assert (S, G) == oracle.choose_slices(A, B), what
    assert st["rho_a"] == pytest.approx(oracle.rho(A), rel=1e-12), what
    assert st["rho_b"] == pytest.approx(oracle.rho(B, by_columns=True), rel=1e-12), what
    C, s, g = ctx.dgemm_auto(dev(torch, As), dev(torch, Bs), bits=0, transa=ta, transb=tb)
    assert (s, g) == (S, G), what
    assert_bitexact(C.cpu().numpy(), oracle.ozaki_dgemm(A, B, s, g), what)


def test_dgemm_auto_performant(oz):
    """The first beta = 0 call of a shape times both paths and keeps one; the
    result is the kept path's (bit-exact for the emulated one, FP64 bound for
    the native one) and later calls report the same path."""
    ozaki, ctx, torch = oz
    u = 2.0 ** -53
    for (m, n, k) in [(64, 48, 40), (512, 512, 512)]:
        A, B = wl.gemm_pair(n, U=10, seed=33, m=m, k=k)
        dA, dB = dev(torch, A), dev(torch, B)
        C, s, g = ctx.dgemm_auto(dA, dB, bits=53, performant=True)
        got = C.cpu().numpy()
        if s == 0:
            hi, lo = oracle.dgemm_dd(A, B)
            gam = k * u / (1 - k * u)
            assert np.all(np.abs((got - hi) - lo) <= gam * (np.abs(A) @ np.abs(B)))
        else:
            assert (s, g) == (7, 7)
            assert_bitexact(got, oracle.ozaki_dgemm(A, B, 7, 7), "performant emulated")
        for _ in range(2):
            _, s2, g2 = ctx.dgemm_auto(dA, dB, bits=53, performant=True)
            assert (s2, g2) == (s, g)
    # a shape first seen with beta != 0 is not timed: the emulated path runs
    A, B = wl.gemm_pair(72, U=10, seed=34, m=70, k=66)
    C0 = np.ones((70, 72))
    C = dev(torch, C0)
    _, s, g = ctx.dgemm_auto(dev(torch, A), dev(torch, B), bits=53, performant=True, beta=1.0, C=C)
    assert (s, g) == (7, 7)
    assert_bitexact(C.cpu().numpy(), oracle.ozaki_dgemm(A, B, 7, 7, beta=1.0, C=C0), "untimed shape")


def test_dgemm_auto_errors(oz):
    ozaki, ctx, torch = oz
    A = dev(torch, np.ones((8, 8)))
    with pytest.raises(ozaki.OzakiError):
        ctx.dgemm_auto(A, A, bits=-1)
    with pytest.raises(ozaki.OzakiError):
        ctx.dgemm_auto(A, A, performant=2)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ozaki.OzakiError) as ei:
        ctx.dgemm_auto(A, A, workspace=small)
    assert ei.value.status == -2
