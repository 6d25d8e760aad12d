"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own formulas: printed values
of the paper (tests/golden/paper_values.json), exact rational arithmetic,
closed forms, characterisations by brute-force search, polynomial identities
and invariances that any correct implementation must satisfy.  A dropped
term, a wrong sign or index or a transposed operand in the oracle breaks at
least one of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2510_04795_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")
U53 = Fraction(1, 2 ** 53)


def exact_matmul(A, B):
    """Exact rational product of two float matrices (tiny sizes only)."""
    M, K = A.shape
    N = B.shape[1]
    FA = [[Fraction(float(A[i, k])) for k in range(K)] for i in range(M)]
    FB = [[Fraction(float(B[k, j])) for j in range(N)] for k in range(K)]
    return [[sum(FA[i][k] * FB[k][j] for k in range(K)) for j in range(N)] for i in range(M)]


# ---------------------------------------------------------------- paper values
def test_slices_for_bits_matches_paper():
    g = json.load(open(GOLDEN))["slices_to_mantissa_bits"]["pairs"]
    for S, bits in g:
        assert oracle.slices_for_bits(bits) == S
        # the next bit needs a new slice: 8S - 1 magnitude bits fit S slices
        assert oracle.slices_for_bits(bits + 1) == S + 1


def test_full_pair_count_matches_paper():
    g = json.load(open(GOLDEN))["full_pair_count"]
    S = g["slices"]
    assert oracle.pair_count(S, 2 * S - 1) == g["pairs"]
    # dropping the lower triangle: S(S+1)/2 pairs at G = S
    for S in range(1, 9):
        assert oracle.pair_count(S, S) == S * (S + 1) // 2
        assert oracle.pair_count(S, 2 * S - 1) == S * S


# ---------------------------------------------------------------- reference GEMMs
def test_dd_gemm_vs_exact_rationals():
    rng = np.random.default_rng(11)
    A = wl.wide_normal(rng, (8, 8), 30)
    B = wl.wide_normal(rng, (8, 8), 30)
    hi, lo = oracle.dgemm_dd(A, B)
    ex = exact_matmul(A, B)
    absAB = np.abs(A) @ np.abs(B)
    for i in range(8):
        for j in range(8):
            err = abs(Fraction(hi[i, j]) + Fraction(lo[i, j]) - ex[i][j])
            assert err <= Fraction(2 * 8) * Fraction(1, 2 ** 104) * Fraction(absAB[i, j]) * 2
            # hi is the FP64 number nearest to hi + lo
            assert abs(lo[i, j]) <= abs(hi[i, j]) * 2.0 ** -53


def test_fp64_gemm_within_gamma_bound():
    rng = np.random.default_rng(12)
    for (M, N, K) in [(5, 7, 9), (3, 4, 33)]:
        A = wl.wide_normal(rng, (M, K), 10)
        B = wl.wide_normal(rng, (K, N), 10)
        C = oracle.dgemm_fp64(A, B)
        ex = exact_matmul(A, B)
        gam = K * U53 / (1 - K * U53)
        absAB = np.abs(A) @ np.abs(B)
        for i in range(M):
            for j in range(N):
                assert abs(Fraction(C[i, j]) - ex[i][j]) <= gam * Fraction(absAB[i, j]) * (1 + U53 * 4)


def test_fp64_gemm_alpha_beta():
    rng = np.random.default_rng(13)
    A = rng.standard_normal((4, 6))
    B = rng.standard_normal((6, 5))
    C0 = rng.standard_normal((4, 5))
    C = oracle.dgemm_fp64(A, B, alpha=2.0, beta=0.5, C=C0)
    ref = oracle.dgemm_fp64(A, B)
    assert np.allclose(C, 2.0 * ref + 0.5 * C0, rtol=1e-15, atol=1e-15)
    Cn = np.full((4, 5), np.nan)
    assert np.all(np.isfinite(oracle.dgemm_fp64(A, B, beta=0.0, C=Cn)))


# ---------------------------------------------------------------- step 1: exponents
def _min_exponent(mu: float) -> int:
    """Smallest integer e with mu <= (127/128) 2^e, by search (mu > 0)."""
    fm = Fraction(mu)
    e = -1100
    while not fm <= Fraction(127, 128) * Fraction(2) ** e:
        e += 1
    return e


@pytest.mark.parametrize("S", [2, 4, 6, 8])
def test_exponent_characterisation(S):
    rng = np.random.default_rng(20 + S)
    rows = [wl.wide_normal(rng, 9, 30) for _ in range(6)]
    rows += [np.array([127 / 128, 0.1, -0.2]), np.array([-(127 / 128 + 2 ** -52), 0.0]),
             np.array([0.0, 0.0, 0.0]), np.array([5e-324, -1e-320]),
             np.array([2.0 ** 1000, -3.0]), np.array([2.0 ** -1000]), np.array([-1.0])]
    for r in rows:
        _, e, bad = oracle.split(r[None, :], S)
        mu = float(np.max(np.abs(r)))
        want = 0 if mu == 0 else _min_exponent(mu)
        assert bad[0] == 0
        assert int(e[0]) == want, (r, int(e[0]), want)


def test_nonfinite_groups_flagged():
    X = np.array([[1.0, np.nan, 2.0], [1.0, 2.0, 3.0], [np.inf, 0.0, 1.0]])
    d, e, bad = oracle.split(X, 5)
    assert list(bad) == [1, 0, 1]
    assert np.all(d[:, 0, :] == 0) and np.all(d[:, 2, :] == 0)
    d, f, badc = oracle.split(X, 5, by_columns=True)
    assert list(badc) == [1, 1, 0]


# ---------------------------------------------------------------- step 2: slices
@pytest.mark.parametrize("S", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("U", [10, 30])
def test_slices_reconstruct_within_half_unit(S, U):
    rng = np.random.default_rng(100 * S + U)
    X = wl.wide_normal(rng, (7, 23), U)
    X[3, :] = 0.0
    X[4, 5] = 5e-324
    d, e, bad = oracle.split(X, S)
    assert d.dtype == np.int8
    assert np.all(np.abs(d[0]) <= 127)
    assert np.all(d >= -128) and np.all(d <= 127)
    for i in range(X.shape[0]):
        unit = Fraction(2) ** (int(e[i]) - 8 * S + 1)
        for j in range(X.shape[1]):
            n = sum(int(d[t, i, j]) * 256 ** (S - 1 - t) for t in range(S))
            err = abs(Fraction(float(X[i, j])) - unit * n)
            assert err <= unit / 2
            if err == unit / 2:       # ties go to the even neighbour
                assert n % 2 == 0


def test_slices_ties_to_even():
    # row maximum 0.5 -> e = 0; S = 4 -> unit 2^-31
    S = 4
    vals = [0.5, 3 * 2.0 ** -32, 5 * 2.0 ** -32, -3 * 2.0 ** -32, 7 * 2.0 ** -32]
    d, e, _ = oracle.split(np.array([vals]), S)
    assert int(e[0]) == 0
    nums = [sum(int(d[t, 0, j]) * 256 ** (S - 1 - t) for t in range(S)) for j in range(len(vals))]
    assert nums[1:] == [2, 2, -2, 4]     # 1.5 -> 2, 2.5 -> 2, -1.5 -> -2, 3.5 -> 4


def test_slices_by_columns_is_transpose_of_rows():
    rng = np.random.default_rng(5)
    X = wl.wide_normal(rng, (9, 13), 20)
    dr, er, _ = oracle.split(X.T.copy(), 6)
    dc, ec, _ = oracle.split(X, 6, by_columns=True)
    assert np.array_equal(er, ec)
    assert np.array_equal(dr, np.transpose(dc, (0, 2, 1)))


# ---------------------------------------------------------------- step 3: pair products
@pytest.mark.parametrize("S", [3, 5, 8])
def test_pair_products_polynomial_identity(S):
    """sum_g x^g Q_g = sum_k (sum_s dA_s x^s)(sum_t dB_t x^t) for 2S-1 points x
    determines every diagonal Q_g (Vandermonde), computed here in Python ints."""
    rng = np.random.default_rng(30 + S)
    A = wl.wide_normal(rng, (4, 6), 15)
    B = wl.wide_normal(rng, (6, 5), 15)
    Ad, _, _ = oracle.split(A, S)
    Bd, _, _ = oracle.split(B, S, by_columns=True)
    G = 2 * S - 1
    Q = oracle.pair_products(Ad, Bd, G)
    for x in range(-S, S):
        pa = sum(Ad[s].astype(object) * x ** s for s in range(S))
        pb = sum(Bd[t].astype(object) * x ** t for t in range(S))
        lhs = sum(Q[g].astype(object) * x ** g for g in range(G))
        rhs = pa.dot(pb)
        assert np.array_equal(lhs, rhs), x
    # truncated mode keeps exactly the leading diagonals
    for Gt in range(1, G):
        assert np.array_equal(oracle.pair_products(Ad, Bd, Gt), Q[:Gt])


def test_pair_products_full_mode_equals_fixed_point_product():
    """Full mode: sum_g 256^(2S-2-g) Q_g equals the integer product of the
    fixed-point representatives sum_t d_t 256^(S-1-t)."""
    S = 4
    rng = np.random.default_rng(7)
    A = wl.wide_normal(rng, (3, 8), 12)
    B = wl.wide_normal(rng, (8, 4), 12)
    Ad, _, _ = oracle.split(A, S)
    Bd, _, _ = oracle.split(B, S, by_columns=True)
    Q = oracle.pair_products(Ad, Bd, 2 * S - 1)
    XA = sum(Ad[t].astype(object) * 256 ** (S - 1 - t) for t in range(S))
    XB = sum(Bd[t].astype(object) * 256 ** (S - 1 - t) for t in range(S))
    tot = sum(Q[g].astype(object) * 256 ** (2 * S - 2 - g) for g in range(2 * S - 1))
    assert np.array_equal(tot, XA.dot(XB))


# ---------------------------------------------------------------- step 4: recombination
def test_recombine_exact_rational_bound_and_alpha_beta():
    S, G = 6, 6
    rng = np.random.default_rng(40)
    A = wl.wide_normal(rng, (5, 40), 10)
    B = wl.wide_normal(rng, (40, 6), 10)
    Ad, e, _ = oracle.split(A, S)
    Bd, f, _ = oracle.split(B, S, by_columns=True)
    Q = oracle.pair_products(Ad, Bd, G)
    C = oracle.recombine(Q, e, f)
    for i in range(5):
        for j in range(6):
            scale = Fraction(2) ** (int(e[i]) + int(f[j]) - 14)
            terms = [Fraction(int(Q[g, i, j])) / Fraction(256) ** g for g in range(G)]
            exact = sum(terms) * scale
            mag = sum(abs(t) for t in terms) * scale
            assert abs(Fraction(C[i, j]) - exact) <= (G - 1) * U53 * mag
    # alpha/beta: out = RNE(alpha * c + RNE(beta * Cin)), checked in exact arithmetic
    Cin = rng.standard_normal((5, 6))
    out = oracle.recombine(Q, e, f, alpha=-1.5, beta=0.375, C=Cin)
    for i in range(5):
        for j in range(6):
            bc = float(Fraction(0.375) * Fraction(Cin[i, j]))
            want = float(Fraction(-1.5) * Fraction(C[i, j]) + Fraction(bc))
            assert out[i, j] == want
    # beta = 0 never reads C
    out0 = oracle.recombine(Q, e, f, alpha=2.0, beta=0.0, C=np.full((5, 6), np.nan))
    assert np.array_equal(out0, 2.0 * C)


def test_recombine_exact_when_representable():
    Q = np.array([[[3]], [[200]], [[-7]]], dtype=np.int64)     # G = 3
    c = oracle.recombine(Q, np.array([5]), np.array([-2]))
    exact = (Fraction(3) + Fraction(200, 256) - Fraction(7, 65536)) * Fraction(2) ** (5 - 2 - 14)
    assert Fraction(c[0, 0]) == exact


def test_recombine_nan_rows_columns():
    Q = np.ones((2, 3, 4), dtype=np.int64)
    out = oracle.recombine(Q, np.zeros(3), np.zeros(4), row_bad=np.array([0, 1, 0]),
                           col_bad=np.array([0, 0, 0, 1]))
    assert np.isnan(out[1]).all() and np.isnan(out[:, 3]).all()
    assert np.isfinite(out[[0, 2]][:, :3]).all()


# ---------------------------------------------------------------- whole emulated GEMM
@pytest.mark.parametrize("S", [5, 6, 7, 8])
@pytest.mark.parametrize("K", [1024, 4096])
def test_integer_inputs_exact(S, K):
    """Integers |a|, |b| <= 2^20: only digits t <= 2 are non-zero, every kept
    pair has s + t <= 4 < G = S, every partial sum is an integer below 2^53, so
    the emulated product equals the exact integer product."""
    rng = np.random.default_rng(50 + S)
    A = rng.integers(-2 ** 20, 2 ** 20, size=(3, K), endpoint=True).astype(np.float64)
    B = rng.integers(-2 ** 20, 2 ** 20, size=(K, 4), endpoint=True).astype(np.float64)
    C = oracle.ozaki_dgemm(A, B, S, S)
    exact = A.astype(object).dot(B.astype(object))
    assert np.array_equal(C.astype(object), exact)
    assert np.all(np.abs(exact.astype(float)) < 2.0 ** 53)


@pytest.mark.parametrize("S", [4, 6, 8])
def test_identity_returns_rounded_operand(S):
    """A = I: C_ij = b_ij rounded to the column's fixed-point grid (within 1 ulp)."""
    rng = np.random.default_rng(60 + S)
    n = 24
    B = wl.wide_normal(rng, (n, n), 20)
    C = oracle.ozaki_dgemm(np.eye(n), B, S, S)
    _, f, _ = oracle.split(B, S, by_columns=True)
    for j in range(n):
        unit = Fraction(2) ** (int(f[j]) - 8 * S + 1)
        for i in range(n):
            want = float(unit * round(Fraction(float(B[i, j])) / unit))
            assert abs(C[i, j] - want) <= np.spacing(abs(want)) if want else C[i, j] == 0


@pytest.mark.parametrize("S,G", [(4, 4), (5, 6), (6, 6), (7, 8), (8, 8), (4, 7)])
def test_within_apriori_bound(S, G):
    rng = np.random.default_rng(70 + S + G)
    for U in (10, 30):
        A = wl.wide_normal(rng, (12, 50), U)
        B = wl.wide_normal(rng, (50, 9), U)
        C = oracle.ozaki_dgemm(A, B, S, G)
        hi, lo = oracle.dgemm_dd(A, B)
        bound = oracle.ozaki_bound(A, B, S, G)
        err = np.abs((C - hi) - lo)
        assert np.all(err <= bound), float(np.max(err / bound))


def test_error_falls_about_256_per_slice():
    rng = np.random.default_rng(80)
    A = wl.wide_normal(rng, (64, 96), 10)
    B = wl.wide_normal(rng, (96, 48), 10)
    hi, lo = oracle.dgemm_dd(A, B)
    errs = [oracle.rel_frobenius(oracle.ozaki_dgemm(A, B, S, S), hi, lo) for S in range(3, 8)]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 30.0
    fp64 = oracle.rel_frobenius(oracle.dgemm_fp64(A, B), hi, lo)
    assert errs[-1] < 10 * fp64   # S = 7 reaches the FP64 level


@pytest.mark.parametrize("S", [4, 6, 8])
def test_invariances_bit_exact(S):
    rng = np.random.default_rng(90 + S)
    A = wl.wide_normal(rng, (10, 31), 20)
    B = wl.wide_normal(rng, (31, 7), 20)
    C = oracle.ozaki_dgemm(A, B, S)
    # power-of-two scaling of a row of A / a column of B scales the output exactly
    A2 = A.copy(); A2[3] *= 2.0 ** 37
    C2 = oracle.ozaki_dgemm(A2, B, S)
    assert np.array_equal(C2[3], C[3] * 2.0 ** 37) and np.array_equal(np.delete(C2, 3, 0), np.delete(C, 3, 0))
    B2 = B.copy(); B2[:, 5] *= 2.0 ** -41
    C3 = oracle.ozaki_dgemm(A, B2, S)
    assert np.array_equal(C3[:, 5], C[:, 5] * 2.0 ** -41)
    # a common permutation of the inner index leaves the output unchanged
    p = rng.permutation(31)
    assert np.array_equal(oracle.ozaki_dgemm(A[:, p], B[p], S), C)
    # transpose symmetry ozaki(B^T, A^T) = ozaki(A, B)^T
    assert np.array_equal(oracle.ozaki_dgemm(B.T.copy(), A.T.copy(), S), C.T)
    # row / column permutations commute
    pr, pc = rng.permutation(10), rng.permutation(7)
    assert np.array_equal(oracle.ozaki_dgemm(A[pr], B[:, pc], S), C[pr][:, pc])
    # transposed storage gives the same product
    assert np.array_equal(oracle.ozaki_dgemm(A.T.copy(), B, S, transa="T"), C)
    assert np.array_equal(oracle.ozaki_dgemm(A, B.T.copy(), S, transb="T"), C)


def test_degenerate_shapes_and_nan():
    rng = np.random.default_rng(3)
    Cin = rng.standard_normal((3, 4))
    out = oracle.ozaki_dgemm(np.zeros((3, 0)), np.zeros((0, 4)), 6, alpha=2.0, beta=0.5, C=Cin)
    assert np.array_equal(out, 0.5 * Cin)
    A = rng.standard_normal((3, 5))
    B = rng.standard_normal((5, 4))
    A[1, 2] = np.nan
    B[0, 3] = np.inf
    C = oracle.ozaki_dgemm(A, B, 6)
    assert np.isnan(C[1]).all() and np.isnan(C[:, 3]).all()
    ok = np.ones((3, 4), bool); ok[1] = False; ok[:, 3] = False
    ref = oracle.ozaki_dgemm(np.delete(A, 1, 0), np.delete(B, 3, 1), 6)
    assert np.array_equal(C[ok].reshape(2, 3), ref)
    z = oracle.ozaki_dgemm(np.zeros((2, 3)), rng.standard_normal((3, 2)), 5)
    assert np.all(z == 0)


# ---------------------------------------------------------------- H_eff . psi
def _kron_matvec(L, R, psi_j):
    H = sum(np.kron(L[k], R[k]) for k in range(L.shape[0]))
    return (H @ psi_j.ravel()).reshape(psi_j.shape)


def test_heff_dense_fp64_matches_kronecker_form():
    L, R, psi = wl.heff_dense(D=6, kop=3, phys=4, seed=1)
    sig = oracle.heff_dense(L, R, psi)
    for j in range(4):
        ref = _kron_matvec(L, R, psi[:, j, :])
        assert np.allclose(sig[:, j, :], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_heff_dense_exact_rational_tiny():
    L, R, psi = wl.heff_dense(D=3, kop=2, phys=2, U=6, seed=2)
    D, p = 3, 2
    for S in (0, 6):
        sig = oracle.heff_dense(L, R, psi, S=S)
        for j in range(p):
            T = [exact_matmul(L[k], psi[:, j, :]) for k in range(2)]
            for a in range(D):
                for b in range(D):
                    ex = sum(sum(T[k][a][c] * Fraction(float(R[k][b, c])) for c in range(D))
                             for k in range(2))
                    mag = sum(abs(float(L[k][a, x])) * abs(float(psi[x, j, c])) * abs(float(R[k][b, c]))
                              for k in range(2) for x in range(D) for c in range(D))
                    tol = 1e-13 if S == 0 else 2.0 ** (-8 * S + 10)
                    assert abs(float(Fraction(sig[a, j, b]) - ex)) <= tol * mag


@pytest.mark.parametrize("S", [0, 5])
def test_heff_dense_physical_index_independent(S):
    """sigma[:, j, :] depends on psi[:, j, :] only, with the same per-row and
    per-column exponents as a phys = 1 problem: bit-exact per slice j."""
    L, R, psi = wl.heff_dense(D=8, kop=3, phys=4, seed=3)
    sig = oracle.heff_dense(L, R, psi, S=S)
    for j in range(4):
        one = oracle.heff_dense(L, R, psi[:, j:j + 1, :].copy(), S=S)
        assert np.array_equal(one[:, 0, :], sig[:, j, :])


@pytest.mark.parametrize("S", [0, 6])
def test_heff_dense_rows_bit_exact(S):
    L, R, psi = wl.heff_dense(D=10, kop=3, phys=4, seed=4)
    full = oracle.heff_dense(L, R, psi, S=S)
    rows = [0, 7, 9]
    part = oracle.heff_dense_rows(L, R, psi, rows, S=S)
    assert np.array_equal(part, full[rows])


def test_heff_sparse_exact_rational_tiny():
    prob = wl.heff_sparse(n_sectors=5, n_triples=12, kop=3, median=3, sigma_log=0.3,
                          lo_hi=(2, 4), density=0.5, reach=1, U=4, seed=5)
    assert len(prob.triples) > 0
    for S in (0, 6):
        sig = oracle.heff_sparse(prob, S=S)
        exact = {b: None for b in prob.psi_blocks}
        mags = {}
        for (op, lo, li, ri, ro, al) in prob.triples:
            T = exact_matmul(prob.L[(op, lo, li)], prob.psi[(li, ri)])
            Rb = prob.R[(op, ro, ri)]
            blk = [[al * sum(T[a][c] * Fraction(float(Rb[b, c])) for c in range(len(T[0])))
                    for b in range(Rb.shape[0])] for a in range(len(T))]
            mag = np.abs(prob.L[(op, lo, li)]) @ np.abs(prob.psi[(li, ri)]) @ np.abs(Rb).T
            if exact[(lo, ro)] is None:
                exact[(lo, ro)] = blk
                mags[(lo, ro)] = mag
            else:
                exact[(lo, ro)] = [[x + y for x, y in zip(r1, r2)] for r1, r2 in zip(exact[(lo, ro)], blk)]
                mags[(lo, ro)] = mags[(lo, ro)] + mag
        tol = 1e-13 if S == 0 else 2.0 ** (-8 * S + 10)
        for b, blk in exact.items():
            if blk is None:
                assert np.all(sig[b] == 0)
                continue
            for a in range(len(blk)):
                for c in range(len(blk[0])):
                    assert abs(float(Fraction(sig[b][a, c]) - blk[a][c])) <= tol * mags[b][a, c]


# ---------------------------------------------------------------- Davidson
def _dense_H(prob):
    H = sum(np.kron(prob.L[k], prob.R[k]) for k in range(prob.L.shape[0]))
    return H + np.diag(prob.delta.ravel())


def test_davidson_brute_force_d16():
    prob = wl.davidson_problem(D=16, kop=32)
    H = _dense_H(prob)
    assert np.allclose(H, H.T)
    ev, evec = np.linalg.eigh(H)
    assert np.allclose(np.diag(H), prob.hdiag.ravel())
    mv = oracle.heff_matvec(prob.L, prob.R, prob.delta)
    theta, x, status, its, hist = oracle.davidson(mv, prob.hdiag, prob.x0, tol=1e-8)
    assert status == oracle.CONVERGED
    gap = ev[1] - ev[0]
    assert abs(theta - ev[0]) <= max(hist[-1] ** 2 / gap * 10, 1e-12) + 1e-10
    assert abs(theta - ev[0]) < 1e-10
    assert abs(abs(x @ evec[:, 0]) - 1) < 1e-10
    # the emulated matvec reaches the same energy far inside 1e-6 Ha
    mvS = oracle.heff_matvec(prob.L, prob.R, prob.delta, S=5)
    thS, _, stS, _, _ = oracle.davidson(mvS, prob.hdiag, prob.x0, tol=1e-8)
    assert stS == oracle.CONVERGED
    assert abs(thS - ev[0]) < 1e-6


def test_davidson_spectral_norm_scaling():
    prob = wl.davidson_problem(D=12, kop=8)
    H = _dense_H(prob) - np.diag(prob.delta.ravel())
    assert abs(np.linalg.norm(H, 2) - 10.0) < 0.05


def test_davidson_small_basis_restart_and_stagnation():
    prob = wl.davidson_problem(D=10, kop=6)
    H = _dense_H(prob)
    ev = np.linalg.eigvalsh(H)
    mv = oracle.heff_matvec(prob.L, prob.R, prob.delta)
    th, _, st, its, _ = oracle.davidson(mv, prob.hdiag, prob.x0, m_max=4, tol=1e-9)
    assert st == oracle.CONVERGED and abs(th - ev[0]) < 1e-9
    # an unreachable tolerance ends in stagnation, not an endless loop
    th, _, st, its, _ = oracle.davidson(mv, prob.hdiag, prob.x0, tol=1e-30, max_iter=200)
    assert st in (oracle.STAGNATED, oracle.MAX_ITER) and abs(th - ev[0]) < 1e-9


def test_lanczos_brute_force_d16():
    prob = wl.davidson_problem(D=16, kop=32)
    H = _dense_H(prob)
    ev, evec = np.linalg.eigh(H)
    mv = oracle.heff_matvec(prob.L, prob.R, prob.delta)
    theta, x, status, its, hist = oracle.lanczos(mv, prob.x0, m_max=32, tol=1e-8)
    assert status == oracle.CONVERGED
    assert abs(theta - ev[0]) < 1e-10
    assert abs(np.linalg.norm(x) - 1) < 1e-12
    assert abs(abs(x @ evec[:, 0]) - 1) < 1e-8
    # a small basis restarts from the Ritz vector and still converges
    th4, _, st4, its4, _ = oracle.lanczos(mv, prob.x0, m_max=4, tol=1e-8, max_iter=2000)
    assert st4 == oracle.CONVERGED and abs(th4 - ev[0]) < 1e-10 and its4 > its


def test_lanczos_ritz_values_of_the_krylov_space():
    """Without restart, step m returns the lowest Rayleigh-Ritz value of H on
    the Krylov space span(x0, H x0, ..., H^{m-1} x0), built here from the
    power basis and a QR factorisation, and its residual estimate is the true
    residual norm |H x - theta x| of the Ritz vector."""
    prob = wl.davidson_problem(D=8, kop=6)
    H = _dense_H(prob)
    x0 = np.asarray(prob.x0, dtype=np.float64).ravel()
    seen = []
    oracle.lanczos(lambda v: H @ v, x0, m_max=40, tol=0.0, max_iter=6,
                   trace=lambda it, th, rho, m: seen.append((th, rho, m)))
    assert [m for _, _, m in seen] == [1, 2, 3, 4, 5, 6]
    for m in range(1, 7):
        K = np.empty((x0.size, m))
        v = x0 / np.linalg.norm(x0)
        for j in range(m):
            K[:, j] = v
            v = H @ v
            v /= np.linalg.norm(v)
        Qk, _ = np.linalg.qr(K)
        w, y = np.linalg.eigh(Qk.T @ H @ Qk)
        th, rho, _ = seen[m - 1]
        assert abs(th - w[0]) < 1e-9 * abs(w[0])
        xr = Qk @ y[:, 0]
        assert abs(rho - np.linalg.norm(H @ xr - w[0] * xr)) < 1e-7 * np.linalg.norm(H, 2)


def test_lanczos_invariant_subspace_and_stagnation():
    # a start vector inside a 3-dimensional invariant subspace: the third step
    # finds beta = 0 and ends converged with the exact eigenvalue of the subspace
    d = np.array([-2.0, 1.0, 3.0, 5.0, 7.0, -9.0])
    x0 = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    th, x, st, its, _ = oracle.lanczos(lambda v: d * v, x0, m_max=10, tol=0.0)
    assert st == oracle.CONVERGED and its == 3 and abs(th + 2.0) < 1e-13
    assert np.allclose(np.abs(x), [1, 0, 0, 0, 0, 0], atol=1e-12)
    # tolerance 1e-30 with an exact matvec: after a restart from a Ritz vector
    # accurate to rounding, beta itself is at rounding level and counts as an
    # invariant subspace (converged)
    prob = wl.davidson_problem(D=10, kop=6)
    ev = np.linalg.eigvalsh(_dense_H(prob))
    mv = oracle.heff_matvec(prob.L, prob.R, prob.delta)
    th, _, st, its, _ = oracle.lanczos(mv, prob.x0, m_max=8, tol=1e-30, max_iter=300)
    assert st == oracle.CONVERGED and its < 100 and abs(th - ev[0]) < 1e-12
    # with a 3-slice matvec the estimate never reaches 1e-30 nor rounding level:
    # the iteration stagnates, at an energy within the matvec's error
    mv3 = oracle.heff_matvec(prob.L, prob.R, prob.delta, S=3)
    th, _, st, _, _ = oracle.lanczos(mv3, prob.x0, m_max=8, tol=1e-30, max_iter=300)
    assert st == oracle.STAGNATED and abs(th - ev[0]) < 1e-5


# ---- automatic slice count (the library's own rule; the paper gives none) --------
def test_auto_slices_keep_native_accuracy():
    """The chosen (S, G) gives an emulated product whose error against the
    double-double reference is within 1.5x of the plain FP64 product's, and
    no cheaper pair count does (the purpose of the rule)."""
    for U in (0, 10, 30):
        A, B = wl.gemm_pair(192, U=U, seed=4)
        hi, lo = oracle.dgemm_dd(A, B)
        e64 = oracle.rel_frobenius(oracle.dgemm_fp64(A, B), hi, lo)
        S, G = oracle.choose_slices(A, B)
        err = oracle.rel_frobenius(oracle.ozaki_dgemm(A, B, S, G), hi, lo)
        assert err <= 1.5 * e64, (U, S, G, err, e64)
        # the next cheaper candidate misses native accuracy (the choice is not wasteful)
        cheaper = [(s, g) for s in range(2, 9) for g in (s, s + 1)
                   if oracle.pair_count(s, g) < oracle.pair_count(S, G)]
        best = max(cheaper, key=lambda sg: oracle.pair_count(*sg))
        err_c = oracle.rel_frobenius(oracle.ozaki_dgemm(A, B, *best), hi, lo)
        assert err_c > 0.5 * e64, (U, best, err_c, e64)


def test_error_model_tracks_measured_errors():
    """Measured / predicted emulated error within [0.3, 3] where the emulation
    error is well above the double-double floor."""
    A, B = wl.gemm_pair(256, U=10, seed=5)
    hi, lo = oracle.dgemm_dd(A, B)
    ra, rb = oracle.rho(A), oracle.rho(B, by_columns=True)
    for (S, G) in [(4, 4), (4, 5), (5, 5), (6, 6), (6, 7), (7, 7)]:
        err = oracle.rel_frobenius(oracle.ozaki_dgemm(A, B, S, G), hi, lo)
        pred = oracle.predicted_emulated_error(S, G, ra, rb)
        assert 0.3 <= err / pred <= 3.0, (S, G, err, pred)
    e64 = oracle.rel_frobenius(oracle.dgemm_fp64(A, B), hi, lo)
    assert 0.3 <= e64 / oracle.predicted_native_error(256) <= 3.0


def test_rho_closed_forms():
    """rho of a constant matrix is 1 * 2^e / |c| (e the bumped exponent);
    zero groups are left out; NaN marks a non-finite group."""
    c = 0.75
    X = np.full((5, 64), c)
    e = 0  # 0.75 = 0.75 * 2^0, mantissa <= 127/128 -> no bump
    assert oracle.rho(X) == pytest.approx(2.0 ** e / c, rel=1e-15)
    X[2] = 0.0
    assert oracle.rho(X) == pytest.approx(2.0 ** e / c, rel=1e-15)
    X[3, 7] = np.nan
    assert np.isnan(oracle.rho(X))
    assert oracle.choose_slices(X, np.ones((64, 3))) == (7, 7)
    assert oracle.choose_slices(np.zeros((4, 8)), np.ones((8, 4))) == (2, 2)


# ---- truncation and renormalisation ------------------------------------------
def test_truncate_planted_spectrum():
    """rho = psi psi^T of a planted Schmidt decomposition: its eigenvalues are
    the squared Schmidt values, the discarded weight their tail sum and the
    kept eigenvectors span the planted left vectors (closed forms of the
    construction)."""
    t = wl.two_site_psi(96, 80, tau=6.0, seed=3)
    s2 = t.schmidt ** 2
    for D in (1, 20, 80):
        U, w, dw = oracle.truncate(t.psi, D)
        assert np.max(np.abs(w - s2[:D])) < 1e-15
        assert abs(dw - s2[D:].sum()) < 1e-14
        sv = np.linalg.svd(t.left[:, :D].T @ U, compute_uv=False)
        assert np.all(np.abs(sv - 1) < 1e-10)
    # emulated rho: the eigenvalue error follows the slice count
    for S, tol in ((7, 1e-15), (4, 1e-8), (3, 1e-6)):
        U, w, dw = oracle.truncate(t.psi, 20, S=S)
        assert np.max(np.abs(w - s2[:20])) < tol, S


def test_renormalize_selector_is_exact():
    """U = columns idx of the identity: U^T O U = O[idx][:, idx] exactly, for
    FP64 and every slice count (integer entries below 2^10 fit any slicing);
    O is not symmetric, so a transposed operand fails."""
    rng = np.random.default_rng(5)
    n, D = 70, 23
    ops = [rng.integers(-1000, 1001, size=(n, n)).astype(np.float64) for _ in range(3)]
    idx = np.sort(rng.choice(n, D, replace=False))[::-1]
    U = np.zeros((n, D))
    U[idx, np.arange(D)] = 1.0
    for S in (0, 2, 5, 8):
        out = oracle.renormalize(U, ops, S=S)
        for O, Op in zip(ops, out):
            assert np.array_equal(Op, O[np.ix_(idx, idx)]), S


def test_renormalize_orthogonal_similarity():
    """A full orthogonal U keeps the spectrum of a symmetric operator."""
    ops = wl.block_operators(60, 2, seed=6)
    U = np.linalg.qr(np.random.default_rng(7).standard_normal((60, 60)))[0]
    for O, Op in zip(ops, oracle.renormalize(U, ops)):
        assert np.max(np.abs(np.linalg.eigvalsh(Op) - np.linalg.eigvalsh(O))) < 1e-13
