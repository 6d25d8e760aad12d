"""GPU parity of the two-site H_eff.psi plans against the CPU oracle.

Emulated plans must match the oracle bit for bit (every sigma tile sums its
triples in list order with the same FP64 steps); native FP64 plans are held
to a bound derived from gamma_K of the two chained products.
"""
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


def dense_plan(ozaki, ctx, torch, L, R, psi, S, G=0, diag=None):
    layout, Lf, Rf, pf, triples = wl.flatten_dense(L, R, psi)
    dL, dR = dev(torch, Lf), dev(torch, Rf)
    dd = dev(torch, diag.ravel()) if diag is not None else None
    plan = ozaki.HeffPlan(ctx, layout, dL, dR, triples, diag=dd, slices=S, ndiag=G)
    return plan, dev(torch, pf), (dL, dR, dd)


def fp64_bound(L, R, psi, K1, K2):
    """Componentwise bound for two chained FP64 GEMM sums, summed over k."""
    u = 2.0 ** -53
    g = (K1 + K2 + 2) * u / (1 - (K1 + K2 + 2) * u)
    D, p, D2 = psi.shape
    aP = np.abs(psi).reshape(D, p * D2)
    tot = np.zeros((D * p, D2))
    for k in range(L.shape[0]):
        tot += (np.abs(L[k]) @ aP).reshape(D * p, D2) @ np.abs(R[k]).T
    return g * tot.reshape(D, p, D2) * (1 + L.shape[0] * u) + 1e-300


@pytest.mark.parametrize("S,G", [(6, 6), (4, 5), (8, 9), (7, 13)])
def test_dense_bitexact(oz, S, G):
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=70, kop=3, phys=4, seed=S)
    plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, S, G)
    sig = plan.apply(dpsi).cpu().numpy().reshape(psi.shape)
    ref = oracle.heff_dense(L, R, psi, S=S, G=G)
    assert_bitexact(sig, ref, "dense S=%d G=%d" % (S, G))
    assert plan.flops == 64 * 70 ** 3 * 3 * 4 / 16


def test_dense_phys16_with_diagonal(oz):
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=40, kop=2, phys=16, seed=3)
    diag = np.random.default_rng(4).standard_normal(psi.shape)
    plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 6, 0, diag=diag)
    sig = plan.apply(dpsi).cpu().numpy().reshape(psi.shape)
    assert_bitexact(sig, oracle.heff_dense(L, R, psi, S=6, diag=diag), "phys16 diag")
    # a second apply on the same plan gives the same bits (no state carried over)
    sig2 = plan.apply(dpsi).cpu().numpy().reshape(psi.shape)
    assert_bitexact(sig2, sig, "repeat")


def test_dense_fp64_within_bound(oz):
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=90, kop=3, phys=4, seed=5)
    plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 0)
    sig = plan.apply(dpsi).cpu().numpy().reshape(psi.shape)
    ref = oracle.heff_dense(L, R, psi, S=0)
    assert np.all(np.abs(sig - ref) <= 2 * fp64_bound(L, R, psi, 90, 90))


def test_dense_fp64_large_tiles_within_bound(oz):
    """FP64 plan with enough first-product tiles for the 128 x 128 tiles and
    a second product on 64 x 64 tiles; sampled rows against the oracle's FP64
    rows, within the chained gamma bound."""
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=512, kop=8, phys=4, seed=7)
    plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 0)
    sig = plan.apply(dpsi).reshape(psi.shape).cpu().numpy()
    rows = [0, 255, 511]
    ref = oracle.heff_dense_rows(L, R, psi, rows, S=0)
    bound = fp64_bound(L, R, psi, 512, 512)[rows]
    assert np.all(np.abs(sig[rows] - ref) <= 2 * bound)


def test_dense_d256_full(oz):
    """D = 256, phys 16: several tiles in every direction, all rows checked."""
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=256, kop=4, phys=16, seed=0)
    plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 6)
    sig = plan.apply(dpsi).cpu().numpy().reshape(psi.shape)
    assert_bitexact(sig, oracle.heff_dense(L, R, psi, S=6), "D=256")


@pytest.mark.parametrize("case", ["phys3_d96", "nonfinite", "nan_chunk2", "inf_chunk3", "chunks_long",
                                  "subnormal_T", "fallback_d70"])
def test_T_exponents_from_first_phase(oz, case):
    """T's row exponents come from the first phase's epilogue (exponent-code
    maxima combined with atomic max) when every T row takes whole 32-column
    groups (phys 1, or right dimensions that are multiples of 32), else from
    a pass over T.  Both give the oracle's bits, also with NaN / Inf inputs,
    zero rows and subnormal T."""
    ozaki, ctx, torch = oz
    D, phys = (70, 4) if case == "fallback_d70" else (300, 1) if case.endswith(("2", "3", "long")) else (96, 3)
    L, R, psi = wl.heff_dense(D=D, kop=2, phys=phys, seed=7)
    if case == "nonfinite":
        psi[5, 1, 7] = np.nan
        psi[10, 0, 3] = np.inf
        L[1][3, :] = 0.0
    # psi's column exponents come from row chunks of 128 (300 rows: three chunks);
    # with phys 1 a non-finite psi entry makes a whole column of T, hence every
    # sigma entry, NaN
    if case == "nan_chunk2":
        psi[140, 0, 9] = np.nan
    if case == "inf_chunk3":
        psi[290, 0, 33] = -np.inf
    if case == "chunks_long":
        psi[:, 0, 50] = 0.0
        psi[:, 0, 60] *= 1e-300
        psi[260, 0, 60] = 5e-300
        psi[250, 0, 70] = 1e3
    if case == "subnormal_T":
        psi = psi * 2.0 ** -1000
        L = L * 2.0 ** -60
    ctx.flags()
    plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 5)
    sig = plan.apply(dpsi).cpu().numpy().reshape(psi.shape)
    ref = oracle.heff_dense(L, R, psi, S=5)
    assert_bitexact(sig, ref, case)
    if case == "nonfinite":
        assert np.isnan(ref).any() and not np.isnan(ref).all()
    if case in ("nan_chunk2", "inf_chunk3"):
        assert np.isnan(ref).all()
    if case in ("nonfinite", "nan_chunk2", "inf_chunk3"):
        assert ctx.flags() & 1
    if case == "chunks_long":
        assert not np.isnan(ref).any()
    if case == "subnormal_T":
        T0 = L[0] @ psi.reshape(D, -1)
        assert np.abs(T0).max() < 2.0 ** -1022


def test_dense_d2048_sampled_rows(oz):
    """D = 2048, phys 16 (the benchmark's shape, fewer operator pairs): rows
    alpha' computed alone by the oracle, whole second products included."""
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=2048, kop=4, phys=16, seed=0)
    plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 6)
    sig = plan.apply(dpsi).reshape(2048, 16, 2048)
    rows = [5, 2047]
    got = sig[rows].cpu().numpy()
    ref = oracle.heff_dense_rows(L, R, psi, rows, S=6)
    assert_bitexact(got, ref, "D=2048 rows")


@pytest.mark.timeout(1200)
def test_dense_benchmark_shape_sampled_rows(oz):
    """The benchmark's dense workload itself: D = 2048, phys 16, Kop = 64,
    S = 6 (a 64-term ordered sigma accumulation per tile), with the plan's
    timed launch choice.  Two rows alpha' (all j, beta') from the oracle."""
    ozaki, ctx, torch = oz
    print("[test] dense D=2048 Kop=64 phys=16 S=6: generating", flush=True)
    L, R, psi = wl.heff_dense(D=2048, kop=64, phys=16, seed=0)
    plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 6)
    print("[test] plan variants %s launches %s; applying" % (plan.variants, plan.launches), flush=True)
    sig = plan.apply(dpsi).reshape(2048, 16, 2048)
    rows = [1037, 2047]
    got = sig[rows].cpu().numpy()
    plan.close()
    del sig, dpsi, keep
    torch.cuda.empty_cache()
    print("[test] oracle rows %s" % rows, flush=True)
    ref = oracle.heff_dense_rows(L, R, psi, rows, S=6)
    assert_bitexact(got, ref, "D=2048 Kop=64 rows")


def small_sparse(seed):
    return wl.heff_sparse(n_sectors=9, n_triples=80, kop=5, median=60, sigma_log=0.7,
                          lo_hi=(7, 150), density=0.35, reach=2, U=12, seed=seed)


def sparse_plan(ozaki, ctx, torch, prob, S, G=0):
    layout, Lf, Rf, pf, triples = wl.flatten_sparse(prob)
    dL, dR = dev(torch, Lf), dev(torch, Rf)
    plan = ozaki.HeffPlan(ctx, layout, dL, dR, triples, slices=S, ndiag=G)
    return plan, dev(torch, pf), (dL, dR)


@pytest.mark.parametrize("S,G", [(6, 6), (5, 6), (8, 8)])
def test_sparse_bitexact(oz, S, G):
    ozaki, ctx, torch = oz
    prob = small_sparse(10 + S)
    plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, S, G)
    sig = wl.unflatten_sparse(prob, plan.apply(dpsi).cpu().numpy())
    ref = oracle.heff_sparse(prob, S=S, G=G)
    for b in prob.psi_blocks:
        assert_bitexact(sig[b], ref[b], "block %s" % (b,))


def test_sparse_fp64(oz):
    ozaki, ctx, torch = oz
    prob = small_sparse(3)
    plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, 0)
    sig = wl.unflatten_sparse(prob, plan.apply(dpsi).cpu().numpy())
    ref = oracle.heff_sparse(prob, S=0)
    mag = {b: np.zeros_like(ref[b]) for b in prob.psi_blocks}
    for (op, lo, li, ri, ro, al) in prob.triples:
        mag[(lo, ro)] += abs(al) * (np.abs(prob.L[(op, lo, li)]) @ np.abs(prob.psi[(li, ri)])) @ np.abs(prob.R[(op, ro, ri)]).T
    u = 2.0 ** -53
    for b in prob.psi_blocks:
        K = 2 * int(prob.dims.max()) + 2 + len(prob.triples)
        assert np.all(np.abs(sig[b] - ref[b]) <= 2 * K * u * mag[b] + 1e-300), b


@pytest.mark.parametrize("launch", [-1, 0, 100000, -2, -3])
def test_sparse_full_size_sampled_blocks(oz, launch):
    """The 40-sector, 2000-triple batch; sigma blocks depend only on their own
    triples, so the oracle recomputes a few blocks alone: the three with the
    fewest triples and the three with the most (the longest ordered
    accumulation chains).  Timed launch choice, one workgroup per tile, the
    streamed kernel on every CU, the resident first phase on the 64 x 64
    tiles (every workgroup walks some 65 tiles of 1 to 47 K blocks) and the
    paired-term second phase (terms of different lengths paired), the last
    two also against the per-tile launch's whole sigma."""
    ozaki, ctx, torch = oz
    prob = wl.heff_sparse()
    ctx.set_heff_launch(launch)
    if launch < -1:
        ctx.set_variant(6, 0, 0)
    try:
        plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, 6)
        if launch < -1:
            ctx.set_heff_launch(0)
            plan0, _, keep0 = sparse_plan(ozaki, ctx, torch, prob, 6)
            assert plan0.launches == (0, 0)
    finally:
        ctx.set_heff_launch(-1)
        ctx.set_variant(6, 0, -1)
    if launch >= 0:
        assert plan.launches == ((1, 1) if launch else (0, 0))
    elif launch == ozaki.OZ_HEFF_LAUNCH_RESIDENT:
        assert plan.launches == (2, 0) and plan.phase(0)[2] == launch
    elif launch == ozaki.OZ_HEFF_LAUNCH_PAIRED_TERMS:
        assert plan.launches == (0, 3) and plan.phase(1)[2] == launch
    out = plan.apply(dpsi)
    if launch < -1:
        assert torch.equal(out, plan0.apply(dpsi))
    sig = wl.unflatten_sparse(prob, out.cpu().numpy())
    counts = {}
    for t in prob.triples:
        counts[(t[1], t[4])] = counts.get((t[1], t[4]), 0) + 1
    order = sorted(counts, key=lambda b: (counts[b], b))
    pick = order[:3] + order[-3:]
    assert counts[pick[-1]] >= 20
    for b in pick:
        sub = wl.HeffSparse(dims=prob.dims, psi_blocks=[b], psi=prob.psi, L=prob.L, R=prob.R,
                            triples=[t for t in prob.triples if (t[1], t[4]) == b])
        ref = oracle.heff_sparse(sub, S=6)
        assert_bitexact(sig[b], ref[b], "cfg4 block %s" % (b,))
    # sigma blocks no triple reaches are zero
    for b in prob.psi_blocks:
        if b not in counts:
            assert np.all(sig[b] == 0)


@pytest.mark.parametrize("S", [6, 0])
def test_chunked_plans_match(oz, S):
    """A small T budget cuts the triple list into chunks (first products
    recomputed where two chunks use them, sigma tiles continuing from their
    stored values): dense and block-sparse results are the oracle's bits
    (emulated) or the unchunked plan's bits (FP64), with graphs replayed."""
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=96, kop=7, phys=4, seed=17)
    prob = small_sparse(23)
    # the same first product used by two far-apart triples lands in two chunks
    tri = list(prob.triples)
    prob.triples = tri + [tri[3], tri[len(tri) // 2]]
    try:
        res = {}
        for budget in (0, 1):   # 1 byte: one first product per chunk
            ctx.set_heff_budget(budget)
            plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, S)
            assert (plan.chunks == 1) if budget == 0 else (plan.chunks == 7)
            a = plan.apply(dpsi).cpu().numpy()
            b = plan.apply(dpsi).cpu().numpy()
            assert_bitexact(a, b, "dense replay")
            splan, spsi, skeep = sparse_plan(ozaki, ctx, torch, prob, S)
            if budget:
                assert splan.chunks > 10
            sa = splan.apply(spsi).cpu().numpy()
            res[budget] = (a, sa, plan.bytes[1], splan.bytes[1])
        assert res[1][2] < res[0][2]
        assert_bitexact(res[1][0], res[0][0], "dense chunked vs one chunk")
        assert_bitexact(res[1][1], res[0][1], "sparse chunked vs one chunk")
        if S:
            assert_bitexact(res[1][0].reshape(psi.shape), oracle.heff_dense(L, R, psi, S=S), "dense oracle")
            ref = oracle.heff_sparse(prob, S=S)
            sig = wl.unflatten_sparse(prob, res[1][1])
            for blk in prob.psi_blocks:
                assert_bitexact(sig[blk], ref[blk], "sparse oracle block %s" % (blk,))
    finally:
        ctx.set_heff_budget(0)


def test_fixed_phase_choice(oz):
    """A plan with both phases fixed to a timed plan's choice reports that
    choice and gives the same bits; an unbuilt variant is rejected."""
    ozaki, ctx, torch = oz
    prob = small_sparse(29)
    plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, 6)
    want = (plan.phase(0), plan.phase(1))
    ref = plan.apply(dpsi).cpu().numpy()
    try:
        for ph in (0, 1):
            ctx.set_heff_phase(ph, *want[ph])
        plan2, _, keep2 = sparse_plan(ozaki, ctx, torch, prob, 6)
        assert (plan2.phase(0), plan2.phase(1)) == want
        assert_bitexact(plan2.apply(dpsi).cpu().numpy(), ref, "fixed phases")
        ctx.set_heff_phase(0, 2, 0, 0)   # 128 x 128 tiles are not built at G = 6
        with pytest.raises(ozaki.OzakiError):
            sparse_plan(ozaki, ctx, torch, prob, 6)
        with pytest.raises(ozaki.OzakiError):
            ctx.set_heff_phase(2, 0, 0, 0)
    finally:
        ctx.set_heff_phase(0, -1)
        ctx.set_heff_phase(1, -1)


@pytest.mark.parametrize("order", [0, 1, 2])
def test_tile_orders_bitexact(oz, order):
    """Every tile order (XCD parts, longest first, whole outputs per XCD),
    per tile, streamed and resident: the oracle's bits (the order moves
    tiles between workgroups, never the arithmetic of one)."""
    ozaki, ctx, torch = oz
    prob = small_sparse(31)
    ref = oracle.heff_sparse(prob, S=6)
    res = ozaki.OZ_HEFF_LAUNCH_RESIDENT
    try:
        for (vl, ll), (vr, lr) in [((3, 0), (4, 0)), ((0, 7), (3, 0)), ((4, 0), (0, 0)), ((0, res), (0, 0)),
                                   ((4, res), (3, 0))]:
            ctx.set_heff_phase(0, vl, order, ll)
            ctx.set_heff_phase(1, vr, order, lr)
            plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, 6)
            assert plan.phase(0) == (vl, order, ll) and plan.phase(1) == (vr, order, lr)
            sig = wl.unflatten_sparse(prob, plan.apply(dpsi).cpu().numpy())
            for b in prob.psi_blocks:
                assert_bitexact(sig[b], ref[b], "order %d L %d R %d block %s" % (order, vl, vr, b))
    finally:
        ctx.set_heff_phase(0, -1)
        ctx.set_heff_phase(1, -1)


def test_plan_argument_errors(oz):
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=8, kop=2, phys=1, seed=0)
    layout, Lf, Rf, pf, triples = wl.flatten_dense(L, R, psi)
    dL, dR = dev(torch, Lf), dev(torch, Rf)
    with pytest.raises(ozaki.OzakiError):
        ozaki.HeffPlan(ctx, layout, dL, dR, [(5, 0, 0, 0, 0, 1.0)], slices=6)   # no operator 5
    with pytest.raises(ozaki.OzakiError):
        ozaki.HeffPlan(ctx, layout, dL, dR, triples, slices=9)
    bad = dict(layout, psi_offset=[0, 10], psi_lr=[0, 0, 0, 0])
    with pytest.raises(ozaki.OzakiError):
        ozaki.HeffPlan(ctx, bad, dL, dR, triples, slices=6)


def test_no_triples(oz):
    """A plan with an empty triple list: sigma is exactly zero, or exactly
    diag * psi with a diagonal term (the product added to +0), for FP64 and
    emulated plans, graph replay on and off."""
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=24, kop=2, phys=4, seed=7)
    layout, Lf, Rf, pf, _ = wl.flatten_dense(L, R, psi)
    dL, dR, dpsi = dev(torch, Lf), dev(torch, Rf), dev(torch, pf)
    diag = np.random.default_rng(8).standard_normal(pf.size)
    for S in (0, 4, 6, 8):
        for d in (None, diag):
            plan = ozaki.HeffPlan(ctx, layout, dL, dR, [], diag=None if d is None else dev(torch, d), slices=S)
            want = np.zeros(pf.size) if d is None else d * pf.ravel()
            for graphs in (True, False):
                plan.set_graphs(graphs)
                assert_bitexact(plan.apply(dpsi).cpu().numpy(), want, "no triples S=%d diag %s" % (S, d is not None))
            plan.close()


def test_apply_argument_errors(oz):
    """psi and sigma whose ranges intersect are refused by the library (equal
    or shifted by one element, either way round); a sigma of the wrong size,
    type or layout by the binding; the plan still applies correctly after."""
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=8, kop=2, phys=1, seed=0)
    plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 6)
    n = plan.n
    buf = torch.zeros(2 * n + 1, dtype=torch.float64, device="cuda")
    buf[:n] = dpsi
    for a, b in [(0, 0), (0, 1), (1, 0), (0, n - 1)]:
        with pytest.raises(ozaki.OzakiError):
            plan.apply(buf[a:a + n], buf[b:b + n])
    with pytest.raises(ValueError):
        plan.apply(dpsi, torch.empty(n - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        plan.apply(dpsi, torch.empty(2 * n, dtype=torch.float64, device="cuda")[::2])
    with pytest.raises(TypeError):
        plan.apply(dpsi, torch.empty(n, dtype=torch.float32, device="cuda"))
    got = plan.apply(buf[:n], buf[n:2 * n]).cpu().numpy().reshape(psi.shape)   # adjacent ranges are fine
    assert_bitexact(got, oracle.heff_dense(L, R, psi, S=6), "after the refused calls")


def test_plan_variants_bitexact(oz):
    """Each fixed tile variant and the autotuned choice give the oracle's bits."""
    ozaki, ctx, torch = oz
    prob = small_sparse(21)
    ref = oracle.heff_sparse(prob, S=6)
    try:
        for (v, tm, tn) in ozaki.pair_variants(6):
            ctx.set_variant(6, 0, v)
            plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, 6)
            assert plan.variants == (v, v)
            sig = wl.unflatten_sparse(prob, plan.apply(dpsi).cpu().numpy())
            for b in prob.psi_blocks:
                assert_bitexact(sig[b], ref[b], "variant %d block %s" % (v, b))
    finally:
        ctx.set_variant(6, 0, -1)
    plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, 6)
    built = [x[0] for x in ozaki.pair_variants(6)]
    assert plan.variants[0] in built and plan.variants[1] in built


@pytest.mark.parametrize("S,G,seed", [(6, 6, 76), (4, 4, 84), (5, 6, 82)])
def test_accumulating_many_short_terms(oz, S, G, seed):
    """The accumulating phase on the 8-wave tiles (three-stage ring) with
    sectors of 1 to 100 states (terms of 1 to 4 K blocks) and about ten
    terms per sigma block, one workgroup per tile, in one chunk and in
    chunks that continue a tile's sums: the oracle's bits."""
    ozaki, ctx, torch = oz
    prob = wl.heff_sparse(n_sectors=8, n_triples=400, kop=8, median=30, sigma_log=1.0,
                          lo_hi=(1, 100), density=0.6, reach=7, U=8, seed=seed)
    assert prob.dims.min() <= 8 and prob.dims.max() > 64
    ref = oracle.heff_sparse(prob, S=S, G=G)
    ctx.set_heff_launch(0)
    try:
        for v in (3, 4):
            ctx.set_variant(S, G, v)
            for budget in (0, 1):
                ctx.set_heff_budget(budget)
                plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, S, G)
                assert plan.variants == (v, v) and plan.launches == (0, 0)
                assert (plan.chunks > 1) == (budget == 1)
                sig = wl.unflatten_sparse(prob, plan.apply(dpsi).cpu().numpy())
                for b in prob.psi_blocks:
                    assert_bitexact(sig[b], ref[b], "variant %d budget %d block %s" % (v, budget, b))
    finally:
        ctx.set_heff_budget(0)
        ctx.set_variant(S, G, -1)
        ctx.set_heff_launch(-1)


@pytest.mark.parametrize("cus", [1, 3, 100000])
def test_streamed_launch_bitexact(oz, cus):
    """The streamed kernel (resident workgroups walk the tile list; the first
    K block of the next tile or term is loaded during the last block of the
    current one) gives the oracle's bits.  On 1 or 3 compute units every
    workgroup walks many tiles and terms, with odd and even block counts."""
    ozaki, ctx, torch = oz
    ctx.set_heff_launch(cus)
    try:
        for S, G in [(6, 6), (7, 7), (5, 6), (3, 5), (8, 15)]:
            L, R, psi = wl.heff_dense(D=70, kop=3, phys=4, seed=40 + S)
            plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, S, G)
            assert plan.launches == (1, 1)
            sig = plan.apply(dpsi).cpu().numpy().reshape(psi.shape)
            assert_bitexact(sig, oracle.heff_dense(L, R, psi, S=S, G=G), "dense S=%d G=%d" % (S, G))
            prob = small_sparse(50 + S)
            plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, S, G)
            assert plan.launches == (1, 1)
            sig = wl.unflatten_sparse(prob, plan.apply(dpsi).cpu().numpy())
            ref = oracle.heff_sparse(prob, S=S, G=G)
            for b in prob.psi_blocks:
                assert_bitexact(sig[b], ref[b], "sparse S=%d G=%d block %s" % (S, G, b))
        prob = small_sparse(61)
        ref = oracle.heff_sparse(prob, S=6)
        for (v, tm, tn) in ozaki.pair_variants(6):
            ctx.set_variant(6, 0, v)
            plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, 6)
            assert plan.variants == (v, v) and plan.launches == (1, 1)
            sig = wl.unflatten_sparse(prob, plan.apply(dpsi).cpu().numpy())
            for b in prob.psi_blocks:
                assert_bitexact(sig[b], ref[b], "streamed variant %d block %s" % (v, b))
    finally:
        ctx.set_heff_launch(-1)
        ctx.set_variant(6, 0, -1)


@pytest.mark.parametrize("cus", [1, 100000])
def test_streamed_tiny_sectors(oz, cus):
    """Sectors of 1 to 40 states (single-K-block items, tile lists shorter
    than the XCD count, so fewer than 8 queues) through the streamed kernel
    and the producer-side exponents: the oracle's bits."""
    ozaki, ctx, torch = oz
    prob = wl.heff_sparse(n_sectors=6, n_triples=30, kop=3, median=6, sigma_log=1.2,
                          lo_hi=(1, 40), density=0.5, reach=2, U=8, seed=3)
    assert prob.dims.min() <= 2
    ctx.set_heff_launch(cus)
    try:
        for S, G in [(6, 6), (3, 5)]:
            plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, S, G)
            assert plan.launches == (1, 1)
            sig = wl.unflatten_sparse(prob, plan.apply(dpsi).cpu().numpy())
            ref = oracle.heff_sparse(prob, S=S, G=G)
            for b in prob.psi_blocks:
                assert_bitexact(sig[b], ref[b], "tiny S=%d block %s" % (S, b))
    finally:
        ctx.set_heff_launch(-1)


@pytest.mark.parametrize("S,G", [(6, 6), (5, 6), (3, 5), (4, 4), (2, 3), (7, 7), (8, 8)])
def test_resident_launch_bitexact(oz, S, G):
    """The resident first phase (a grid that fits at once, each workgroup
    streaming the K blocks of its scheduled tiles through one ring, the next
    tile's first blocks loading during the current tile's last blocks and
    epilogue) for every tile variant it is built for: the oracle's bits on a
    dense problem, a sparse one and one of 1- to 40-state sectors (tiles of
    one K block, so a tile's successors fill the ring behind it), and the
    per-tile launch's bits on all of them."""
    ozaki, ctx, torch = oz
    res = ozaki.OZ_HEFF_LAUNCH_RESIDENT
    L, R, psi = wl.heff_dense(D=70, kop=3, phys=4, seed=70 + S)
    ref_d = oracle.heff_dense(L, R, psi, S=S, G=G)
    probs = [small_sparse(80 + S),
             wl.heff_sparse(n_sectors=6, n_triples=30, kop=3, median=6, sigma_log=1.2, lo_hi=(1, 40), density=0.5,
                            reach=2, U=8, seed=4)]
    refs = [oracle.heff_sparse(p, S=S, G=G) for p in probs]
    kinds = set()
    try:
        for (v, tm, tn) in ozaki.pair_variants(S, G):
            ctx.set_variant(S, G, v)
            ctx.set_heff_launch(res)
            plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, S, G)
            assert plan.variants == (v, v) and plan.launches[0] in (0, 2) and plan.launches[1] == 0
            kinds.add(plan.launches[0])
            out = plan.apply(dpsi)
            assert_bitexact(out.cpu().numpy().reshape(psi.shape), ref_d, "dense variant %d" % v)
            ctx.set_heff_launch(0)
            plan0, _, keep0 = dense_plan(ozaki, ctx, torch, L, R, psi, S, G)
            assert torch.equal(out, plan0.apply(dpsi))
            for prob, ref in zip(probs, refs):
                ctx.set_heff_launch(res)
                # one chunk, and chunks with a schedule each that continue the sums
                for budget in (0, 1):
                    ctx.set_heff_budget(budget)
                    plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, S, G)
                    assert plan.launches[0] in (0, 2) and plan.launches[1] == 0
                    assert (plan.chunks > 1) == (budget == 1)
                    sig = wl.unflatten_sparse(prob, plan.apply(dpsi).cpu().numpy())
                    for b in prob.psi_blocks:
                        assert_bitexact(sig[b], ref[b], "sparse variant %d budget %d block %s" % (v, budget, b))
                ctx.set_heff_budget(0)
    finally:
        ctx.set_heff_budget(0)
        ctx.set_heff_launch(-1)
        ctx.set_variant(S, G, -1)
    # built for the 8-wave tiles with G <= 8, and for the 64 x 64 tile from S = 3, G = 5 to S = 6
    assert 2 in kinds


@pytest.mark.parametrize("S,G", [(6, 6), (5, 6), (4, 4), (3, 5), (2, 3), (6, 7)])
def test_paired_terms_bitexact(oz, S, G):
    """The paired-term second phase (eight waves per 64 x 64 tile, two
    groups with a ring each taking the terms two at a time, their FP64 values
    added in term order through LDS): the oracle's bits on a dense problem
    with an odd number of terms per tile (the last round has one term), a
    sparse one whose paired terms differ in length (the shorter group's
    steps load and multiply nothing) and one of 1- to 40-state sectors, in
    one chunk and in chunks that continue the sums; and the per-tile
    launch's bits."""
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=70, kop=3, phys=4, seed=90 + S)
    ref_d = oracle.heff_dense(L, R, psi, S=S, G=G)
    probs = [small_sparse(95 + S),
             wl.heff_sparse(n_sectors=6, n_triples=30, kop=3, median=6, sigma_log=1.2, lo_hi=(1, 40), density=0.5,
                            reach=2, U=8, seed=5)]
    refs = [oracle.heff_sparse(p, S=S, G=G) for p in probs]
    try:
        ctx.set_variant(S, G, 0)
        for budget in (0, 1):
            ctx.set_heff_budget(budget)
            ctx.set_heff_launch(ozaki.OZ_HEFF_LAUNCH_PAIRED_TERMS)
            plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, S, G)
            assert plan.launches == (0, 3) and (plan.chunks > 1) == (budget == 1)
            out = plan.apply(dpsi)
            assert_bitexact(out.cpu().numpy().reshape(psi.shape), ref_d, "dense budget %d" % budget)
            ctx.set_heff_launch(0)
            plan0, _, keep0 = dense_plan(ozaki, ctx, torch, L, R, psi, S, G)
            assert torch.equal(out, plan0.apply(dpsi))
            for prob, ref in zip(probs, refs):
                ctx.set_heff_launch(ozaki.OZ_HEFF_LAUNCH_PAIRED_TERMS)
                plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, S, G)
                assert plan.launches == (0, 3)
                sig = wl.unflatten_sparse(prob, plan.apply(dpsi).cpu().numpy())
                for b in prob.psi_blocks:
                    assert_bitexact(sig[b], ref[b], "sparse budget %d block %s" % (budget, b))
    finally:
        ctx.set_heff_budget(0)
        ctx.set_heff_launch(-1)
        ctx.set_variant(S, G, -1)


@pytest.mark.parametrize("seed", range(6))
def test_random_sparse_every_launch(oz, seed):
    """Seeded random block-sparse problems (5 to 9 sectors of 1 to 200
    states, so tiles of one K block, edges inside a 32-block and paired terms
    of unequal length all occur) under every launch of the grouped phases:
    one workgroup per tile, streamed, resident first phase, paired-term
    second phase, and the timed choice; S from 3 to 8: the oracle's bits."""
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(1000 + seed)
    S = int(rng.integers(3, 9))
    G = [S, S + 1][int(rng.integers(0, 2))] if S < 8 else S
    prob = wl.heff_sparse(n_sectors=int(rng.integers(5, 10)), n_triples=int(rng.integers(20, 90)),
                          kop=int(rng.integers(2, 6)), median=float(rng.uniform(6, 100)), sigma_log=1.0,
                          lo_hi=(1, 200), density=float(rng.uniform(0.3, 0.6)), reach=2, U=10, seed=2000 + seed)
    ref = oracle.heff_sparse(prob, S=S, G=G)
    res, paired = ozaki.OZ_HEFF_LAUNCH_RESIDENT, ozaki.OZ_HEFF_LAUNCH_PAIRED_TERMS
    kinds = set()
    try:
        # the 64 x 64 tile (resident up to S = 6, paired terms) and the
        # 8-wave 128 x 64 tile (resident at every S here)
        for v in (0, 3):
            ctx.set_variant(S, G, v)
            for launch in (0, 100000, res, paired, -1):
                ctx.set_heff_launch(launch)
                plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, S, G)
                kinds.update(plan.launches)
                sig = wl.unflatten_sparse(prob, plan.apply(dpsi).cpu().numpy())
                for b in prob.psi_blocks:
                    assert_bitexact(sig[b], ref[b], "seed %d S=%d G=%d variant %d launch %d (kinds %s) block %s"
                                    % (seed, S, G, v, launch, plan.launches, b))
        assert {0, 1, 2} <= kinds
    finally:
        ctx.set_heff_launch(-1)
        ctx.set_variant(S, G, -1)


@pytest.mark.parametrize("seed", range(6))
def test_random_dense_every_launch(oz, seed):
    """Seeded random dense problems (D from 5 to 100, phys 1, 2, 4 or 16,
    1 to 5 operator pairs, so right dimensions off the 32-column groups
    and the unfused exponent pass occur) under every grouped launch, S from
    3 to 8: the oracle's bits."""
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(3000 + seed)
    S = int(rng.integers(3, 9))
    G = [S, S + 1][int(rng.integers(0, 2))] if S < 8 else S
    D, phys, kop = int(rng.integers(5, 101)), int(rng.choice([1, 2, 4, 16])), int(rng.integers(1, 6))
    L, R, psi = wl.heff_dense(D=D, kop=kop, phys=phys, seed=4000 + seed)
    ref = oracle.heff_dense(L, R, psi, S=S, G=G)
    try:
        for v in (0, 3):
            ctx.set_variant(S, G, v)
            for launch in (0, 100000, ozaki.OZ_HEFF_LAUNCH_RESIDENT, ozaki.OZ_HEFF_LAUNCH_PAIRED_TERMS, -1):
                ctx.set_heff_launch(launch)
                plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, S, G)
                got = plan.apply(dpsi).cpu().numpy().reshape(psi.shape)
                assert_bitexact(got, ref, "seed %d S=%d G=%d D=%d phys %d kop %d variant %d launch %d (kinds %s)"
                                % (seed, S, G, D, phys, kop, v, launch, plan.launches))
    finally:
        ctx.set_heff_launch(-1)
        ctx.set_variant(S, G, -1)


def test_fixed_launch_phases(oz):
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=40, kop=2, phys=4, seed=2)
    res = ozaki.OZ_HEFF_LAUNCH_RESIDENT
    try:
        # the paired-term kernel serves the second phase only, on variant 0
        ctx.set_heff_phase(0, 0, 0, ozaki.OZ_HEFF_LAUNCH_PAIRED_TERMS)
        ctx.set_heff_phase(1, 0, 0, 0)
        with pytest.raises(ozaki.OzakiError):
            dense_plan(ozaki, ctx, torch, L, R, psi, 6)
        ctx.set_heff_phase(0, 0, 0, 0)
        ctx.set_heff_phase(1, 3, 0, ozaki.OZ_HEFF_LAUNCH_PAIRED_TERMS)
        with pytest.raises(ozaki.OzakiError):
            dense_plan(ozaki, ctx, torch, L, R, psi, 6)
        ctx.set_heff_phase(1, 0, 1, ozaki.OZ_HEFF_LAUNCH_PAIRED_TERMS)
        plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 6)
        assert plan.phase(1) == (0, 1, ozaki.OZ_HEFF_LAUNCH_PAIRED_TERMS) and plan.launches == (0, 3)
        assert_bitexact(plan.apply(dpsi).cpu().numpy().reshape(psi.shape), oracle.heff_dense(L, R, psi, S=6),
                        "fixed paired-term phase")
        ctx.set_heff_phase(0, 0, 0, 0)
        ctx.set_heff_phase(1, 0, 0, res)
        with pytest.raises(ozaki.OzakiError):
            dense_plan(ozaki, ctx, torch, L, R, psi, 6)
        # the 16-wave tile has no resident kernel
        ctx.set_heff_phase(0, 6, 0, res)
        ctx.set_heff_phase(1, 0, 0, 0)
        with pytest.raises(ozaki.OzakiError):
            dense_plan(ozaki, ctx, torch, L, R, psi, 4)
        ctx.set_heff_phase(0, 0, 0, res)
        plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 6)
        assert plan.phase(0) == (0, 0, res) and plan.launches == (2, 0)
        assert_bitexact(plan.apply(dpsi).cpu().numpy().reshape(psi.shape), oracle.heff_dense(L, R, psi, S=6),
                        "fixed resident phase")
    finally:
        ctx.set_heff_phase(0, -1)
        ctx.set_heff_phase(1, -1)


def test_launch_modes(oz):
    ozaki, ctx, torch = oz
    with pytest.raises(ozaki.OzakiError):
        ctx.set_heff_launch(-4)
    L, R, psi = wl.heff_dense(D=40, kop=2, phys=4, seed=1)
    try:
        ctx.set_heff_launch(0)
        plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 6)
        assert plan.launches == (0, 0)
        a = plan.apply(dpsi)
        ctx.set_heff_launch(2)
        plan2, _, keep2 = dense_plan(ozaki, ctx, torch, L, R, psi, 6)
        assert plan2.launches == (1, 1)
        assert torch.equal(a, plan2.apply(dpsi))
    finally:
        ctx.set_heff_launch(-1)
    # timed choice: only the first phase may stream or run resident, only
    # the second pair its terms
    plan3, _, keep3 = dense_plan(ozaki, ctx, torch, L, R, psi, 6)
    assert plan3.launches[0] in (0, 1, 2) and plan3.launches[1] in (0, 3)
    assert torch.equal(a, plan3.apply(dpsi))
    plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 0)
    assert plan.launches == (-1, -1)


@pytest.mark.parametrize("kind", ["dense", "sparse", "fp64"])
def test_graph_replay_matches_eager(oz, kind):
    """Applies replayed from captured graphs give the eager launches' bits on
    every replay, with other work and synchronisations in between, and read
    the buffers' current contents."""
    ozaki, ctx, torch = oz
    S = 0 if kind == "fp64" else 6
    if kind == "sparse":
        prob = small_sparse(31)
        plan, dpsi, keep = sparse_plan(ozaki, ctx, torch, prob, S)
    else:
        L, R, psi = wl.heff_dense(D=72, kop=3, phys=4, seed=8)
        diag = np.random.default_rng(9).standard_normal(psi.shape)
        plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, S, diag=diag)
    plan.set_graphs(False)
    ref = plan.apply(dpsi).cpu().numpy()
    assert plan.graph_count == 0
    plan.set_graphs(True)
    sig = torch.empty_like(dpsi)
    other = torch.empty_like(dpsi)
    psi2 = dpsi * 0.5 - 1.0
    plan.set_graphs(False)
    ref2 = plan.apply(psi2).cpu().numpy()
    plan.set_graphs(True)
    for rep in range(4):
        sig.fill_(float("nan"))
        plan.apply(dpsi, sig)
        torch.cuda.synchronize()
        assert_bitexact(sig.cpu().numpy(), ref, "%s replay %d" % (kind, rep))
        plan.apply(psi2, other)                       # a second graph, interleaved
        (other * 2.0).sum().item()                    # eager work and a host sync between replays
        assert_bitexact(other.cpu().numpy(), ref2, "%s second pair replay %d" % (kind, rep))
    assert plan.graph_count == 2
    # the graph reads whatever psi holds now
    dpsi.copy_(psi2)
    plan.apply(dpsi, sig)
    assert_bitexact(sig.cpu().numpy(), ref2, "%s new contents" % kind)
    assert plan.graph_count == 2
    if kind == "dense" and S:
        want = oracle.heff_dense(L, R, psi * 0.5 - 1.0, S=S, diag=diag).ravel()
        assert_bitexact(sig.cpu().numpy(), want, "dense oracle")


def test_graph_cache_eviction(oz):
    """More distinct (psi, sigma) pairs than the cache holds: evicted pairs are
    captured again and every result stays exact."""
    ozaki, ctx, torch = oz
    L, R, psi = wl.heff_dense(D=24, kop=2, phys=1, seed=12)
    plan, dpsi, keep = dense_plan(ozaki, ctx, torch, L, R, psi, 5)
    plan.set_graphs(False)
    ref = plan.apply(dpsi).cpu().numpy()
    plan.set_graphs(True)
    outs = [torch.empty_like(dpsi) for _ in range(100)]
    for o in outs:
        plan.apply(dpsi, o)
    assert plan.graph_count == 96
    for o in outs[:3]:
        o.zero_()
        plan.apply(dpsi, o)
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert_bitexact(o.cpu().numpy(), ref, "pair %d" % i)
