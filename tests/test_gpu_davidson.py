"""GPU Davidson (device-resident FP64 solver around the H_eff matvec) against
brute-force diagonalisation and the CPU oracle's Davidson."""
import numpy as np
import pytest

import oracle
from paper_2510_04795_amd import workloads as wl

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


def solver(ozaki, ctx, torch, prob, S, G=0, m_max=32, tol=1e-8, max_iter=300):
    layout, Lf, Rf, _, triples = wl.flatten_dense(prob.L, prob.R, prob.x0[:, None, :])
    keep = [dev(torch, Lf), dev(torch, Rf), dev(torch, prob.delta.ravel())]
    plan = ozaki.HeffPlan(ctx, layout, keep[0], keep[1], triples, diag=keep[2], slices=S, ndiag=G)
    hd = dev(torch, prob.hdiag.ravel())
    x0 = dev(torch, prob.x0.ravel())
    dav = ozaki.Davidson(ctx, plan, hd, x0, m_max=m_max, tol=tol, max_iter=max_iter)
    return dav, (plan, keep, hd, x0)


def brute(prob):
    H = sum(np.kron(prob.L[k], prob.R[k]) for k in range(prob.L.shape[0])) + np.diag(prob.delta.ravel())
    return np.linalg.eigh(H)


def test_d16_against_brute_force(oz):
    ozaki, ctx, torch = oz
    prob = wl.davidson_problem(D=16, kop=32)
    ev, evec = brute(prob)
    dav, keep = solver(ozaki, ctx, torch, prob, 0)
    theta, status, its, res = dav.run()
    assert status == "converged" and res <= 1e-8
    assert abs(theta - ev[0]) < 1e-10
    x = dav.vector().cpu().numpy()
    assert abs(abs(x @ evec[:, 0]) - 1) < 1e-10
    for S in (4, 6, 8):
        dav, keep = solver(ozaki, ctx, torch, prob, S)
        th, st, its_s, res_s = dav.run()
        assert st == "converged"
        assert abs(th - ev[0]) < 1e-6, (S, th - ev[0])


@pytest.mark.parametrize("S", [0, 5])
def test_matches_oracle_davidson(oz, S):
    """Same problem, same start: energies agree far inside the 1e-6 Ha target
    and the iteration counts are close (the Rayleigh-Ritz solvers differ:
    Jacobi on the device, LAPACK on the CPU)."""
    ozaki, ctx, torch = oz
    prob = wl.davidson_problem(D=40, kop=8)
    dav, keep = solver(ozaki, ctx, torch, prob, S)
    th, st, its, res = dav.run()
    mv = oracle.heff_matvec(prob.L, prob.R, prob.delta, S=S)
    th_ref, _, st_ref, its_ref, _ = oracle.davidson(mv, prob.hdiag, prob.x0, tol=1e-8)
    assert st == "converged" and st_ref == oracle.CONVERGED
    assert abs(th - th_ref) < 1e-9
    assert abs(its - its_ref) <= 2


@pytest.mark.parametrize("S,m_max", [(0, 32), (6, 32), (5, 4)])
def test_graph_replay_matches_direct(oz, S, m_max):
    """Steps replayed from the per-(basis size, Ritz buffer) graphs give the
    directly issued steps' bits: theta and residual of every step, the basis
    size, the status and the Ritz vector reported after every step (with a
    restart of a four-vector basis included)."""
    ozaki, ctx, torch = oz
    prob = wl.davidson_problem(D=24, kop=6, seed=3)
    runs = []
    for graphs in (False, True):
        dav, keep = solver(ozaki, ctx, torch, prob, S, m_max=m_max, tol=1e-10)
        dav.set_graphs(graphs)
        hist = []
        while True:
            info = dav.step()
            hist.append((info.theta, info.resnorm, info.m, info.status, dav.vector().cpu().numpy().tobytes()))
            if info.status != ozaki.OZ_OK:
                break
        runs.append((hist, dav.graph_count))
        dav.close()
    (h0, n0), (h1, n1) = runs
    assert n0 == 0 and n1 > 0
    assert len(h0) == len(h1) > 3
    for a, b in zip(h0, h1):
        assert a[:4] == b[:4] and a[4] == b[4]
    assert h1[-1][3] in (ozaki.OZ_CONVERGED, ozaki.OZ_STAGNATED)


def test_restart_small_basis(oz):
    ozaki, ctx, torch = oz
    prob = wl.davidson_problem(D=12, kop=6)
    ev, _ = brute(prob)
    dav, keep = solver(ozaki, ctx, torch, prob, 0, m_max=4, tol=1e-9)
    th, st, its, res = dav.run()
    assert st == "converged" and abs(th - ev[0]) < 1e-9


def test_unreachable_tolerance_stops(oz):
    """Two slices cannot resolve the residual below ~1e-3: the solver must stop
    (stagnation or the iteration cap), not loop forever."""
    ozaki, ctx, torch = oz
    prob = wl.davidson_problem(D=16, kop=8)
    dav, keep = solver(ozaki, ctx, torch, prob, 2, tol=1e-14, max_iter=120)
    th, st, its, res = dav.run()
    assert st in ("stagnated", "max_iter")
    with pytest.raises(ozaki.OzakiError):
        dav.step()


def test_bad_arguments(oz):
    ozaki, ctx, torch = oz
    prob = wl.davidson_problem(D=8, kop=2)
    prob.x0[:] = 0.0
    with pytest.raises(ozaki.OzakiError):
        solver(ozaki, ctx, torch, prob, 0)
    prob = wl.davidson_problem(D=8, kop=2)
    with pytest.raises(ozaki.OzakiError):
        solver(ozaki, ctx, torch, prob, 0, m_max=1)



def test_binding_checks_vector_sizes(oz):
    """hdiag, x0, the plan's diagonal and the vector output must hold the
    plan's n elements: the binding refuses others before the library could
    read or write past them."""
    ozaki, ctx, torch = oz
    prob = wl.davidson_problem(D=8, kop=2)
    layout, Lf, Rf, _, triples = wl.flatten_dense(prob.L, prob.R, prob.x0[:, None, :])
    dL, dR = dev(torch, Lf), dev(torch, Rf)
    n = prob.x0.size
    with pytest.raises(ValueError):
        ozaki.HeffPlan(ctx, layout, dL, dR, triples, diag=dev(torch, prob.delta.ravel()[:-1]), slices=6)
    with pytest.raises(TypeError):
        ozaki.HeffPlan(ctx, layout, dL, dR, triples, diag=dev(torch, prob.delta.ravel()).float(), slices=6)
    plan = ozaki.HeffPlan(ctx, layout, dL, dR, triples, diag=dev(torch, prob.delta.ravel()), slices=6)
    hd, x0 = dev(torch, prob.hdiag.ravel()), dev(torch, prob.x0.ravel())
    with pytest.raises(ValueError):
        ozaki.Davidson(ctx, plan, hd[:-1], x0)
    with pytest.raises(ValueError):
        ozaki.Davidson(ctx, plan, hd, torch.cat([x0, x0]))
    with pytest.raises(ValueError):
        ozaki.Lanczos(ctx, plan, x0[:n - 2])
    dav = ozaki.Davidson(ctx, plan, hd, x0)
    dav.step()
    with pytest.raises(ValueError):
        dav.vector(torch.empty(n - 1, dtype=torch.float64, device="cuda"))
    assert dav.vector().numel() == n
    lz = ozaki.Lanczos(ctx, plan, x0)
    lz.step()
    with pytest.raises(ValueError):
        lz.vector(torch.empty(2 * n, dtype=torch.float64, device="cuda")[::2])
    assert lz.vector().numel() == n
    dav.close()
    lz.close()
    plan.close()



@pytest.mark.parametrize("seed", range(8))
def test_random_problems_against_brute_force(oz, seed):
    """Seeded random small problems (D = 4..20, 1 to 8 operator pairs, with
    or without the planted low state, basis limits 4, 8 and 32 so restarts
    occur): Davidson and Lanczos reach the lowest eigenvalue of the dense
    matrix (numpy eigh), FP64 within 1e-9 relative with the eigenvector,
    emulated S = 4..8 within 1e-6 (the energy target)."""
    ozaki, ctx, torch = oz
    rng = np.random.default_rng(500 + seed)
    D, kop = int(rng.integers(4, 21)), int(rng.integers(1, 9))
    well = float(rng.choice([-30.0, -5.0, 0.0]))
    m_max = int(rng.choice([4, 8, 32]))
    S = int(rng.choice([4, 5, 6, 7, 8]))
    prob = wl.davidson_problem(D=D, kop=kop, well=well, seed=600 + seed)
    ev, evec = brute(prob)
    scale = max(1.0, abs(ev[0]))
    what = "seed %d D=%d kop=%d well=%g m_max=%d" % (seed, D, kop, well, m_max)
    for make in (solver, lanczos_solver):
        sol, keep = make(ozaki, ctx, torch, prob, 0, m_max=m_max, tol=1e-9, max_iter=600)
        th, st, its, res = sol.run()
        assert st == "converged", (what, make.__name__, st, its, res)
        assert abs(th - ev[0]) <= 1e-9 * scale, (what, make.__name__, th - ev[0])
        x = sol.vector().cpu().numpy()
        assert abs(abs(x @ evec[:, 0]) - 1) < 1e-8 or ev[1] - ev[0] < 1e-6 * scale, (what, make.__name__)
        sol.close()
        sol, keep = make(ozaki, ctx, torch, prob, S, m_max=m_max, tol=1e-8, max_iter=600)
        th, st, its, res = sol.run()
        assert st in ("converged", "stagnated"), (what, make.__name__, S, st)
        assert abs(th - ev[0]) <= 1e-6 * scale, (what, make.__name__, S, th - ev[0])
        sol.close()


# ---------------------------------------------------------------- Lanczos
def lanczos_solver(ozaki, ctx, torch, prob, S, G=0, m_max=32, tol=1e-8, max_iter=300):
    layout, Lf, Rf, _, triples = wl.flatten_dense(prob.L, prob.R, prob.x0[:, None, :])
    keep = [dev(torch, Lf), dev(torch, Rf), dev(torch, prob.delta.ravel())]
    plan = ozaki.HeffPlan(ctx, layout, keep[0], keep[1], triples, diag=keep[2], slices=S, ndiag=G)
    x0 = dev(torch, prob.x0.ravel())
    lz = ozaki.Lanczos(ctx, plan, x0, m_max=m_max, tol=tol, max_iter=max_iter)
    return lz, (plan, keep, x0)


def test_lanczos_d16_against_brute_force(oz):
    ozaki, ctx, torch = oz
    prob = wl.davidson_problem(D=16, kop=32)
    ev, evec = brute(prob)
    lz, keep = lanczos_solver(ozaki, ctx, torch, prob, 0)
    theta, status, its, res = lz.run()
    assert status == "converged" and res <= 1e-8
    assert abs(theta - ev[0]) < 1e-10
    x = lz.vector().cpu().numpy()
    assert abs(np.linalg.norm(x) - 1) < 1e-12
    assert abs(abs(x @ evec[:, 0]) - 1) < 1e-8
    for S in (4, 6):
        lz, keep = lanczos_solver(ozaki, ctx, torch, prob, S)
        th, st, _, _ = lz.run()
        assert st == "converged" and abs(th - ev[0]) < 1e-6, (S, th - ev[0])


@pytest.mark.parametrize("S", [0, 3, 5])
def test_lanczos_matches_oracle(oz, S):
    """Same problem and start: the device and the oracle Lanczos agree in
    energy far inside the matvec's own error and in the iteration count (the
    tridiagonal eigensolvers differ: Jacobi on the host, LAPACK in the oracle)."""
    ozaki, ctx, torch = oz
    prob = wl.davidson_problem(D=40, kop=8)
    lz, keep = lanczos_solver(ozaki, ctx, torch, prob, S, m_max=12)
    th, st, its, res = lz.run()
    mv = oracle.heff_matvec(prob.L, prob.R, prob.delta, S=S)
    th_ref, x_ref, st_ref, its_ref, _ = oracle.lanczos(mv, prob.x0, m_max=12, tol=1e-8)
    assert st == st_ref == oracle.CONVERGED
    # with S = 3 a last-bit change of the vector can move a slice boundary and
    # the matvec by its own error (~1e-7 relative): the runs then differ slightly
    assert abs(th - th_ref) < {0: 1e-10, 3: 1e-6, 5: 1e-9}[S]
    assert abs(its - its_ref) <= (3 if S == 3 else 2)
    x = lz.vector().cpu().numpy()
    assert abs(abs(x @ x_ref) - 1) < 1e-8


def test_lanczos_restart_vector(oz):
    """m_max = 4: the fourth step restarts from the Ritz vector, which the
    solver then returns; the oracle's fourth-step Ritz vector is the same."""
    ozaki, ctx, torch = oz
    prob = wl.davidson_problem(D=12, kop=6)
    lz, keep = lanczos_solver(ozaki, ctx, torch, prob, 0, m_max=4, tol=1e-12)
    for _ in range(4):
        info = lz.step()
    assert info.status == 0 and info.iter == 4
    x = lz.vector().cpu().numpy()
    mv = oracle.heff_matvec(prob.L, prob.R, prob.delta)
    th4, x4, _, _, _ = oracle.lanczos(mv, prob.x0, m_max=4, tol=1e-12, max_iter=4)
    assert abs(info.theta - th4) < 1e-11
    assert abs(abs(x @ x4) / np.linalg.norm(x4) - 1) < 1e-10
    ev, _ = brute(prob)
    th, st, its, _ = lz.run()
    assert st == "converged" and abs(th - ev[0]) < 1e-10


def test_lanczos_invariant_subspace(oz):
    """Diagonal L_k, R_k give a diagonal H; a start vector on three basis
    states spans an invariant subspace, found at the third step."""
    ozaki, ctx, torch = oz
    prob = wl.davidson_problem(D=6, kop=2)
    rng = np.random.default_rng(7)
    for k in range(2):
        prob.L[k] = np.diag(rng.standard_normal(6))
        prob.R[k] = np.diag(rng.standard_normal(6))
    prob.delta[:] = 0.0
    prob.x0[:] = 0.0
    prob.x0[0, 0] = prob.x0[2, 3] = prob.x0[5, 1] = 1.0
    hd = sum(np.outer(np.diag(prob.L[k]), np.diag(prob.R[k])) for k in range(2))
    lz, keep = lanczos_solver(ozaki, ctx, torch, prob, 0, tol=0.0)
    th, st, its, _ = lz.run()
    assert st == "converged" and its == 3
    assert abs(th - min(hd[0, 0], hd[2, 3], hd[5, 1])) < 1e-13


def test_lanczos_stagnation_and_errors(oz):
    ozaki, ctx, torch = oz
    prob = wl.davidson_problem(D=10, kop=6)
    lz, keep = lanczos_solver(ozaki, ctx, torch, prob, 3, m_max=8, tol=1e-30)
    th, st, its, res = lz.run()
    assert st == "stagnated"
    with pytest.raises(ozaki.OzakiError):
        lz.step()
    lz, keep = lanczos_solver(ozaki, ctx, torch, prob, 0)
    with pytest.raises(ozaki.OzakiError):
        lz.vector()
    with pytest.raises(ozaki.OzakiError):
        lanczos_solver(ozaki, ctx, torch, prob, 0, m_max=1)
    with pytest.raises(ozaki.OzakiError):
        lanczos_solver(ozaki, ctx, torch, prob, 0, m_max=65)
    prob.x0[:] = 0.0
    with pytest.raises(ozaki.OzakiError):
        lanczos_solver(ozaki, ctx, torch, prob, 0)
