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
