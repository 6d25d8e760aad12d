"""The allocation-free GEMM entry point (ozaki_dgemm_static, for callers
that cannot allocate device memory) against ozaki_dgemm with a caller
workspace: the same bits, on two calls in a row (the second smaller, so the
shared static buffer holds the first call's data), for the emulated and the
native path, and a clear error above the static size."""
import numpy as np
import pytest

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


def pair(torch, n, m, k, U, seed):
    A, B = wl.gemm_pair(n, U=U, seed=seed, m=m, k=k)
    return torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()


@pytest.mark.parametrize("S,G", [(6, 6), (7, 8), (3, 5), (0, 0)])
def test_static_matches_workspace_call(oz, S, G):
    ozaki, ctx, torch = oz
    print("[test] static workspace S=%d G=%d" % (S, G), flush=True)
    for (n, m, k, ta, tb, beta, seed) in [(1500, 1100, 1300, "N", "T", 0.0, 1), (200, 170, 90, "T", "N", -0.5, 2)]:
        A, B = pair(torch, n, m, k, 10, seed)
        if ta == "T":
            A = A.t().contiguous()
        if tb == "T":
            B = B.t().contiguous()
        M = A.size(1) if ta == "T" else A.size(0)
        N = B.size(0) if tb == "T" else B.size(1)
        C0 = torch.from_numpy(np.random.default_rng(seed).standard_normal((M, N))).cuda()
        ref = ctx.dgemm(A, B, slices=S, ndiag=G, alpha=1.25, beta=beta, C=C0.clone(), transa=ta, transb=tb)
        got = ctx.dgemm_static(A, B, C0.clone(), slices=S, ndiag=G, alpha=1.25, beta=beta, transa=ta, transb=tb)
        torch.cuda.synchronize()
        assert_bitexact(got.cpu().numpy(), ref.cpu().numpy(), "S=%d G=%d %dx%dx%d" % (S, G, M, N, k))


def test_static_too_large(oz):
    ozaki, ctx, torch = oz
    need = ozaki._lib.ozaki_dgemm_workspace_bytes(4096, 4096, 4096, 6, 0)
    assert need > ozaki.OZ_STATIC_WORKSPACE_BYTES
    A = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda")
    C = torch.empty_like(A)
    with pytest.raises(ozaki.OzakiError) as ei:
        ctx.dgemm_static(A, A, C, slices=6)
    assert ei.value.status == -2 and "static" in str(ei.value)
    # the native path needs no workspace at any size
    ctx.dgemm_static(A, A, C, slices=0)
    torch.cuda.synchronize()
    assert float(C.abs().max()) == 0.0
