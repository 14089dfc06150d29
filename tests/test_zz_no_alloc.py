"""nsk_rhs_noalloc (lifted gradients, geometry and element order in the
library's static device scratch) against nsk_rhs (the same kernels on the
caller's bound workspace): bitwise equal, on two calls in a row whose second
problem is smaller, then the first again, with bound and unbound contexts, in
FP64 and mixed precision."""
import pytest

from paper_1912_12059_amd import inputs as I

pytestmark = pytest.mark.gpu

PHYS = dict(T=0.85, eps=1e-3, kappa=1e-5, alpha=1000.0, beta=1e-3)


def _reference(gpu, dim, N, nel, prec, seed):
    """The state, nsk_rhs of it on a bound context, and an unbound context of
    the same problem."""
    import torch

    m, U = I.smooth_random(dim, N, nel, seed=seed)
    s = gpu.Solver(dim=dim, N=N, nel=tuple(nel), precision=prec, **PHYS)
    Ud = torch.from_numpy(U.reshape(-1)).to("cuda:0")
    R = torch.empty_like(Ud)
    gpu.nsk_rhs(s.ctx, Ud.data_ptr(), R.data_ptr())
    torch.cuda.synchronize()
    mesh, keep = gpu.make_mesh(dim, N, tuple(nel))
    unbound = gpu.nsk_create(mesh, gpu.make_params(precision=prec, **PHYS))
    return s, unbound, Ud, R


def _noalloc(gpu, ctx, Ud):
    import torch

    R = torch.full_like(Ud, float("nan"))
    torch.cuda.synchronize()
    gpu.nsk_rhs_noalloc(ctx, Ud.data_ptr(), R.data_ptr(), 0)
    torch.cuda.synchronize()
    return R


@pytest.mark.parametrize("prec", [0, 1])
def test_rhs_noalloc_equals_rhs(gpu, prec):
    import torch

    big = _reference(gpu, 3, 4, (6, 5, 4), prec, seed=71)
    small = _reference(gpu, 2, 3, (5, 4), prec, seed=72)
    try:
        for s, unbound, Ud, R in (big, small, big):
            for ctx in (s.ctx, unbound):
                got = _noalloc(gpu, ctx, Ud)
                assert bool(torch.isfinite(R).all())
                assert torch.equal(got, R)
    finally:
        for s, unbound, _, _ in (big, small):
            s.close()
            gpu.nsk_destroy(unbound)
