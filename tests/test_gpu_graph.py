"""Single-mesh steps replayed as a captured HIP graph (pairs of steps on a
non-null bound stream) against the same steps launched one by one (the null
stream cannot be captured): bitwise equal after every call, with eager torch
work and synchronisations between the replays, across a change of step size
and of launch shape (each re-captures)."""
import numpy as np
import pytest

from paper_1912_12059_amd import inputs as I

pytestmark = pytest.mark.gpu

PHYS = dict(T=0.85, eps=1e-3, kappa=1e-5, alpha=1000.0, beta=1e-3)


def _pair(gpu, m, **kw):
    import torch

    base = dict(dim=m.dim, N=m.N, nel=tuple(m.nel), lo=tuple(m.lo) + (0.0,) * 3, hi=tuple(m.hi) + (1.0,) * 3)
    graphed = gpu.Solver(stream=torch.cuda.Stream(), **base, **kw)
    eager = gpu.Solver(**base, **kw)
    assert eager.stream.cuda_stream == 0  # the null stream: launched stage by stage
    return graphed, eager


@pytest.mark.parametrize("dim,N,nel,prec", [(1, 3, (64,), 0), (2, 4, (9, 7), 0), (3, 4, (5, 4, 3), 0),
                                            (3, 3, (6, 5, 4), 1)])
def test_graph_replay_equals_eager_steps(gpu, dim, N, nel, prec):
    import torch

    m, U = I.smooth_random(dim, N, nel, seed=90 + dim)
    g, e = _pair(gpu, m, precision=prec, **PHYS)
    for s in (g, e):
        s.set_state(U)
    # 2 and 4 steps replay the graph; 3 replays it once and adds one step
    for k, (dt, n) in enumerate(((1e-6, 2), (1e-6, 4), (1e-6, 3), (7e-7, 2), (7e-7, 5))):
        g.rk_step(dt, n)
        e.rk_step(dt, n)
        a = torch.randn(1 << 16, device="cuda:0")  # eager work between replays
        float(a.sum())
        torch.cuda.synchronize()
        assert torch.equal(g.get_state(), e.get_state()), k
        if k == 2:
            gpu.nsk_set_tile(g.ctx, 1, 2)  # a new launch shape re-captures
    fin = g.get_state().cpu().numpy()
    assert np.all(np.isfinite(fin)) and not np.array_equal(fin, U.reshape(fin.shape))
    g.close()
    e.close()


def test_side_stream_solver_full_size_3d_mixed(gpu):
    """A solver bound to a side stream right after torch allocates its
    multi-GB buffers (zero-filled on torch's current stream), stepped ten
    times as graph replays, equals the null-stream solver bitwise: the
    binding orders its stream after torch's work."""
    import torch

    m, U = I.collision_3d(nel=(96, 48, 48), N=4, We=100.0)
    U0 = torch.from_numpy(U.reshape(-1)).to("cuda:0")
    del U
    outs = []
    for stream in (torch.cuda.Stream(), None):
        s = gpu.Solver(dim=3, N=4, nel=(96, 48, 48), lo=(0, 0, 0), hi=(2, 1, 1), precision=1, stream=stream,
                       **PHYS)
        s.set_state(U0)
        s.rk_step(s.dt_estimate(0.5), 10)
        outs.append(s.get_state()[0].reshape(-1).clone())
        s.close()
        del s
    assert bool(torch.isfinite(outs[0]).all()) and torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("every_stage", [1, 0])
def test_graph_replay_with_closure(gpu, every_stage):
    """Steps of a closure context (closure kernel every stage, or once per
    step with its source reused by the later stages) captured into the step
    graph equal stage-by-stage launches bit for bit."""
    import torch

    from paper_1912_12059_amd import closure as CL

    m, U = I.smooth_random(3, 4, (5, 4, 3), seed=95)
    net = CL.Network(seed=2)
    norm = dict(CL.default_norm(1e-4), out_m=1e-2, out_c=1e-2)
    base = dict(dim=3, N=4, nel=(5, 4, 3), alpha=200.0, kappa=1e-4, every_stage=every_stage)
    g = CL.closure_solver(net, norm, stream=torch.cuda.Stream(), **base)
    e = CL.closure_solver(net, norm, **base)
    for s in (g, e):
        s.set_state(U)
    for n in (2, 3, 4):
        g.rk_step(2e-6, n)
        e.rk_step(2e-6, n)
        torch.cuda.synchronize()
        assert torch.equal(g.get_state(), e.get_state()), n
    assert bool(torch.isfinite(g.get_state()).all())
    g.close()
    e.close()


@pytest.mark.parametrize("prec,flux", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_one_launch_steps_equal_staged_steps(gpu, prec, flux):
    """The 1D slab workload (64 elements, N = 3) fits one workgroup of the
    first tile variant, so all its steps run in one launch (on the null
    stream and on a side stream).  The second variant takes two workgroups
    and runs the same steps stage by stage (launches on the null stream,
    graph replays on a side stream).  All four agree bit for bit."""
    import torch

    m, U = I.slab_1d()
    kw = dict(dim=1, N=3, nel=(64,), alpha=500.0, beta=1e-3, eps=1e-3, kappa=1e-5, precision=prec, flux=flux)
    one = gpu.Solver(**kw)
    one_side = gpu.Solver(stream=torch.cuda.Stream(), **kw)
    staged = gpu.Solver(**kw)
    graphed = gpu.Solver(stream=torch.cuda.Stream(), **kw)
    for s in (staged, graphed):
        gpu.nsk_set_tile(s.ctx, 1, 0)
    solvers = (one, one_side, staged, graphed)
    for s in solvers:
        s.set_state(U)
    dt = one.dt_estimate(0.5)
    for n in (1, 2, 5, 40):
        for s in solvers:
            s.rk_step(dt, n)
        torch.cuda.synchronize()
        ref = staged.get_state()
        for s in (one, one_side, graphed):
            assert torch.equal(s.get_state(), ref), n
    fin = ref.cpu().numpy()
    assert np.all(np.isfinite(fin)) and not np.array_equal(fin, U.reshape(fin.shape))
    for s in solvers:
        s.close()
