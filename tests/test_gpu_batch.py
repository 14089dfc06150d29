"""Batched form: instances of uneven mesh and degree in per-degree kernels
(one workgroup per item or a persistent grid), two steps per captured HIP
graph.  Every batched instance must give
the same bits as the same instance run alone (identical arithmetic, only the
launch shape differs), on every graph replay."""
import numpy as np
import pytest

from paper_1912_12059_amd import inputs as I

pytestmark = pytest.mark.gpu

PHYS = dict(T=0.85, eps=1e-3, kappa=1e-5, alpha=1000.0, beta=1e-3)
MESHES = [
    {"nel": (6, 4, 4), "N": 3, "hi": (1.5, 1.0, 1.0)},
    {"nel": (5, 4, 3), "N": 4, "hi": (1.25, 1.0, 0.75)},
    {"nel": (4, 3, 3), "N": 5, "hi": (1.0, 0.75, 0.75)},
    {"nel": (7, 4, 3), "N": 3, "hi": (1.75, 1.0, 0.75)},
    {"nel": (3, 3, 3), "N": 4, "hi": (0.75, 0.75, 0.75)},
]


def _states():
    out = []
    for k, m in enumerate(MESHES):
        _, U = I.smooth_random(3, m["N"], m["nel"], seed=100 + k, hi=m["hi"])
        out.append(U)
    return out


def _single(gpu, m, U, dt, nsteps, precision):
    s = gpu.Solver(dim=3, N=m["N"], nel=m["nel"], hi=m["hi"], precision=precision, **PHYS)
    s.set_state(U)
    s.rk_step(dt, nsteps)
    out = s.get_state().cpu().numpy()
    s.close()
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single_runs_on_every_replay(gpu, precision):
    import torch

    states = _states()
    b = gpu.Batch(MESHES, precision=precision, **PHYS)
    for i, U in enumerate(states):
        b.set_state(i, U)
    dt = 1.5e-6
    ref = [U.copy() for U in states]
    for replay in range(3):
        b.rk_step(dt, 2)                       # one graph replay
        # eager work of the program between replays
        x = torch.ones(1 << 20, device="cuda:0")
        x.mul_(2.0)
        torch.cuda.synchronize()
        for i, m in enumerate(MESHES):
            ref[i] = _single(gpu, m, ref[i], dt, 2, precision)
            got = b.get_state(i).cpu().numpy().reshape(ref[i].shape)
            assert np.all(np.isfinite(got))
            assert np.array_equal(got, ref[i]), (replay, i)
    b.close()


def test_batch_odd_steps_and_dt_change(gpu):
    states = _states()
    b = gpu.Batch(MESHES, precision=0, **PHYS)
    for i, U in enumerate(states):
        b.set_state(i, U)
    b.rk_step(1e-6, 3)      # one replay + one ordinary step
    b.rk_step(2e-6, 2)      # new dt: graph captured again
    for i, m in enumerate(MESHES):
        ref = _single(gpu, m, _single(gpu, m, states[i], 1e-6, 3, 0), 2e-6, 2, 0)
        assert np.array_equal(b.get_state(i).cpu().numpy().reshape(ref.shape), ref), i
    b.close()


def test_batch_autotune_and_dt(gpu):
    states = _states()
    b = gpu.Batch(MESHES, precision=1, **PHYS)
    for i, U in enumerate(states):
        b.set_state(i, U)
    ms = gpu.nsk_batch_autotune(b.b, 2)
    groups = gpu.nsk_batch_groups(b.b)
    assert sorted(g["N"] for g in groups) == [3, 4, 5]
    assert all(g["variant"] in (0, 1) and g["gridmul"] in (0, 2, 4, 8) and 0 <= g["order"] < 6
               and g["chunk_mib"] in (0, 128, 256, 512) for g in groups)
    assert all(x > 0 for x in ms[: gpu.BATCH_TUNE_SLOTS * len(groups)])
    # the autotuner writes only scratch: states are untouched
    for i, U in enumerate(states):
        assert np.array_equal(b.get_state(i).cpu().numpy().reshape(U.shape), U)
    dts = []
    for i, m in enumerate(MESHES):
        s = gpu.Solver(dim=3, N=m["N"], nel=m["nel"], hi=m["hi"], precision=1, **PHYS)
        s.set_state(states[i])
        dts.append(s.dt_estimate(0.5))
        s.close()
    assert b.dt_estimate(0.5) == min(dts)
    b.close()


def test_batch_instance_matches_oracle(O, gpu):
    states = _states()
    b = gpu.Batch(MESHES, precision=0, **PHYS)
    for i, U in enumerate(states):
        b.set_state(i, U)
    b.rk_step(1e-6, 4)
    for i in (0, 2):
        m = MESHES[i]
        P = O.Problem(dim=3, N=m["N"], nel=m["nel"], hi=m["hi"], **PHYS)
        ref = O.run(P, states[i], 1e-6, 4)
        got = b.get_state(i).cpu().numpy().reshape(ref.shape)
        for v in range(5):
            scale = np.abs(ref[v]).max()
            assert np.abs(got[v] - ref[v]).max() <= 1e-10 * scale, (i, v)
    b.close()


@pytest.mark.parametrize("gridmul", [0, 4])
def test_batch_chunks_of_instances(gpu, gridmul):
    """Instances whose working set exceeds the 64 MiB chunk budget run as
    separate chunks, each through all the stages of a replay; the result
    must still be the single runs' bits."""
    meshes = [{"nel": (20, 20, 19), "N": 4, "hi": (1.0, 1.0, 0.95)},
              {"nel": (19, 20, 20), "N": 4, "hi": (0.95, 1.0, 1.0)},
              {"nel": (8, 6, 6), "N": 3, "hi": (1.0, 0.75, 0.75)}]
    states = []
    for k, m in enumerate(meshes):
        _, U = I.smooth_random(3, m["N"], m["nel"], seed=200 + k, hi=m["hi"])
        states.append(U)
    # working set of the first two instances: (15 + 9) doubles x 0.95M nodes > 64 MiB
    assert 24 * 8 * 20 * 20 * 19 * 125 > 64 << 20
    b = gpu.Batch(meshes, precision=0, **PHYS)
    for i, U in enumerate(states):
        b.set_state(i, U)
    groups = gpu.nsk_batch_groups(b.b)
    for gi, g in enumerate(groups):
        gpu.nsk_batch_set_group(b.b, gi, 0, gridmul, 3, 64)
    assert all(g["chunk_mib"] == 64 and g["gridmul"] == gridmul for g in gpu.nsk_batch_groups(b.b))
    b.rk_step(1e-6, 2)
    for i, m in enumerate(meshes):
        ref = _single(gpu, m, states[i], 1e-6, 2, 0)
        assert np.array_equal(b.get_state(i).cpu().numpy().reshape(ref.shape), ref), i
    b.close()


def test_batched_sweep_full_size_matches_single_runs(gpu):
    """The 24-instance collision sweep at its full size (159M nodes, N in
    {3, 4, 5}), mixed precision, autotuned: after one graph replay (two
    steps) every instance equals its single run bit for bit."""
    import torch

    sweep = I.batched_sweep()
    meshes = [{"nel": s["nel"], "N": s["N"], "lo": s["lo"], "hi": s["hi"]} for s in sweep]
    b = gpu.Batch(meshes, precision=1, **PHYS)
    init = []
    for i, s in enumerate(sweep):
        _, U = I.collision_3d(nel=s["nel"], N=s["N"], We=s["We"], radius=s["radius"], lo=s["lo"], hi=s["hi"],
                              impact=s["impact"], device="cuda:0")
        U = U.reshape(-1)
        init.append(U)
        b.set_state(i, U)
    gpu.nsk_batch_autotune(b.b, 1)
    dt = b.dt_estimate(0.5)
    b.rk_step(dt, 2)
    for i, m in enumerate(meshes):
        s = gpu.Solver(dim=3, N=m["N"], nel=m["nel"], lo=m["lo"], hi=m["hi"], precision=1, **PHYS)
        s.set_state(init[i])
        s.rk_step(dt, 2)
        ref = s.get_state().reshape(-1)
        got = b.get_state(i)
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref), i
        s.close()
    b.close()
