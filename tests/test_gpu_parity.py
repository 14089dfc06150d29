"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerance for FP64 right-hand sides (derived from the arithmetic, see
tests/tolerances.py): per variable, |R_gpu - R_cpu| <= RHS_ULPS ulps of the
largest single term summed into R.  Trajectories: relative max-norm
difference per variable <= 1e-10.
"""
import numpy as np
import pytest

from paper_1912_12059_amd import inputs as I
from tolerances import RHS_ULPS, record, rhs_err_ulps, term_scales

pytestmark = pytest.mark.gpu

TRAJ_TOL = 1e-10


def _hmin(m):
    return min(float(np.diff(m.breaks(d)).min()) for d in range(m.dim))


def _rhs_check(O, m, U, R, Rc, alpha):
    ulps = rhs_err_ulps(R, Rc, term_scales(O, m.N, _hmin(m), U, alpha))
    assert ulps <= RHS_ULPS, f"{ulps:.1f} ulps of the term scale"


def _problem(O, m, **kw):
    nel = tuple(m.nel) + (1,) * (3 - len(m.nel))
    lo = tuple(m.lo) + (0.0,) * (3 - len(m.lo))
    hi = tuple(m.hi) + (1.0,) * (3 - len(m.hi))
    return O.Problem(dim=m.dim, N=m.N, nel=nel, lo=lo, hi=hi, xbreaks=m.xbreaks, **kw)


def _solver(gpu, m, **kw):
    return gpu.Solver(dim=m.dim, N=m.N, nel=tuple(m.nel), lo=tuple(m.lo) + (0.0,) * 3,
                      hi=tuple(m.hi) + (1.0,) * 3, xbreaks=m.xbreaks, **kw)


def _relerr_per_var(a, b, scale=None):
    """max over variables of max|a_v - b_v| / max|b_v| (or / scale[v]),
    recorded against TRAJ_TOL."""
    a = np.asarray(a).reshape(b.shape)
    out = []
    for v in range(b.shape[0]):
        sc = np.max(np.abs(b[v])) if scale is None else scale[v]
        out.append(np.max(np.abs(a[v] - b[v])) / (sc if sc > 0 else 1.0))
    record("trajectory, relative error per variable", max(out), TRAJ_TOL)
    return max(out)


PHYS = dict(T=0.85, eps=1e-3, kappa=1e-5, alpha=500.0, beta=1e-3)


@pytest.mark.parametrize("dim,N,nel", [
    (1, 1, (7,)), (1, 3, (64,)), (1, 6, (5,)),
    # several workgroups of the 1D tiles (83, 51, 42 elements) and a ragged tail
    (1, 2, (200,)), (1, 4, (130,)), (1, 5, (100,)),
    (2, 2, (5, 4)), (2, 4, (7, 6)), (2, 5, (3, 4)),
    (3, 1, (4, 3, 5)), (3, 2, (5, 3, 2)), (3, 3, (4, 3, 3)), (3, 4, (3, 4, 3)), (3, 5, (3, 2, 3)),
])
def test_rhs_parity_smooth(O, gpu, dim, N, nel):
    m, U = I.smooth_random(dim, N, nel, seed=11 + dim * 7 + N)
    s = _solver(gpu, m, **PHYS)
    R = s.rhs(U).cpu().numpy()
    Rc = O.rhs(_problem(O, m, **PHYS), U)
    _rhs_check(O, m, U, R, Rc, PHYS["alpha"])
    s.close()


@pytest.mark.parametrize("diss_c", [0, 1])
def test_rhs_parity_nonuniform(O, gpu, diss_c):
    g = np.random.Generator(np.random.PCG64(5))
    xb = [np.sort(np.concatenate([[0.0, 1.0], g.uniform(0.05, 0.95, 5)])) for _ in range(3)]
    m, U = I.smooth_random(3, 3, (6, 6, 6), seed=9, xbreaks=xb)
    kw = dict(PHYS, diss_c=diss_c)
    s = _solver(gpu, m, **kw)
    R = s.rhs(U).cpu().numpy()
    Rc = O.rhs(_problem(O, m, **kw), U)
    _rhs_check(O, m, U, R, Rc, kw["alpha"])
    s.close()


def test_rhs_parity_config_1d(O, gpu):
    m, U = I.slab_1d()
    s = _solver(gpu, m, **PHYS)
    R = s.rhs(U).cpu().numpy()
    Rc = O.rhs(_problem(O, m, **PHYS), U)
    _rhs_check(O, m, U, R, Rc, PHYS["alpha"])


@pytest.mark.parametrize("alpha", [500.0, 2000.0])
def test_rhs_parity_config_2d_full(O, gpu, alpha):
    """The 2D droplet workload at its full size (96 x 96 elements, N = 4,
    230,400 nodes): every node of the right-hand side against the oracle,
    in the launch shape the autotuner picks."""
    m, U = I.droplets_2d()
    phys = dict(PHYS, alpha=alpha)
    s = _solver(gpu, m, **phys)
    s.set_state(U)
    gpu.nsk_autotune(s.ctx, 2)
    R = s.rhs(U).cpu().numpy()
    Rc = O.rhs(_problem(O, m, **phys), U)
    _rhs_check(O, m, U, R, Rc, alpha)
    s.close()


def test_trajectory_1d_config(O, gpu):
    """64 elements, N=3, alpha=500: the full 2000-step run."""
    m, U = I.slab_1d()
    P = _problem(O, m, **PHYS)
    dt = O.dt(P, U, 0.5)
    s = _solver(gpu, m, **PHYS)
    s.set_state(U)
    dt_gpu = s.dt_estimate(0.5)
    assert abs(dt_gpu - dt) <= 1e-12 * dt
    s.rk_step(dt, 2000)
    got = s.get_state().cpu().numpy()
    ref = O.run(P, U, dt, 2000)
    rel = np.linalg.norm(got[0] - ref[0]) / np.linalg.norm(ref[0])
    assert rel <= TRAJ_TOL
    assert _relerr_per_var(got, ref) <= TRAJ_TOL


def test_planar_interface_sec411(O, gpu):
    """The planar interface of Sec. 4.1.1 (eps = 0.01, kappa = 1e-4,
    alpha = 100, beta = 0.01, N = 3, 100 elements on periodic (0, 1)) from
    off-equilibrium phase densities 0.40 / 1.70, its step limited by the
    viscous momentum bound.  The GPU trajectory equals the oracle's over the
    first 2000 steps; run on to t = 2 (about 65,000 steps) the energy never
    grows, the kinetic energy falls below 1e-6 and the bulk densities come
    within 1e-3 of the Maxwell densities, as in the oracle's own pin."""
    import torch

    rv, rl, _, _ = O.maxwell(0.85)
    E, kap = 100, 1e-4
    phys = dict(eps=0.01, kappa=kap, alpha=100.0, beta=0.01)
    P = O.Problem(dim=1, N=3, nel=(E, 1, 1), **phys)
    X = O.node_coords(P)[0]
    w = 2 * np.sqrt(kap)
    rho = 0.40 + 0.5 * (1.70 - 0.40) * (np.tanh((X - 0.3) / w) - np.tanh((X - 0.7) / w))
    U = np.stack([rho, 0 * rho, rho.copy()])
    s = gpu.Solver(dim=1, N=3, nel=(E,), stream=torch.cuda.Stream(), **phys)
    s.set_state(U)
    dt = O.dt(P, U, 0.5)
    assert abs(s.dt_estimate(0.5) - dt) <= 1e-12 * dt
    s.rk_step(dt, 2000)
    got = s.get_state().cpu().numpy()
    ref = O.run(P, U, dt, 2000)
    assert _relerr_per_var(got, ref) <= TRAJ_TOL
    nsteps = int(np.ceil(2.0 / dt))
    e_prev = s.diagnostics()["e_total"]
    done = 2000
    while done < nsteps:
        k = min(1000, nsteps - done)
        s.rk_step(dt, k)
        done += k
        e = s.diagnostics()["e_total"]
        assert e <= e_prev + 1e-12 * abs(e_prev), done
        e_prev = e
    d = s.diagnostics()
    assert d["status"] == 0 and d["e_kin"] < 1e-6
    fin = s.get_state().cpu().numpy()
    vap = fin[0][np.abs(X - 0.0) < 0.06].mean()
    liq = fin[0][np.abs(X - 0.5) < 0.06].mean()
    record("planar interface, |rho - Maxwell| in the bulk", max(abs(vap - rv), abs(liq - rl)), 1e-3)
    assert abs(vap - rv) < 1e-3 and abs(liq - rl) < 1e-3
    s.close()


def test_trajectory_2d_droplets_small(O, gpu):
    """2D droplet geometry on a coarser 24x24 mesh, N=4, 50 steps."""
    m, U = I.droplets_2d(nel=24)
    kw = dict(PHYS, alpha=2000.0)
    P = _problem(O, m, **kw)
    dt = O.dt(P, U, 0.5)
    s = _solver(gpu, m, **kw)
    s.set_state(U)
    s.rk_step(dt, 50)
    got = s.get_state().cpu().numpy()
    ref = O.run(P, U, dt, 50)
    assert _relerr_per_var(got, ref) <= TRAJ_TOL


def test_trajectory_3d_collision_small(O, gpu):
    """3D head-on collision geometry on 12x6x6 elements, N=4, 10 steps."""
    m, U = I.collision_3d(nel=(12, 6, 6), N=4, We=100.0)
    kw = dict(PHYS, alpha=1000.0)
    P = _problem(O, m, **kw)
    dt = O.dt(P, U, 0.5)
    s = _solver(gpu, m, **kw)
    s.set_state(U)
    s.rk_step(dt, 10)
    got = s.get_state().cpu().numpy()
    ref = O.run(P, U, dt, 10)
    assert _relerr_per_var(got, ref) <= TRAJ_TOL


def test_diagnostics_parity(O, gpu):
    m, U = I.smooth_random(2, 4, (6, 5), seed=21)
    s = _solver(gpu, m, **PHYS)
    s.set_state(U)
    d = s.diagnostics()
    dc = O.diagnostics(_problem(O, m, **PHYS), U)
    np.testing.assert_allclose(d["mass"], dc["mass"], rtol=1e-13, atol=1e-15)
    for k in ("e_kin", "e_total", "l2_rho_minus_c", "rho_min", "rho_max", "max_wavespeed"):
        assert d[k] == pytest.approx(dc[k], rel=1e-12), k
    assert d["nonfinite"] == 0 and d["status"] == 0


def test_nonphysical_state_flagged(gpu):
    m, U = I.smooth_random(1, 3, (8,), seed=2)
    U = U.copy()
    U[0, 3, 1] = np.nan
    s = _solver(gpu, m, **PHYS)
    s.set_state(U)
    d = s.diagnostics()
    assert d["nonfinite"] == 1 and d["status"] == gpu.NSK_ENONPHYS
    U[0, 3, 1] = 3.2
    s.set_state(U)
    d = s.diagnostics()
    assert d["nonfinite"] == 0 and d["status"] == gpu.NSK_ENONPHYS


def test_mass_conservation_gpu(gpu):
    m, U = I.slab_1d()
    s = _solver(gpu, m, **PHYS)
    s.set_state(U)
    m0 = s.diagnostics()["mass"]
    s.rk_step(4.6e-6, 500)
    m1 = s.diagnostics()["mass"]
    # only rho is conserved: momentum and c carry sources
    assert abs(m1[0] - m0[0]) <= 1e-13 * abs(m0[0])


def test_bitwise_determinism(gpu):
    m, U = I.smooth_random(3, 4, (6, 5, 4), seed=31)
    outs = []
    for _ in range(2):
        s = _solver(gpu, m, **dict(PHYS, alpha=1000.0))
        s.set_state(U)
        s.rk_step(2e-6, 7)
        outs.append(s.get_state().cpu().numpy())
        s.close()
    assert np.all(np.isfinite(outs[0]))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("dim,N,nel", [(1, 3, (37,)), (2, 4, (13, 11)), (3, 3, (7, 5, 3)), (3, 4, (5, 5, 3))])
def test_launch_shapes_bitwise_identical(gpu, dim, N, nel):
    """Every (elements-per-workgroup, element work order) launch shape gives
    the same bits, for ragged element counts that leave partial workgroups
    and partial tiles."""
    m, U = I.smooth_random(dim, N, nel, seed=40 + N)
    outs = []
    for variant in (0, 1):
        for order in range(6):
            s = _solver(gpu, m, **PHYS)
            gpu.nsk_set_tile(s.ctx, variant, order)
            s.set_state(U)
            s.rk_step(1e-6, 3)
            outs.append(s.get_state().cpu().numpy())
            s.close()
    assert np.all(np.isfinite(outs[0]))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_autotune_keeps_results(gpu):
    m, U = I.smooth_random(3, 4, (6, 5, 4), seed=8)
    s = _solver(gpu, m, **PHYS)
    s.set_state(U)
    variant, order, ms = gpu.nsk_autotune(s.ctx, 2)
    assert variant in (0, 1) and 0 <= order < 6 and all(x > 0 or x == -1 for x in ms)
    # the first shape within 1% of the fastest
    best = min(x for x in ms if x > 0)
    assert variant * 6 + order == next(k for k, x in enumerate(ms) if x > 0 and x <= best * 1.01)
    got = s.get_state().cpu().numpy()
    assert np.array_equal(got, U)  # autotuning does not touch the state
    s.close()


def test_autotune_skips_coinciding_variant(gpu):
    """At N = 4 in 3D both tile variants hold one element per workgroup (a
    125-node element's LDS does not fit twice in the 40 KB budget), so the
    tuner times variant 0 only, reports -1 for variant 1 and returns 0; with
    N = 2 (27 nodes) the variants differ and all six tiled orders of both
    are timed."""
    m, U = I.smooth_random(3, 4, (6, 5, 4), seed=9)
    s = _solver(gpu, m, **PHYS)
    s.set_state(U)
    variant, order, ms = gpu.nsk_autotune(s.ctx, 1)
    assert variant == 0 and all(x == -1 for x in ms[6:]) and all(x > 0 for x in ms[:6])
    s.close()
    m, U = I.smooth_random(3, 2, (6, 5, 4), seed=9)
    s = _solver(gpu, m, **PHYS)
    s.set_state(U)
    variant, order, ms = gpu.nsk_autotune(s.ctx, 1)
    assert all(x > 0 for x in ms)
    s.close()


def test_full_size_3d_sampled(O, gpu):
    """The 96x48x48, N=4 collision (27.6M nodes) on the GPU in the launch
    configuration the benchmark times; sampled elements are recomputed by the
    oracle on a 5x5x5-element periodic patch centred on each sample (the
    right-hand side of an element depends on elements at most two away)."""
    import torch

    nel = (96, 48, 48)
    m, U = I.collision_3d(nel=nel, N=4, We=100.0)
    kw = dict(PHYS, alpha=1000.0)
    s = _solver(gpu, m, **kw)
    Ut = torch.from_numpy(U.reshape(-1)).to("cuda:0")
    R = torch.empty_like(Ut)
    gpu.nsk_rhs(s.ctx, Ut.data_ptr(), R.data_ptr(), 0.0)
    torch.cuda.synchronize()
    R = R.reshape(U.shape)
    g = np.random.Generator(np.random.PCG64(77))
    # bias samples towards the interface and the droplet motion
    rho = U[0]
    inter = np.where((rho.max(axis=1) > 1.0) & (rho.min(axis=1) < 1.0))[0]
    samples = list(g.choice(inter, 12, replace=False)) + list(g.integers(0, m.nelem, 4))
    h = [(m.hi[d] - m.lo[d]) / nel[d] for d in range(3)]
    scales = term_scales(O, 4, min(h), U, kw["alpha"])
    for e in samples:
        ex, ey, ez = e % nel[0], (e // nel[0]) % nel[1], e // (nel[0] * nel[1])
        idx = [[(c + k) % nel[d] for k in range(-2, 3)] for d, c in enumerate((ex, ey, ez))]
        patch = np.empty((5, 125, 125))
        pe = 0
        for kz in idx[2]:
            for ky in idx[1]:
                for kx in idx[0]:
                    patch[:, pe, :] = U[:, kx + nel[0] * (ky + nel[1] * kz), :]
                    pe += 1
        P = O.Problem(dim=3, N=4, nel=(5, 5, 5), lo=(0, 0, 0), hi=(5 * h[0], 5 * h[1], 5 * h[2]), **kw)
        Rp = O.rhs(P, patch)
        centre = 2 + 5 * (2 + 5 * 2)
        got = R[:, e, :].cpu().numpy()
        ref = Rp[:, centre, :]
        ulps = rhs_err_ulps(got, ref, scales)
        assert ulps <= RHS_ULPS, (e, ulps)
    s.close()


def _patch(U, nel, e, r):
    """The (2r+1)^3-element block of U centred on element e (periodic)."""
    ex, ey, ez = e % nel[0], (e // nel[0]) % nel[1], e // (nel[0] * nel[1])
    ix = [(ex + k) % nel[0] for k in range(-r, r + 1)]
    iy = [(ey + k) % nel[1] for k in range(-r, r + 1)]
    iz = [(ez + k) % nel[2] for k in range(-r, r + 1)]
    ids = [x + nel[0] * (y + nel[1] * z) for z in iz for y in iy for x in ix]
    return U[:, ids, :]


def test_full_size_3d_one_step_sampled(O, gpu):
    """One LSRK4(5) step of the 96x48x48, N=4 collision (27.6M nodes) on the
    GPU in the launch shape the benchmark times (autotuned), FP64.  A stage
    reaches elements at most two away (lifting, then the neighbours' lifted
    gradients), so the five stages of a step reach ten: sampled elements are
    recomputed by the oracle on the periodic 23x23x23-element block centred on
    each, whose wrapped boundary is eleven elements away.  Errors are relative
    to each variable's largest magnitude on the whole mesh after the step."""
    import torch

    nel = (96, 48, 48)
    r = 11
    m, U = I.collision_3d(nel=nel, N=4, We=100.0)
    kw = dict(PHYS, alpha=1000.0)
    s = _solver(gpu, m, **kw)
    s.set_state(torch.from_numpy(U.reshape(-1)).to("cuda:0"))
    gpu.nsk_autotune(s.ctx, 2)
    dt = s.dt_estimate(0.5)
    s.rk_step(dt, 1)
    got = s.get_state()
    scale = [float(torch.max(torch.abs(got[v]))) for v in range(5)]
    got = got.cpu().numpy()
    s.close()
    g = np.random.Generator(np.random.PCG64(78))
    rho = U[0]
    inter = np.where((rho.max(axis=1) > 1.0) & (rho.min(axis=1) < 1.0))[0]
    samples = list(g.choice(inter, 2, replace=False)) + list(g.integers(0, m.nelem, 1))
    h = [(m.hi[d] - m.lo[d]) / nel[d] for d in range(3)]
    w = 2 * r + 1
    P = O.Problem(dim=3, N=4, nel=(w, w, w), lo=(0, 0, 0), hi=(w * h[0], w * h[1], w * h[2]), **kw)
    centre = r + w * (r + w * r)
    for e in samples:
        ref = O.run(P, _patch(U, nel, e, r), dt, 1)[:, centre, :]
        err = _relerr_per_var(got[:, e, :], ref, scale)
        assert err <= TRAJ_TOL, (e, err)
