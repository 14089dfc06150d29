"""HLLC flux (flux = 1) on the GPU against the FP64 oracle: right-hand side
within the round-off bound of the Rusanov tests (the HLLC flux is
continuous where it switches branches, so different rounding on the two
sides cannot open a gap), trajectories, launch-shape independence and the
mixed-precision form."""
import numpy as np
import pytest

from paper_1912_12059_amd import inputs as I
from test_gpu_parity import PHYS, TRAJ_TOL, _problem, _relerr_per_var, _rhs_check, _solver
from tolerances import RHS_ULPS, rhs_err_ulps, term_scales

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,N,nel", [(1, 3, (9,)), (2, 4, (7, 5)), (3, 3, (4, 3, 5)), (3, 4, (3, 4, 3))])
@pytest.mark.parametrize("diss_c", [0, 1])
def test_hllc_rhs_parity(O, gpu, dim, N, nel, diss_c):
    m, U = I.smooth_random(dim, N, nel, seed=70 + dim + N, vmax=0.5)
    phys = dict(PHYS, diss_c=diss_c)
    s = _solver(gpu, m, flux=1, **phys)
    R = s.rhs(U).cpu().numpy()
    Rc = O.rhs(_problem(O, m, flux=1, **phys), U)
    _rhs_check(O, m, U, R, Rc, PHYS["alpha"])
    s.close()


@pytest.mark.parametrize("diss_c", [0, 1])
def test_hllc_rhs_parity_nonuniform(O, gpu, diss_c):
    """Random element breakpoints in every direction."""
    g = np.random.Generator(np.random.PCG64(13))
    xb = [np.sort(np.concatenate([[0.0, 1.0], g.uniform(0.05, 0.95, 5)])) for _ in range(3)]
    m, U = I.smooth_random(3, 3, (6, 6, 6), seed=19, xbreaks=xb, vmax=0.5)
    phys = dict(PHYS, diss_c=diss_c)
    s = _solver(gpu, m, flux=1, **phys)
    R = s.rhs(U).cpu().numpy()
    Rc = O.rhs(_problem(O, m, flux=1, **phys), U)
    _rhs_check(O, m, U, R, Rc, PHYS["alpha"])
    s.close()


def test_hllc_rhs_parity_collision(O, gpu):
    """Moving droplets: contacts with both signs of S* inside the interfaces."""
    m, U = I.collision_3d(nel=(12, 6, 6), N=4, We=100.0, hi=(2.0, 1.0, 1.0), impact=0.1)
    phys = dict(PHYS, alpha=1000.0)
    s = _solver(gpu, m, flux=1, **phys)
    R = s.rhs(U).cpu().numpy()
    Rc = O.rhs(_problem(O, m, flux=1, **phys), U)
    _rhs_check(O, m, U, R, Rc, phys["alpha"])
    s.close()


def test_hllc_trajectory_1d_config(O, gpu):
    m, U = I.slab_1d()
    s = _solver(gpu, m, flux=1, **PHYS)
    s.set_state(U)
    dt = s.dt_estimate(0.5)
    s.rk_step(dt, 500)
    got = s.get_state().cpu().numpy()
    ref = O.run(_problem(O, m, flux=1, **PHYS), U, dt, 500)
    assert _relerr_per_var(got, ref) <= TRAJ_TOL
    s.close()


@pytest.mark.parametrize("dim,N,nel", [(2, 4, (13, 11)), (3, 4, (5, 5, 3))])
def test_hllc_launch_shapes_bitwise_identical(gpu, dim, N, nel):
    m, U = I.smooth_random(dim, N, nel, seed=90 + N)
    outs = []
    for variant in (0, 1):
        for order in (0, 2, 5):
            s = _solver(gpu, m, flux=1, **PHYS)
            gpu.nsk_set_tile(s.ctx, variant, order)
            s.set_state(U)
            s.rk_step(1e-6, 3)
            outs.append(s.get_state().cpu().numpy())
            s.close()
    assert np.all(np.isfinite(outs[0]))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_hllc_mixed_precision(O, gpu):
    """Mixed precision with HLLC: 100 steps of a small collision against the
    FP64 oracle, the bound of the Rusanov mixed test."""
    m, U = I.collision_3d(nel=(12, 6, 6), N=4, We=100.0, hi=(2.0, 1.0, 1.0))
    phys = dict(PHYS, alpha=1000.0)
    s = _solver(gpu, m, flux=1, precision=1, **phys)
    s.set_state(U)
    dt = s.dt_estimate(0.5)
    s.rk_step(dt, 100)
    got = s.get_state().cpu().numpy()
    ref = O.run(_problem(O, m, flux=1, **phys), U, dt, 100)
    rel = np.linalg.norm(got[0] - ref[0]) / np.linalg.norm(ref[0])
    print(f"\nHLLC mixed vs FP64 oracle, rel L2(rho) after 100 steps: {rel:.3e}")
    assert rel <= 1e-6
    s.close()


def test_hllc_full_size_3d_sampled(O, gpu):
    """The 96x48x48, N = 4 collision (27.6M nodes) with the HLLC flux on the
    GPU; sampled elements (most at the interfaces, where contacts of both
    signs occur) are recomputed by the oracle on a 5x5x5-element periodic
    patch centred on each (an element's right-hand side depends on elements
    at most two away)."""
    import torch

    nel = (96, 48, 48)
    m, U = I.collision_3d(nel=nel, N=4, We=100.0)
    kw = dict(PHYS, alpha=1000.0)
    s = _solver(gpu, m, flux=1, **kw)
    Ut = torch.from_numpy(U.reshape(-1)).to("cuda:0")
    R = torch.empty_like(Ut)
    gpu.nsk_rhs(s.ctx, Ut.data_ptr(), R.data_ptr(), 0.0)
    torch.cuda.synchronize()
    R = R.reshape(U.shape)
    s.close()
    g = np.random.Generator(np.random.PCG64(83))
    rho = U[0]
    inter = np.where((rho.max(axis=1) > 1.0) & (rho.min(axis=1) < 1.0))[0]
    samples = list(g.choice(inter, 12, replace=False)) + list(g.integers(0, m.nelem, 4))
    h = [(m.hi[d] - m.lo[d]) / nel[d] for d in range(3)]
    scales = term_scales(O, 4, min(h), U, kw["alpha"])
    centre = 2 + 5 * (2 + 5 * 2)
    for e in samples:
        ex, ey, ez = e % nel[0], (e // nel[0]) % nel[1], e // (nel[0] * nel[1])
        near = [((ex + kx) % nel[0]) + nel[0] * (((ey + ky) % nel[1]) + nel[1] * ((ez + kz) % nel[2]))
                for kz in range(-2, 3) for ky in range(-2, 3) for kx in range(-2, 3)]
        patch = np.ascontiguousarray(U[:, near, :])
        P = O.Problem(dim=3, N=4, nel=(5, 5, 5), lo=(0, 0, 0), hi=(5 * h[0], 5 * h[1], 5 * h[2]), flux=1, **kw)
        Rp = O.rhs(P, patch)
        ulps = rhs_err_ulps(R[:, e, :].cpu().numpy(), Rp[:, centre, :], scales)
        assert ulps <= RHS_ULPS, (e, ulps)



def test_merging_droplets_sec42(O, gpu):
    """The first 2D case of Sec. 4.2: droplets of radii 0.2 and 0.1 centred
    at (0.4, 0.5) and (0.7, 0.5), touching at x = 0.6, between the Maxwell
    densities (alpha = 100, beta = 0.001, eps = 0.01, kappa = 1e-4, N = 3,
    100^2 elements, HLLC flux).  The first 100 steps equal the oracle's; run on
    to t = 0.1 the liquid neck at x = 0.6 widens at every check as the two
    merge, the total energy never grows and mass stays exact."""
    import torch

    E, kap = 100, 1e-4
    rv, rl, _, _ = O.maxwell(0.85)
    phys = dict(alpha=100.0, beta=0.001, eps=0.01, kappa=kap, flux=1)
    P = O.Problem(dim=2, N=3, nel=(E, E, 1), **phys)
    x, y = O.node_coords(P)[:2]
    w = 2 * np.sqrt(kap)
    rho = rl + sum(0.5 * (rv - rl) * np.tanh((np.hypot(x - cx, y - cy) - r) / w)
                   for cx, cy, r in ((0.4, 0.5, 0.2), (0.7, 0.5, 0.1)))
    U = np.stack([rho, 0 * rho, 0 * rho, rho.copy()])
    s = gpu.Solver(dim=2, N=3, nel=(E, E), stream=torch.cuda.Stream(), **phys)
    s.set_state(U)
    dt = O.dt(P, U, 0.5)
    assert abs(s.dt_estimate(0.5) - dt) <= 1e-12 * dt
    s.rk_step(dt, 100)
    assert _relerr_per_var(s.get_state().cpu().numpy(), O.run(P, U, dt, 100)) <= TRAJ_TOL
    mid = 0.5 * (rl + rv)
    line = np.abs(x - 0.6) < 0.004

    def neck(V):
        return np.ptp(y[line][V[0][line] > mid])

    m0 = s.diagnostics()["mass"][0]
    widths, energies = [neck(U)], [s.diagnostics()["e_total"]]
    t = 100 * dt
    for tk in (0.02, 0.05, 0.1):
        n = int(round((tk - t) / dt))
        s.rk_step(dt, n)
        t += n * dt
        d = s.diagnostics()
        assert d["status"] == 0 and abs(d["mass"][0] / m0 - 1) < 1e-13
        widths.append(neck(s.get_state().cpu().numpy().reshape(U.shape)))
        energies.append(d["e_total"])
    assert all(b > a for a, b in zip(widths, widths[1:])), widths
    assert widths[-1] > 1.25 * widths[0], widths
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(energies, energies[1:])), energies
    s.close()
