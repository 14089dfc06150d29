"""GPU edge cases: degenerate periodic grids (one element in a direction,
the element its own neighbour on both sides; a single element), a constant
state, and calls that do nothing (zero steps), for both models and every
numerical flux, against the oracle through the C ABI at the right-hand-side
bar of tests/tolerances.py."""
import numpy as np
import pytest

from paper_1912_12059_amd import inputs as I
from tolerances import RHS_ULPS, rhs_err_ulps, term_scales, term_scales_nsk

pytestmark = pytest.mark.gpu


def _setup(O, gpu, dim, N, nel, model, flux, seed=3):
    m, U = I.smooth_random(dim, N, nel, seed=seed, rho_range=(1.5, 1.9))
    kw = dict(eps=1e-2, kappa=1e-4)
    if model == 1:
        U = np.ascontiguousarray(U[:-1])
        s = gpu.Solver(dim=dim, N=N, nel=tuple(nel), model=1, flux=2, **kw)
    else:
        kw.update(alpha=500.0, beta=1e-2)
        s = gpu.Solver(dim=dim, N=N, nel=tuple(nel), flux=flux, **kw)
    P = O.Problem(dim=dim, N=N, nel=tuple(nel) + (1,) * (3 - dim), model=model, flux=flux, **kw)
    return m, U, s, P, kw


def _check(O, m, P, U, R, Rc, model, kw):
    if model == 1:
        sc = term_scales_nsk(O, P, U, kw["kappa"], kw["eps"])
    else:
        h = min(float(np.diff(P.breaks(d)).min()) for d in range(P.dim))
        sc = term_scales(O, P.N, h, U, kw["alpha"])
    ulps = rhs_err_ulps(R, Rc, sc)
    assert ulps <= RHS_ULPS, f"{ulps:.1f} ulps"


@pytest.mark.parametrize("model,flux", [(0, 0), (0, 1), (1, 2)])
@pytest.mark.parametrize("dim,N,nel", [(1, 3, (1,)), (2, 4, (1, 1)), (2, 2, (1, 5)), (3, 2, (1, 1, 1)),
                                       (3, 4, (1, 1, 1)), (3, 3, (2, 1, 3))])
def test_degenerate_grids_parity(O, gpu, model, flux, dim, N, nel):
    m, U, s, P, kw = _setup(O, gpu, dim, N, nel, model, flux)
    R = s.rhs(U).cpu().numpy()
    _check(O, m, P, U, R, O.rhs(P, U), model, kw)
    s.close()


@pytest.mark.parametrize("model,flux", [(0, 0), (0, 1), (1, 2)])
def test_degenerate_grid_trajectory(O, gpu, model, flux):
    """A 3D grid with one element in y: 20 steps against the oracle."""
    m, U, s, P, kw = _setup(O, gpu, 3, 3, (3, 1, 2), model, flux)
    dt = O.dt(P, U, 0.5)
    s.set_state(U)
    assert abs(s.dt_estimate(0.5) - dt) <= 1e-12 * dt
    s.rk_step(dt, 20)
    got = s.get_state().cpu().numpy()
    ref = O.run(P, U, dt, 20)
    for v in range(ref.shape[0]):
        assert np.abs(got[v] - ref[v]).max() <= 1e-10 * max(np.abs(ref[v]).max(), 1e-300)
    s.close()


@pytest.mark.parametrize("model,flux", [(0, 0), (0, 1), (1, 2)])
def test_constant_state_is_steady(gpu, model, flux):
    """A uniform state at rest: every term of R vanishes up to round-off, and
    100 steps leave it unchanged to round-off."""
    dim, N, nel = 3, 3, (3, 2, 2)
    nv = dim + (1 if model == 1 else 2)
    U = np.zeros((nv, 12, (N + 1) ** dim))
    U[0] = 1.8
    if model == 0:
        U[-1] = 1.8
    kw = dict(eps=1e-2, kappa=1e-4)
    if model == 1:
        s = gpu.Solver(dim=dim, N=N, nel=nel, model=1, flux=2, **kw)
    else:
        s = gpu.Solver(dim=dim, N=N, nel=nel, flux=flux, alpha=500.0, beta=1e-2, **kw)
    R = s.rhs(U).cpu().numpy()
    assert np.abs(R).max() <= 1e-9  # round-off of terms of size ~ (2/h) C_D p_alpha ~ 5e4
    s.set_state(U)
    s.rk_step(s.dt_estimate(0.5), 100)
    assert np.abs(s.get_state().cpu().numpy() - U).max() <= 1e-12
    s.close()


def test_zero_steps_leave_the_state(gpu):
    m, U = I.smooth_random(2, 3, (4, 3), seed=5, rho_range=(1.5, 1.9))
    s = gpu.Solver(dim=2, N=3, nel=(4, 3), alpha=500.0, beta=1e-2, eps=1e-2, kappa=1e-4)
    s.set_state(U)
    s.rk_step(1e-4, 0)
    assert np.array_equal(s.get_state().cpu().numpy(), U)
    st = s.esdirk_step(1e-3, 0)
    assert st["steps"] == 0 and st["rhs_evals"] == 0
    assert np.array_equal(s.get_state().cpu().numpy(), U)
    s.close()


@pytest.mark.parametrize("model", [0, 1])
def test_dt_estimate_viscosity_limited(O, gpu, model):
    """Where the viscous momentum bound is the active one (eps = 0.01 on 128
    elements, a slab of liquid in vapour), the library's step equals the
    oracle's: the rate (4/3) eps / rho_min on both sides, for model II and
    the original NSK path.  A state with a non-positive density gets
    NSK_ENONPHYS."""
    from paper_1912_12059_amd import inputs as I

    nel = (128,)
    m, U = I.slab_1d(nel=nel[0])
    # kappa = 1e-5 keeps the original path's capillary bound below the viscous one
    kw = dict(eps=0.01, kappa=1e-4 if model == 0 else 1e-5)
    if model == 0:
        kw.update(alpha=100.0, beta=0.01)
        s = gpu.Solver(dim=1, N=3, nel=nel, **kw)
        P = O.Problem(dim=1, N=3, nel=(nel[0], 1, 1), **kw)
    else:
        U = U[:2]
        s = gpu.Solver(dim=1, N=3, nel=nel, model=1, **kw)
        P = O.Problem(dim=1, N=3, nel=(nel[0], 1, 1), model=1, **kw)
    s.set_state(U)
    dt = O.dt(P, U, 0.5)
    assert abs(s.dt_estimate(0.5) - dt) <= 1e-12 * dt
    h = 1.0 / nel[0]
    assert dt == pytest.approx(0.5 / (49 * (4.0 / 3.0) * 0.01 / U[0].min() / h ** 2), rel=1e-12)
    Ubad = U.copy()
    Ubad[0].flat[5] = -0.1
    s.set_state(Ubad)
    with pytest.raises(gpu.NskError) as e:
        s.dt_estimate(0.5)
    assert e.value.code == gpu.NSK_ENONPHYS
    s.close()
