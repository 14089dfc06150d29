"""GPU implicit stepping (ESDIRK4(6) with Jacobian-free Newton-GMRES,
nsk_esdirk_step) against the oracle's ESDIRK4(6) with dense Newton stage
solves, through the C ABI.

Both solve the same stage equations; the GPU stops at a relative stage
residual of 1e-13 and the oracle at machine precision, so after a few steps
the states agree to about 1e-12 relative; the bar written here is 1e-9 per
variable (relative to the variable's largest value)."""
import numpy as np
import pytest

from oracle import esdirk as E
from paper_1912_12059_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-9
TIGHT = dict(newton_tol=1e-13, newton_max=30, gmres_rtol=1e-8, gmres_m=40)


def _relerr(a, b):
    a = np.asarray(a).reshape(b.shape)
    return max(np.abs(a[v] - b[v]).max() / max(np.abs(b[v]).max(), 1e-300) for v in range(b.shape[0]))


def _solver(gpu, m, **kw):
    return gpu.Solver(dim=m.dim, N=m.N, nel=tuple(m.nel), lo=tuple(m.lo) + (0.0,) * 3,
                      hi=tuple(m.hi) + (1.0,) * 3, xbreaks=m.xbreaks, **kw)


def _problem(O, m, **kw):
    nel = tuple(m.nel) + (1,) * (3 - len(m.nel))
    hi = tuple(m.hi) + (1.0,) * (3 - len(m.hi))
    return O.Problem(dim=m.dim, N=m.N, nel=nel, hi=hi, xbreaks=m.xbreaks, **kw)


def test_esdirk_parity_nsk_1d(O, gpu):
    """Original NSK path, 1D, 8 elements, N = 2, liquid phase, 4 steps of a
    step 3.5 times the explicit limit."""
    m, U = I.smooth_random(1, 2, (8,), seed=4, rho_range=(1.6, 1.9))
    U = np.ascontiguousarray(U[:-1])
    kw = dict(eps=1e-2, kappa=1e-4)
    P = _problem(O, m, model=1, **kw)
    dt = 0.02
    ref = E.run(P, U, dt, 4)
    s = _solver(gpu, m, model=1, flux=2, **kw)
    s.set_state(U)
    st = s.esdirk_step(dt, 4, **TIGHT)
    assert st["converged"] == 1 and st["steps"] == 4
    assert _relerr(s.get_state().cpu().numpy(), ref) <= TOL
    s.close()


@pytest.mark.parametrize("precond,basis_fp32,reorth_tol", [(0, 0, 0.5), (1, 0, 0.5), (1, 1, 0.5), (1, 1, 0.0)])
def test_esdirk_parity_model2_stiff_1d(O, gpu, precond, basis_fp32, reorth_tol):
    """Model II with the stiff relaxation source (alpha/beta = 5e5), 1D,
    10 elements, N = 2: 3 steps of 50 times the explicit step, with and
    without the source preconditioner, with an FP64 and an FP32 Krylov basis,
    and with a single Gram-Schmidt pass (the Newton residuals stay FP64, so
    every variant converges to the same stages)."""
    m, U = I.smooth_random(1, 2, (10,), seed=6, rho_range=(1.6, 1.9), dc=0.0)
    kw = dict(eps=1e-2, kappa=1e-4, alpha=500.0, beta=1e-3)
    P = _problem(O, m, **kw)
    dt = 50 * O.dt(P, U, 0.5)
    ref = E.run(P, U, dt, 3)
    s = _solver(gpu, m, **kw)
    s.set_state(U)
    st = s.esdirk_step(dt, 3, precond=precond, basis_fp32=basis_fp32, reorth_tol=reorth_tol, **TIGHT)
    assert st["converged"] == 1
    assert _relerr(s.get_state().cpu().numpy(), ref) <= TOL
    s.close()


def test_esdirk_parity_model2_hllc_1d(O, gpu):
    """Model II with the HLLC flux, 1D, 10 elements, N = 2, both phases:
    3 steps of 20 times the explicit step (the flux's branches are the same
    on both sides; the finite-difference Jacobian-vector products see the
    branch of the state they perturb)."""
    m, U = I.smooth_random(1, 2, (10,), seed=9)
    kw = dict(eps=1e-2, kappa=1e-4, alpha=500.0, beta=1e-2)
    P = _problem(O, m, flux=1, **kw)
    dt = 20 * O.dt(P, U, 0.5)
    ref = E.run(P, U, dt, 3)
    s = _solver(gpu, m, flux=1, **kw)
    s.set_state(U)
    st = s.esdirk_step(dt, 3, **TIGHT)
    assert st["converged"] == 1
    assert _relerr(s.get_state().cpu().numpy(), ref) <= TOL
    s.close()


@pytest.mark.parametrize("dim,N,nel", [(2, 2, (4, 3)), (3, 1, (2, 2, 2))])
def test_esdirk_parity_model2_multid(O, gpu, dim, N, nel):
    """Model II in 2D and 3D across both phases, 2 steps of 20 times the
    explicit step."""
    m, U = I.smooth_random(dim, N, nel, seed=12 + dim)
    kw = dict(eps=1e-2, kappa=1e-4, alpha=500.0, beta=1e-2)
    P = _problem(O, m, **kw)
    dt = 20 * O.dt(P, U, 0.5)
    ref = E.run(P, U, dt, 2)
    s = _solver(gpu, m, **kw)
    s.set_state(U)
    st = s.esdirk_step(dt, 2, precond=1, **TIGHT)
    assert st["converged"] == 1
    assert _relerr(s.get_state().cpu().numpy(), ref) <= TOL
    s.close()


def test_esdirk_preconditioner_cuts_krylov_iterations(gpu):
    """The node-local source preconditioner gives the same solution (within
    the solver tolerance) with fewer Jacobian-vector products."""
    m, U = I.collision_3d(nel=(12, 6, 6), N=4, We=100.0)
    kw = dict(eps=1e-3, kappa=1e-5, alpha=1000.0, beta=1e-3)
    out, its = [], []
    for pc in (0, 1):
        s = _solver(gpu, m, **kw)
        s.set_state(U)
        dt = 20 * s.dt_estimate(0.5)
        st = s.esdirk_step(dt, 1, precond=pc, newton_tol=1e-10, gmres_rtol=1e-4, gmres_m=40)
        assert st["converged"] == 1
        out.append(s.get_state().cpu().numpy())
        its.append(st["gmres_iters"])
        s.close()
    assert its[1] < its[0], its
    assert _relerr(out[1], out[0]) <= 1e-7


@pytest.mark.parametrize("basis_fp32", [0, 1])
def test_esdirk_matches_explicit_on_3d_collision(gpu, basis_fp32):
    """The 3D collision geometry (24x12x12, N = 4): 2 implicit steps of 25
    times the explicit step against 50 explicit LSRK4(5) steps; both
    integrators are fourth order, so the two states differ by the time
    discretisation error only."""
    m, U = I.collision_3d(nel=(24, 12, 12), N=4, We=100.0)
    kw = dict(eps=1e-3, kappa=1e-5, alpha=1000.0, beta=1e-3)
    s = _solver(gpu, m, **kw)
    s.set_state(U)
    dte = s.dt_estimate(0.5)
    s.rk_step(dte, 50)
    ref = s.get_state().cpu().numpy()
    s.set_state(U)
    st = s.esdirk_step(25 * dte, 2, precond=1, newton_tol=1e-10, gmres_rtol=1e-4, gmres_m=40, basis_fp32=basis_fp32)
    assert st["converged"] == 1
    got = s.get_state().cpu().numpy()
    rel = np.linalg.norm(got[0] - ref[0]) / np.linalg.norm(ref[0])
    assert rel < 1e-6, rel
    s.close()


def test_esdirk_bitwise_reproducible(gpu):
    m, U = I.smooth_random(3, 3, (4, 3, 3), seed=21, rho_range=(1.6, 1.9))
    kw = dict(eps=1e-2, kappa=1e-4, alpha=500.0, beta=1e-3)
    outs = []
    for _ in range(2):
        s = _solver(gpu, m, **kw)
        s.set_state(U)
        s.esdirk_step(20 * s.dt_estimate(0.5), 2, precond=1)
        outs.append(s.get_state().cpu().numpy())
        s.close()
    assert np.all(np.isfinite(outs[0])) and np.array_equal(outs[0], outs[1])


def test_esdirk_reports_non_convergence(gpu):
    """A stage that misses the tolerance within newton_max corrections ends
    the call with NSK_ENOCONV and leaves the state at the last completed step."""
    m, U = I.smooth_random(1, 3, (16,), seed=2, rho_range=(1.6, 1.9), dc=0.0)
    kw = dict(eps=1e-2, kappa=1e-4, alpha=500.0, beta=1e-3)
    s = _solver(gpu, m, **kw)
    s.set_state(U)
    dt = 200 * s.dt_estimate(0.5)
    with pytest.raises(gpu.NskError) as e:
        s.esdirk_step(dt, 3, newton_tol=1e-14, newton_max=1, gmres_rtol=0.5, gmres_m=2)
    assert e.value.code == gpu.NSK_ENOCONV
    assert e.value.stats["converged"] == 0 and e.value.stats["steps"] == 0
    assert np.array_equal(s.get_state().cpu().numpy(), U.reshape(s.shape))
    s.close()
