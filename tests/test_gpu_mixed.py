"""Mixed-precision form against the FP64 oracle.

The mixed form evaluates fluxes, traces, the volume and surface integrals
and the lifted gradients in FP32, and keeps FP64 for the state and the
Runge-Kutta register, the relaxation source alpha rho grad c and
(alpha/beta)(rho - c), and the Van-der-Waals EoS inside the spinodal band.

Bounds (derived from the arithmetic): the right-hand side is a sum of O(10)
terms each rounded at 2^-24 relative to the largest term, so per variable
|R_mixed - R_fp64| <= MIXED_ULPS * 2^-24 * (term scale).  A trajectory adds
at most dt times that per step, and a step inside the stability region does
not amplify earlier differences, so the relative L2 error of rho after time
t is at most 2 t MIXED_ULPS 2^-24 s_rho / rms(rho) (tolerances.mixed_traj_bound;
the factor 2 allows for physical growth).  The achieved errors are recorded
next to that bound.
"""
import numpy as np
import pytest

from paper_1912_12059_amd import inputs as I
from tolerances import MIXED_ULPS, mixed_traj_bound, record, term_scales

pytestmark = pytest.mark.gpu
PHYS = dict(T=0.85, eps=1e-3, kappa=1e-5, alpha=1000.0, beta=1e-3)


def _problem(O, m, **kw):
    nel = tuple(m.nel) + (1,) * (3 - len(m.nel))
    lo = tuple(m.lo) + (0.0,) * (3 - len(m.lo))
    hi = tuple(m.hi) + (1.0,) * (3 - len(m.hi))
    return O.Problem(dim=m.dim, N=m.N, nel=nel, lo=lo, hi=hi, **kw)


def _solver(gpu, m, **kw):
    return gpu.Solver(dim=m.dim, N=m.N, nel=tuple(m.nel), lo=tuple(m.lo) + (0.0,) * 3,
                      hi=tuple(m.hi) + (1.0,) * 3, **kw)


def _l2_rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dim,N,nel", [(1, 3, (64,)), (2, 4, (8, 7)), (3, 4, (5, 4, 3)), (3, 3, (6, 5, 4)),
                                       # low and high degrees: several workgroups and a ragged tail
                                       (1, 5, (100,)), (1, 6, (90,)), (2, 1, (9, 11)), (2, 2, (9, 7))])
def test_mixed_rhs_within_fp32_rounding(O, gpu, dim, N, nel):
    m, U = I.smooth_random(dim, N, nel, seed=60 + N)
    s = _solver(gpu, m, precision=1, **PHYS)
    R = s.rhs(U).cpu().numpy()
    Rc = O.rhs(_problem(O, m, **PHYS), U)
    h = min(float(np.diff(m.breaks(d)).min()) for d in range(dim))
    scales = term_scales(O, N, h, U, PHYS["alpha"])
    err = np.abs(R - Rc).reshape(U.shape[0], -1).max(axis=1) / (2.0 ** -24 * scales)
    record("mixed rhs, FP32 ulps of term scale", err.max(), MIXED_ULPS)
    assert err.max() <= MIXED_ULPS, err
    s.close()


def test_mixed_source_term_is_fp64(O, gpu):
    """Uniform rho and c with rho - c = 3.1e-7, about 2.6 FP32 ulps at 1.2:
    R_c = (alpha/beta)(rho - c) plus FP32 noise of the surface terms.  The
    largest noise is the Rusanov jump lambda (c_R - c_L) / 2 of two FP32
    traces of the same constant taken with mirrored weights: about
    lambda * 2^-24 * c * (2/h) * max|L|/w ~ 2e-4 absolute, 6e-4 relative.
    An FP32 evaluation of (alpha/beta)(rho - c) would be off by 15-25 %."""
    m = I.Mesh(3, 3, (4, 3, 3))
    U = np.zeros((5, m.nelem, m.nnode))
    U[0] = 1.2
    U[4] = 1.2 - 3.1e-7
    s = _solver(gpu, m, precision=1, **PHYS)
    R = s.rhs(U).cpu().numpy()
    want = PHYS["alpha"] / PHYS["beta"] * (1.2 - (1.2 - 3.1e-7))
    np.testing.assert_allclose(R[4], want, rtol=5e-3)
    s.close()


def test_mixed_trajectory_3d_collision(O, gpu):
    """3D collision geometry, 12x6x6 elements, N=4, 100 steps."""
    m, U = I.collision_3d(nel=(12, 6, 6), N=4, We=100.0)
    P = _problem(O, m, **PHYS)
    dt = O.dt(P, U, 0.5)
    s = _solver(gpu, m, precision=1, **PHYS)
    s.set_state(U)
    s.rk_step(dt, 100)
    got = s.get_state().cpu().numpy()
    ref = O.run(P, U, dt, 100)
    err = _l2_rel(got[0], ref[0])
    bound = mixed_traj_bound(O, 4, min(np.diff(m.breaks(d)).min() for d in range(3)), U, PHYS["alpha"], 100 * dt)
    record("mixed vs FP64 oracle, rel L2(rho)", err, bound)
    assert err <= bound
    s.close()


def test_mixed_trajectory_1d_config(O, gpu):
    """The 1D slab workload, 2000 steps."""
    m, U = I.slab_1d()
    kw = dict(PHYS, alpha=500.0)
    P = _problem(O, m, **kw)
    dt = O.dt(P, U, 0.5)
    s = _solver(gpu, m, precision=1, **kw)
    s.set_state(U)
    s.rk_step(dt, 2000)
    got = s.get_state().cpu().numpy()
    ref = O.run(P, U, dt, 2000)
    err = _l2_rel(got[0], ref[0])
    bound = mixed_traj_bound(O, 3, float(np.diff(m.breaks(0)).min()), U, kw["alpha"], 2000 * dt)
    record("mixed vs FP64 oracle, rel L2(rho)", err, bound)
    assert err <= bound
    s.close()


def test_mixed_full_size_3d_mass_and_error(gpu):
    """The 96x48x48, N=4 collision (alpha = 1000, We = 100), 200 steps in both
    forms from the same state.  Face fluxes are computed identically by both
    elements, so mass moves only through FP32 rounding inside elements; the
    relative drift stays below 1e-10.  The mixed run stays within the
    derived trajectory bound (relative L2 of rho) of the FP64 run."""
    import torch

    from oracle import oracle as O

    m, U = I.collision_3d(nel=(96, 48, 48), N=4, We=100.0, hi=(2.0, 1.0, 1.0))
    U0 = torch.from_numpy(U.reshape(-1)).to("cuda:0")
    h_min = min(float(np.diff(m.breaks(d)).min()) for d in range(3))
    bound_per_time = mixed_traj_bound(O, 4, h_min, U, PHYS["alpha"], 1.0)
    del U
    finals, drift = [], []
    for prec in (0, 1):
        s = _solver(gpu, m, precision=prec, **PHYS)
        s.set_state(U0)
        m0 = s.diagnostics()["mass"][0]
        dt = s.dt_estimate(0.5)
        s.rk_step(dt, 200)
        d = s.diagnostics()
        assert d["status"] == 0
        drift.append(abs(d["mass"][0] - m0) / m0)
        finals.append(s.get_state()[0].reshape(-1).clone())
        s.close()
    err = float(torch.linalg.vector_norm(finals[1] - finals[0]) / torch.linalg.vector_norm(finals[0]))
    bound = bound_per_time * 200 * dt
    record("mass drift, FP64", drift[0], 1e-13)
    record("mass drift, mixed", drift[1], 1e-10)
    record("mixed vs FP64, rel L2(rho)", err, bound)
    assert drift[0] <= 1e-13 and drift[1] <= 1e-10
    assert err <= bound
