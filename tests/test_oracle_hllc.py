"""Pins of the oracle's HLLC flux (barotropic form of Toro's HLLC for the
model II convective part) by properties that fix it: consistency, upwinding
of supersonic states, exact resolution of a stationary contact (where the
Rusanov flux diffuses) and mirror symmetry."""
import numpy as np
import pytest

PH = dict(T=0.85, eps=1e-3, kappa=1e-5, alpha=500.0, beta=1e-3)


def _p(O, dim, flux=1, diss_c=1):
    return O.Problem(dim=dim, N=2, nel=(2, 2, 2)[:dim] + (1,) * (3 - dim), flux=flux, diss_c=diss_c, **PH)


def _phys(O, P, d, u):
    """Model II convective flux of a point state, from the paper's definition."""
    dim = P.dim
    rho = u[0]
    pa = O.pressure(P.T, rho) + 0.5 * P.alpha * rho * rho
    F = np.zeros(dim + 2)
    F[0] = u[1 + d]
    for j in range(dim):
        F[1 + j] = u[1 + d] * u[1 + j] / rho + (pa if j == d else 0.0)
    return F


def _state(rng, dim, rho=None, vmax=0.5):
    rho = rng.uniform(0.3, 1.9) if rho is None else rho
    v = rng.uniform(-vmax, vmax, dim)
    return np.concatenate([[rho], rho * v, [rho + rng.uniform(-0.05, 0.05)]])


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_consistency(O, dim):
    rng = np.random.default_rng(dim)
    P = _p(O, dim)
    for _ in range(20):
        u = _state(rng, dim)
        for d in range(dim):
            np.testing.assert_allclose(O.numflux(P, d, u, u), _phys(O, P, d, u), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_supersonic_states_are_upwinded(O, dim):
    P = _p(O, dim)
    rng = np.random.default_rng(10 + dim)
    for sign in (1.0, -1.0):
        for _ in range(5):
            uL, uR = _state(rng, dim, rho=0.5), _state(rng, dim, rho=0.55)
            for d in range(dim):
                a = np.sqrt(O.dpressure(P.T, 0.55) + P.alpha * 0.55)
                uL[1 + d] = sign * 0.5 * (a + 5.0)
                uR[1 + d] = sign * 0.55 * (a + 5.0)
                F = O.numflux(P, d, uL, uR)
                up = uL if sign > 0 else uR
                np.testing.assert_allclose(F, _phys(O, P, d, up), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_stationary_contact_is_exact(O, dim):
    """Equal density and normal velocity zero, jump in the tangential
    velocity: no mass or tangential momentum crosses, the normal momentum
    flux is the pressure.  Rusanov diffuses the jump."""
    P = _p(O, dim)
    Pr = _p(O, dim, flux=0)
    rho = 1.4
    pa = O.pressure(P.T, rho) + 0.5 * P.alpha * rho * rho
    for d in range(dim):
        uL = np.full(dim + 2, 0.0)
        uR = np.full(dim + 2, 0.0)
        uL[0] = uR[0] = rho
        uL[-1] = uR[-1] = rho
        for j in range(dim):
            if j != d:
                uL[1 + j], uR[1 + j] = rho * 0.3, -rho * 0.2
        F = O.numflux(P, d, uL, uR)
        assert F[0] == 0.0
        assert F[1 + d] == pytest.approx(pa, rel=1e-15)
        for j in range(dim):
            if j != d:
                assert F[1 + j] == 0.0
        Fr = O.numflux(Pr, d, uL, uR)
        assert abs(Fr[1 + (d + 1) % dim]) > 1.0


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("diss_c", [0, 1])
def test_mirror_symmetry(O, dim, diss_c):
    """Reflecting x_d -> -x_d swaps the states and the sign of their normal
    velocities; the flux of mass, of the tangential momenta and of c changes
    sign, that of the normal momentum does not."""
    P = _p(O, dim, diss_c=diss_c)
    rng = np.random.default_rng(20 + dim)
    for _ in range(20):
        uL, uR = _state(rng, dim), _state(rng, dim)
        for d in range(dim):
            F = O.numflux(P, d, uL, uR)
            mL, mR = uR.copy(), uL.copy()
            mL[1 + d] *= -1
            mR[1 + d] *= -1
            G = O.numflux(P, d, mL, mR)
            for v in range(dim + 2):
                s = 1.0 if v == 1 + d else -1.0
                assert G[v] == pytest.approx(s * F[v], rel=1e-12, abs=1e-12), (d, v)


def test_c_flux(O):
    """c has no convective flux: HLLC adds only the HLL dissipation
    SL SR (cR - cL)/(SR - SL) (diss_c = 1), which has the sign of -(cR - cL)."""
    P1, P0 = _p(O, 1, diss_c=1), _p(O, 1, diss_c=0)
    uL = np.array([1.0, 0.1, 1.02])
    uR = np.array([1.1, 0.05, 1.06])
    assert O.numflux(P0, 0, uL, uR)[2] == 0.0
    assert O.numflux(P1, 0, uL, uR)[2] < 0.0
