"""Pins of the oracle's thermodynamics (Sec. 2.1) and of the droplet
initial-state construction (Sec. 4.3.1) against values the paper prints and
against identities the Van-der-Waals model must satisfy."""
import math
import os

import numpy as np
import pytest
from scipy import integrate

GOLD = os.path.join(os.path.dirname(__file__), "golden")
T = 0.85


def _golden(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_maxwell_matches_printed_values(O):
    rv, rl, _, _ = O.maxwell(T)
    g = {r[0]: float(r[1]) for r in _golden("maxwell_T085.txt")}
    assert abs(rv - g["rho_vap_sat"]) < 0.5e-4
    assert abs(rl - g["rho_liq_sat"]) < 0.5e-4
    assert abs(0.5 * (rv + rl) - g["rho_mean"]) < 0.5e-4


def test_maxwell_equal_area_in_specific_volume(O):
    """Equal-area rule: the isotherm p(1/v) between the saturated specific
    volumes has the same integral as the saturation pressure line.  The oracle
    solves the equal-chemical-potential form; this is an independent check."""
    rv, rl, ps, _ = O.maxwell(T)
    area, _ = integrate.quad(lambda v: O.pressure(T, 1.0 / v), 1.0 / rl, 1.0 / rv, epsabs=1e-13, epsrel=1e-13)
    assert area == pytest.approx(ps * (1.0 / rv - 1.0 / rl), rel=1e-10)
    assert O.pressure(T, rv) == pytest.approx(O.pressure(T, rl), rel=1e-12)


def test_pressure_is_rho_dW_minus_W(O):
    """p = rho W' - W (Sec. 2.1), checked with central differences of W."""
    for rho in (0.2, 0.5, 1.0, 1.4, 2.1, 2.7):
        h = 1e-5
        dW = (O.W(T, rho + h) - O.W(T, rho - h)) / (2 * h)
        assert O.dW(T, rho) == pytest.approx(dW, rel=1e-8, abs=1e-9)
        assert O.pressure(T, rho) == pytest.approx(rho * dW - O.W(T, rho), rel=1e-8, abs=1e-9)
        dp = (O.pressure(T, rho + h) - O.pressure(T, rho - h)) / (2 * h)
        assert O.dpressure(T, rho) == pytest.approx(dp, rel=1e-7, abs=1e-8)
        d2W = (O.dW(T, rho + h) - O.dW(T, rho - h)) / (2 * h)
        assert O.d2W(T, rho) == pytest.approx(d2W, rel=1e-7, abs=1e-8)
        assert O.dpressure(T, rho) == pytest.approx(rho * O.d2W(T, rho), rel=1e-12)


def test_reduced_vdw_critical_point(O):
    """With a = 3, b = 1/3, R = 8/3 the critical point is rho = T = p = 1:
    p'(1) = p''(1) = 0 at T = 1 and p(1) = 1."""
    assert O.pressure(1.0, 1.0) == pytest.approx(1.0, rel=1e-14)
    assert abs(O.dpressure(1.0, 1.0)) < 1e-13
    h = 1e-4
    d2p = (O.dpressure(1.0, 1.0 + h) - O.dpressure(1.0, 1.0 - h)) / (2 * h)
    assert abs(d2p) < 1e-6


def test_spinodal_and_min_W2(O):
    sv, sl = O.spinodal(T)
    assert abs(O.dpressure(T, sv)) < 1e-12 and abs(O.dpressure(T, sl)) < 1e-12
    assert 0 < sv < 1 < sl < 3
    # p' < 0 strictly inside, > 0 outside
    assert O.dpressure(T, 0.5 * (sv + sl)) < 0 and O.dpressure(T, 0.5 * sv) > 0 and O.dpressure(T, 2.0) > 0
    # closed form: W''(rho) = R T / (rho (1 - b rho)^2) - 2a has its minimum at
    # rho = 1 with value 6 T - 6 for the reduced constants
    assert O.d2W(T, 1.0) == pytest.approx(6 * T - 6, rel=1e-13)
    grid = np.linspace(sv, sl, 2001)
    vals = np.array([O.d2W(T, r) for r in grid])
    assert abs(grid[np.argmin(vals)] - 1.0) < 1e-3


@pytest.mark.parametrize("row", _golden("hoc_table.txt"), ids=lambda r: r[0])
def test_young_laplace_reproduces_hoc_table(O, row):
    """Sec. 4.3.1: sigma from the collision Weber number, Young-Laplace phase
    pressures, inversion of the isotherm.  The table is reproduced with
    sigma = 2 r rho_c v_rel^2 / We_coll (the printed formula omits the square
    of v_rel; with it, all four rows match to the printed digits)."""
    _, Re, We, eps, gamma, vrel, rl_ref, rv_ref = row
    We, vrel = float(We), float(vrel)
    sigma = 2 * 0.1 * 1.0 * vrel ** 2 / We
    rl, rv = O.young_laplace(T, sigma, 0.1)
    assert abs(rl - float(rl_ref)) < 0.5e-4
    assert abs(rv - float(rv_ref)) < 0.5e-4
    # fixed Weber number 6000 = 1/(eps^2 gamma) of the same table
    assert 1.0 / (float(eps) ** 2 * float(gamma)) == pytest.approx(6000, rel=3e-3)  # eps printed to 3 digits


def test_young_laplace_zero_tension_is_maxwell(O):
    rv, rl, _, _ = O.maxwell(T)
    l, v = O.young_laplace(T, 0.0, 0.2)
    assert l == pytest.approx(rl, abs=1e-11) and v == pytest.approx(rv, abs=1e-11)


def test_surface_integral_quadrature_converged(O):
    """The composite rule converges: the same integral by adaptive quadrature
    of the excess free energy (the integrand vanishes quadratically at both
    saturated densities)."""
    rv, rl, ps, mus = O.maxwell(T)
    f = lambda r: math.sqrt(max(0.0, 2 * (O.W(T, r) - mus * r + ps)))
    ref, _ = integrate.quad(f, rv, rl, epsabs=1e-13, epsrel=1e-12, limit=200)
    assert O.surface_integral(T) == pytest.approx(ref, rel=1e-9)
