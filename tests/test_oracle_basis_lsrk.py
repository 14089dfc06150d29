"""Pins of the oracle's 1D Gauss-Legendre basis (Sec. 3.1) and of its
low-storage Runge-Kutta scheme against library routines, closed forms and the
classical order conditions."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as P


@pytest.mark.parametrize("N", range(1, 9))
def test_nodes_weights_match_numpy(O, N):
    b = O.basis(N)
    x, w = npleg.leggauss(N + 1)
    np.testing.assert_allclose(b.xi, x, atol=1e-15)
    np.testing.assert_allclose(b.w, w, atol=1e-15)


@pytest.mark.parametrize("N", range(1, 9))
def test_quadrature_exact_to_degree_2N_plus_1(O, N):
    b = O.basis(N)
    for k in range(2 * N + 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert np.dot(b.w, b.xi ** k) == pytest.approx(exact, abs=1e-14)


@pytest.mark.parametrize("N", range(1, 9))
def test_derivative_matrix_exact_for_polynomials(O, N):
    b = O.basis(N)
    g = np.random.Generator(np.random.PCG64(N))
    for _ in range(3):
        c = g.normal(size=N + 1)
        f = P.polyval(b.xi, c)
        df = P.polyval(b.xi, P.polyder(c))
        np.testing.assert_allclose(b.D @ f, df, atol=1e-12 * (1 + np.abs(df).max()))
    assert np.abs(b.D.sum(axis=1)).max() < 1e-13


@pytest.mark.parametrize("N", range(1, 9))
def test_boundary_interpolation(O, N):
    b = O.basis(N)
    assert b.Lp.sum() == pytest.approx(1.0, abs=1e-14)
    assert b.Lm.sum() == pytest.approx(1.0, abs=1e-14)
    g = np.random.Generator(np.random.PCG64(100 + N))
    c = g.normal(size=N + 1)
    f = P.polyval(b.xi, c)
    assert b.Lp @ f == pytest.approx(P.polyval(1.0, c), abs=1e-12)
    assert b.Lm @ f == pytest.approx(P.polyval(-1.0, c), abs=1e-12)


@pytest.mark.parametrize("N", range(1, 9))
def test_summation_by_parts(O, N):
    b = O.basis(N)
    M = np.diag(b.w)
    lhs = M @ b.D + (M @ b.D).T
    rhs = np.outer(b.Lp, b.Lp) - np.outer(b.Lm, b.Lm)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("N", range(1, 8))
def test_weak_operator_is_integral_against_test_derivative(O, N):
    """Dhat f at node i equals (1/w_i) int_{-1}^{1} f l_i' dx for the
    interpolant f (evaluated with a 30-point numpy Gauss rule)."""
    b = O.basis(N)
    xq, wq = npleg.leggauss(30)
    g = np.random.Generator(np.random.PCG64(7 + N))
    f = g.normal(size=N + 1)
    # Lagrange basis on the oracle nodes via numpy polynomial fits
    n = N + 1
    V = np.vander(b.xi, n, increasing=True)
    coef = np.linalg.solve(V, np.eye(n))  # column j: coefficients of l_j
    fq = P.polyval(xq, np.linalg.solve(V, f))
    for i in range(n):
        dli = P.polyval(xq, P.polyder(coef[:, i]))
        assert b.Dhat[i] @ f == pytest.approx(np.dot(wq, fq * dli) / b.w[i], abs=1e-11)


# --------------------------------------------------------------------------
# low-storage RK4(5)
# --------------------------------------------------------------------------
def _butcher(A, B):
    """Butcher tableau of the 2N-storage scheme dU_s = A_s dU_{s-1} + k_s,
    U_s = U_{s-1} + B_s dU_s, k_s = dt R(U_{s-1})."""
    s = len(A)
    a = np.zeros((s + 1, s))
    for st in range(1, s + 1):          # row st: coefficients of U_st
        for j in range(st):              # k_{j+1}
            tot = 0.0
            for q in range(j, st):
                prod = 1.0
                for mm in range(j + 1, q + 1):
                    prod *= A[mm]
                tot += B[q] * prod
            a[st, j] = tot
    return a[:s], a[s]


def test_lsrk_order_conditions(O):
    A, B, Cc = O.lsrk45()
    a, b = _butcher(A, B)
    c = a.sum(axis=1)
    np.testing.assert_allclose(c, Cc, atol=1e-14)
    conds = [
        (b.sum(), 1.0),
        (b @ c, 1 / 2),
        (b @ c ** 2, 1 / 3),
        (b @ (a @ c), 1 / 6),
        (b @ c ** 3, 1 / 4),
        (b @ (c * (a @ c)), 1 / 8),
        (b @ (a @ c ** 2), 1 / 12),
        (b @ (a @ (a @ c)), 1 / 24),
    ]
    for got, want in conds:
        assert got == pytest.approx(want, abs=1e-14)
    # the scheme is not fifth order: at least one fifth-order condition fails
    assert abs(b @ c ** 4 - 1 / 5) > 1e-6 or abs(b @ (a @ (a @ (a @ c))) - 1 / 120) > 1e-6


def test_lsrk_stability_polynomial(O):
    A, B, _ = O.lsrk45()
    a, b = _butcher(A, B)
    g = O.lsrk_stability_poly()
    one = np.ones(5)
    want = [1.0, b @ one, b @ (a @ one), b @ (a @ (a @ one)), b @ (a @ (a @ (a @ one))),
            b @ (a @ (a @ (a @ (a @ one))))]
    np.testing.assert_allclose(g, want, atol=1e-14)
    np.testing.assert_allclose(g[:5], [1, 1, 1 / 2, 1 / 6, 1 / 24], atol=1e-14)


def test_lsrk_real_axis_limit(O):
    g = O.lsrk_stability_poly()
    # |R(-x)| = 1: roots of R(-x) - 1 and R(-x) + 1 on x > 0
    gm = g * (-1.0) ** np.arange(6)
    roots = []
    for shift in (-1.0, 1.0):
        p = gm.copy()
        p[0] += shift
        r = np.roots(p[::-1])
        roots += [z.real for z in r if abs(z.imag) < 1e-9 and z.real > 1e-9]
    xr = min(roots)
    assert O.lsrk_real_limit() == pytest.approx(xr, rel=1e-10)
    assert 4.6 < xr < 4.7
