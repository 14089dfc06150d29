"""Pins of the oracle's FV sub-cell shock capturing (Sec. 3.2) for
relaxation model II: the sub-cell averaging matrix against exact integrals,
the Persson-Peraire indicator on polynomials and steps, the DG operator
recovered when no element is troubled, exact mass conservation across mixed
DG/FV grids, no new extrema in a shock tube where DG alone overshoots, a
two-phase Riemann problem that breaks DG alone but not with sub-cells,
second-order convergence with every element on sub-cells, and troubled
elements only where the profile is steep."""
import numpy as np
import pytest

T = 0.85


def _lsrk(O, P, U, dt, n, rhs):
    """n LSRK4(5) steps with the right-hand side rhs; stops once non-finite."""
    A, B, _ = O.lsrk45()
    U = U.copy()
    dU = np.zeros_like(U)
    with np.errstate(all="ignore"):
        for _ in range(n):
            for s in range(5):
                dU = A[s] * dU + dt * rhs(U)
                U = U + B[s] * dU
            if not np.all(np.isfinite(U)):
                break
    return U


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_subcell_matrix_exact_means(O, N):
    M, Mi = O.subcell_matrices(N)
    b = O.basis(N)
    edges = np.linspace(-1.0, 1.0, N + 2)
    for p in range(N + 1):
        u = b.xi ** p
        exact = (edges[1:] ** (p + 1) - edges[:-1] ** (p + 1)) / ((p + 1) * np.diff(edges))
        np.testing.assert_allclose(M @ u, exact, atol=1e-14)
    np.testing.assert_allclose(M @ Mi, np.eye(N + 1), atol=1e-12)


def test_persson_indicator(O):
    N = 4
    P = O.Problem(dim=2, N=N, nel=(3, 2, 1))
    X = O.node_coords(P)
    U = np.zeros(P.shape())
    # degree N-1 in each direction: no energy in the highest modes
    U[0] = 1.2 + 0.1 * X[0] ** 3 - 0.05 * X[1] ** 2 * X[0]
    assert np.all(O.persson(P, U) < -25)
    # a state made of the highest mode only: indicator 0
    b = O.basis(N)
    idx = np.arange(P.nnode)
    i, j = idx % (N + 1), idx // (N + 1)
    from numpy.polynomial import legendre
    top = legendre.legval(b.xi[i], [0] * N + [1]) * legendre.legval(b.xi[j], [1])
    U[0] = np.broadcast_to(top, U[0].shape)
    assert np.all(np.abs(O.persson(P, U)) < 1e-12)
    # a step inside an element: large indicator there
    U[0] = np.where(X[0] < 0.5, 1.8, 0.4)
    ind = O.persson(P, U)
    ex = np.arange(P.nelem) % 3
    assert np.all(ind[ex == 1] > -2.0) and np.all(ind[ex != 1] < -25)


def _shock_state(O, P, left=1.8, right=1.7):
    """A density step at rest with a constant c (no relaxation source)."""
    X = O.node_coords(P)[0]
    rho = np.where(X < 0.5, left, right) + 0.0 * X
    return np.stack([rho, 0 * rho, 0 * rho + 0.5 * (left + right)])


def test_no_troubled_elements_recovers_dg(O):
    P = O.Problem(dim=2, N=3, nel=(5, 4, 1), eps=1e-2, kappa=1e-4, alpha=500.0, beta=1e-2)
    from paper_1912_12059_amd import inputs as I
    m, U = I.smooth_random(2, 3, (5, 4), seed=3)
    R, flags = O.rhs_subcell(P, U, 1e9)
    assert not flags.any()
    assert np.array_equal(R, O.rhs(P, U))


@pytest.mark.parametrize("dim,N,nel", [(1, 3, (12,)), (2, 2, (6, 5)), (3, 2, (4, 3, 3))])
def test_mass_conserved_across_mixed_grids(O, dim, N, nel):
    """With some elements on sub-cells and the rest DG, the quadrature
    integral of the density rate vanishes (the DG/FV face flux is the same on
    both sides)."""
    from paper_1912_12059_amd import inputs as I
    m, U = I.smooth_random(dim, N, nel, seed=7 + dim, rho_range=(0.4, 1.8))
    P = O.Problem(dim=dim, N=N, nel=tuple(nel) + (1,) * (3 - dim), eps=1e-2, kappa=1e-4, alpha=500.0, beta=1e-2)
    ind = O.persson(P, U)
    thr = float(np.median(ind))
    R, flags = O.rhs_subcell(P, U, thr)
    assert 0 < flags.sum() < P.nelem
    b = O.basis(N)
    idx = np.arange(P.nnode)
    wq = np.ones(P.nnode)
    for d in range(dim):
        wq = wq * b.w[(idx // (N + 1) ** d) % (N + 1)] * 0.5 / nel[d]
    scale = np.abs(R[0] * wq).sum()
    assert abs((R[0] * wq).sum()) <= 1e-13 * scale


def test_shock_tube_no_new_extrema(O):
    """A density step in the liquid phase, at rest, inviscid (eps = 0,
    kappa = 0), with c constant and beta so large that it stays so: the
    source alpha rho grad c vanishes and the system is the isothermal
    p-system with p_alpha, whose Riemann solutions stay between the two
    initial densities.  With every element on sub-cells the sub-cell means
    stay within those bounds (to 4e-16); DG alone overshoots (by 7e-3)."""
    P = O.Problem(dim=1, N=3, nel=(40, 1, 1), eps=0.0, kappa=0.0, alpha=50.0, beta=1e6)
    U = _shock_state(O, P)
    dt = O.dt(P, U, 0.3)
    n = 60
    Uf = _lsrk(O, P, U, dt, n, lambda x: O.rhs_subcell(P, x, -1e9)[0])
    M, _ = O.subcell_matrices(3)
    means = Uf[0] @ M.T
    assert means.min() >= 1.7 - 1e-9 and means.max() <= 1.8 + 1e-9
    Ud = O.run(P, U, dt, n)
    assert Ud[0].max() > 1.8 + 1e-4 or Ud[0].min() < 1.7 - 1e-4


def test_all_subcell_second_order(O):
    """Every element on sub-cells: a smooth density wave in the liquid phase
    converges with order about 2 (second-order MUSCL on the (N+1)E cells;
    measured 1.79 between successive refinements)."""
    errs = []
    for E in (8, 16, 32):
        P = O.Problem(dim=1, N=2, nel=(E, 1, 1), eps=1e-2, kappa=1e-4, alpha=100.0, beta=1e-1)
        X = O.node_coords(P)[0]
        M, _ = O.subcell_matrices(2)
        rho = 1.8 + 0.02 * np.sin(2 * np.pi * X)
        U = np.stack([rho, 0 * rho, rho.copy()])
        tend = 0.05
        dt = O.dt(P, U, 0.3)
        n = int(np.ceil(tend / dt))
        Uf = _lsrk(O, P, U, tend / n, n, lambda x: O.rhs_subcell(P, x, -1e9)[0])
        errs.append(Uf)
    # compare successive refinements through their element means (Cauchy sequence)
    def emean(U, E):
        b = O.basis(2)
        return (U[0] * b.w).sum(axis=1) / 2.0
    e1 = np.abs(emean(errs[0], 8) - emean(errs[1], 16).reshape(8, 2).mean(axis=1)).max()
    e2 = np.abs(emean(errs[1], 16) - emean(errs[2], 32).reshape(16, 2).mean(axis=1)).max()
    assert np.log2(e1 / e2) > 1.5, (e1, e2)


def test_indicator_flags_only_the_steep_part(O):
    """A 1D profile with one sharp interface and smooth elsewhere: only the
    elements at the interface are troubled."""
    P = O.Problem(dim=1, N=4, nel=(30, 1, 1), eps=1e-2, kappa=1e-4, alpha=500.0, beta=1e-2)
    X = O.node_coords(P)[0]
    rho = 1.0 + 0.5 * np.tanh((X - 0.5) / 0.003) + 0.05 * np.sin(2 * np.pi * X)
    U = np.stack([rho, 0 * rho, rho.copy()])
    _, flags = O.rhs_subcell(P, U, -3.0)
    xc = X.mean(axis=1)
    assert flags.any()
    assert np.all(np.abs(xc[flags] - 0.5) < 0.1)


def _riemann(O):
    """A liquid slab (rho 1.8) on (0.25, 0.75) in vapour (rho 0.3), its two
    halves moving inwards at 0.5: two-phase interfaces far thinner than an
    element (2 sqrt(kappa) = 6e-4, h = 0.01)."""
    P = O.Problem(dim=1, N=3, nel=(100, 1, 1), eps=1e-4, kappa=1e-7, alpha=100.0, beta=1e-2)
    X = O.node_coords(P)[0]
    inside = (X > 0.25) & (X < 0.75)
    rho = np.where(inside, 1.8, 0.3) + 0 * X
    v = np.where(X < 0.5, 0.5, -0.5) * inside
    return P, np.stack([rho, rho * v, rho.copy()])


def test_two_phase_riemann_problem_needs_subcells(O):
    """Sec. 3.2: DG alone oscillates at the sharp phase boundaries until the
    run breaks off (non-finite within 400 steps); with sub-cells in the
    troubled elements (threshold -4) the run stays finite, the density stays
    in (0.2, 2.2) and mass is conserved."""
    P, U = _riemann(O)
    dt = O.dt(P, U, 0.4)
    Ud = _lsrk(O, P, U, dt, 400, lambda x: O.rhs(P, x))
    assert not np.all(np.isfinite(Ud))
    Us = _lsrk(O, P, U, dt, 400, lambda x: O.rhs_subcell(P, x, -4.0)[0])
    assert np.all(np.isfinite(Us))
    assert 0.2 < Us[0].min() and Us[0].max() < 2.2
    b = O.basis(3)
    mass = lambda W: (W[0] * b.w).sum() / 200.0
    assert abs(mass(Us) - mass(U)) <= 1e-13 * mass(U)
