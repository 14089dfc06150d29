"""Pins of the oracle's DGSEM operator for relaxation model II (Sec. 2.3 and
3.1): free-stream preservation, weak = strong form (summation by parts), exact
BR1 lifting of polynomials, symmetry under axis permutation and reflection,
mass conservation, design-order convergence on a manufactured solution, and
relaxation of a planar interface to the Maxwell densities with non-increasing
energy (Sec. 2.3 energy functional; Sec. 4.1.1 observations)."""
import numpy as np
import pytest
import sympy as sp

from paper_1912_12059_amd import inputs as I

T = 0.85


def _prob(O, m, **kw):
    nel = tuple(m.nel) + (1,) * (3 - len(m.nel))
    lo = tuple(m.lo) + (0.0,) * (3 - len(m.lo))
    hi = tuple(m.hi) + (1.0,) * (3 - len(m.hi))
    return O.Problem(dim=m.dim, N=m.N, nel=nel, lo=lo, hi=hi, xbreaks=m.xbreaks, **kw)


def _term_scale(O, P, U):
    """Size of the largest single term summed into R (operator bound times
    flux size): (2/h_min) (max row sum |Dhat| + max |L|/w) (|F| + lambda |U|)."""
    b = O.basis(P.N)
    cD = max(np.abs(b.Dhat).sum(axis=1).max(), (np.abs(b.Lp) + np.abs(b.Lm)).max() / b.w.min())
    hmin = min(np.diff(P.breaks(d)).min() for d in range(P.dim))
    rho = U[0]
    pa = np.array([O.pressure(T, r) for r in rho.ravel()[:: max(1, rho.size // 2000)]]) + 0.5 * P.alpha * rho.max() ** 2
    lam = np.sqrt(P.alpha * rho.max() + 10.0) + 1.0
    F = np.abs(U).max() * lam + np.abs(pa).max()
    return 2.0 / hmin * cD * F


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("N", [1, 3, 5])
@pytest.mark.parametrize("uniform", [True, False])
@pytest.mark.parametrize("flux", [0, 1])
def test_free_stream(O, dim, N, uniform, flux):
    g = np.random.Generator(np.random.PCG64(dim * 10 + N))
    nel = (4, 3, 3)[:dim]
    xb = None if uniform else [np.sort(np.concatenate([[0.0, 1.0], g.uniform(0.05, 0.95, nel[d] - 1)]))
                               for d in range(dim)]
    m = I.Mesh(dim, N, nel, xbreaks=xb)
    P = _prob(O, m, alpha=500.0, beta=1e-3, eps=1e-3, kappa=1e-5, flux=flux)
    U = np.zeros(P.shape())
    U[0] = 1.3
    for d in range(dim):
        U[1 + d] = 1.3 * (0.2 - 0.1 * d)
    U[-1] = 1.3
    R = O.rhs(P, U)
    assert np.abs(R).max() <= 1e-13 * _term_scale(O, P, U)


@pytest.mark.parametrize("dim,N,nel", [(1, 3, (9,)), (2, 4, (5, 4)), (3, 2, (3, 4, 3)), (3, 4, (3, 3, 2))])
@pytest.mark.parametrize("diss_c", [0, 1])
@pytest.mark.parametrize("flux", [0, 1])
def test_weak_equals_strong(O, dim, N, nel, diss_c, flux):
    """The weak form writes HLLC as HLL mass/normal-momentum fluxes plus the
    upwinded tangential momentum; the strong form writes it with star
    states.  The two are the same flux algebraically."""
    m, U = I.smooth_random(dim, N, nel, seed=dim + N)
    P = _prob(O, m, alpha=500.0, beta=1e-3, eps=1e-3, kappa=1e-5, diss_c=diss_c, flux=flux)
    R = O.rhs(P, U)
    Rs = O.rhs_strong(P, U)
    assert np.abs(R - Rs).max() <= 1e-13 * _term_scale(O, P, U)
    assert np.abs(R).max() > 1.0  # non-trivial


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_br1_lifting_exact_for_continuous_polynomials(O, dim):
    """With the central flux, the lifted gradient of a globally continuous
    periodic polynomial of degree <= N is its exact derivative."""
    N = 4
    nel = (5, 4, 3)[:dim]
    m = I.Mesh(dim, N, nel)
    P = _prob(O, m, alpha=10.0, beta=0.1, eps=0.01, kappa=1e-3)
    X = I.node_coords(m)
    f = lambda x: x ** 2 * (1 - x) ** 2          # degree 4, f(0) = f(1) = 0
    df = lambda x: 2 * x * (1 - x) ** 2 - 2 * x ** 2 * (1 - x)
    U = np.zeros(P.shape())
    U[0] = 1.5  # constant density: v = m / rho is the same polynomial / 1.5
    c = np.ones(X.shape[1:])
    for d in range(dim):
        c = c * (1.0 + f(X[d]))
    U[-1] = c
    for d in range(dim):
        U[1 + d] = 1.5 * (0.3 * f(X[(d + 1) % dim]) + 0.1 * f(X[d]))
    _, Q = O.rhs(P, U, return_Q=True)
    for d in range(dim):
        # gradient of c
        dc = df(X[d]) * np.prod([1.0 + f(X[k]) for k in range(dim) if k != d], axis=0) if dim > 1 else df(X[0])
        np.testing.assert_allclose(Q[d, dim], dc, atol=1e-12)
        for j in range(dim):
            want = 0.1 * df(X[j]) if d == j else 0.0
            if (j + 1) % dim == d and dim > 1:
                want = want + 0.3 * df(X[d])
            if dim == 1:
                want = 0.4 * df(X[0])
            np.testing.assert_allclose(Q[d, j], want, atol=1e-12)


def test_axis_permutation_and_reflection(O):
    """R commutes with swapping the x and y axes (fields and momentum
    components swapped) and with reflecting x (x-momentum negated)."""
    N, E = 3, 5
    m, U = I.smooth_random(2, N, (E, E), seed=4)
    P = _prob(O, m, alpha=300.0, beta=2e-3, eps=2e-3, kappa=1e-5)
    R = O.rhs(P, U)
    np1 = N + 1

    def swap(A):
        # element (ex, ey) node (i, j) -> element (ey, ex) node (j, i)
        B = A.reshape(A.shape[0], E, E, np1, np1)  # [var][ey][ex][j][i]
        B = B.transpose(0, 2, 1, 4, 3).reshape(A.shape)
        return B[[0, 2, 1, 3]]

    def reflect(A):
        B = A.reshape(A.shape[0], E, E, np1, np1)[:, :, ::-1, :, ::-1].reshape(A.shape).copy()
        B[1] *= -1
        return B

    np.testing.assert_allclose(O.rhs(P, swap(U)), swap(R), atol=1e-12 * np.abs(R).max())
    np.testing.assert_allclose(O.rhs(P, reflect(U)), reflect(R), atol=1e-12 * np.abs(R).max())


def test_2d_state_constant_in_y_matches_1d(O):
    N, E = 3, 8
    m1, U1 = I.smooth_random(1, N, (E,), seed=12)
    P1 = _prob(O, m1, alpha=400.0, beta=1e-3, eps=1e-3, kappa=1e-5)
    R1 = O.rhs(P1, U1)
    P2 = O.Problem(dim=2, N=N, nel=(E, 3, 1), alpha=400.0, beta=1e-3, eps=1e-3, kappa=1e-5)
    U2 = np.zeros(P2.shape())
    for ey in range(3):
        for j in range(N + 1):
            for v2, v1 in ((0, 0), (1, 1), (3, 2)):
                U2[v2].reshape(3, E, N + 1, N + 1)[ey, :, j, :] = U1[v1]
    R2 = O.rhs(P2, U2)
    for ey in range(3):
        for j in range(N + 1):
            for v2, v1 in ((0, 0), (1, 1), (3, 2)):
                np.testing.assert_allclose(R2[v2].reshape(3, E, N + 1, N + 1)[ey, :, j, :], R1[v1],
                                           atol=1e-12 * np.abs(R1).max())
            assert np.abs(R2[2]).max() <= 1e-12 * np.abs(R1).max()


def test_mass_conservation_1d_config(O):
    m, U = I.slab_1d()
    P = _prob(O, m, alpha=500.0, beta=1e-3, eps=1e-3, kappa=1e-5)
    dt = O.dt(P, U, 0.5)
    m0 = O.diagnostics(P, U)["mass"][0]
    U2 = O.run(P, U, dt, 2000)
    m1 = O.diagnostics(P, U2)["mass"][0]
    assert abs(m1 - m0) <= 1e-13 * abs(m0)


def test_dt_rule_components(O):
    """The time step is CFL times the smallest of the convective bound, the
    viscous momentum bound and the bound of the equation for c, in which the
    diffusion rate (2N+1)^2 sum_d (kappa/beta)/h_d^2 and the source rate
    alpha/(beta |z_R|) add.  At the 1D workload the c bound is the active one."""
    m, U = I.slab_1d()
    P = _prob(O, m, alpha=500.0, beta=1e-3, eps=1e-3, kappa=1e-5)
    zr = O.lsrk_real_limit()
    rate_c = 7 ** 2 * (1e-5 / 1e-3) * 64 ** 2 + 500.0 / (1e-3 * zr)
    assert O.dt(P, U, 0.5) == pytest.approx(0.5 / rate_c, rel=1e-14)
    # a convective limit: a large beta removes the stiffness of the c equation
    P2 = _prob(O, m, alpha=500.0, beta=10.0, eps=1e-3, kappa=1e-5)
    rho = U[0]
    a = np.sqrt(np.array([O.dpressure(T, r) for r in rho.ravel()]) + 500.0 * rho.ravel())
    lam = (np.abs(U[1] / U[0]).ravel() + a).max() * 64
    assert O.dt(P2, U, 0.5) == pytest.approx(0.5 / (7 * lam), rel=1e-12)
    # a viscous momentum limit: large eps, weak c stiffness; the rate is that
    # of the longitudinal mode of v = m / rho at the smallest density
    P3 = _prob(O, m, alpha=500.0, beta=10.0, eps=5.0, kappa=1e-5)
    nu = (4.0 / 3.0) * 5.0 / U[0].min()
    assert O.dt(P3, U, 0.5) == pytest.approx(0.5 / (49 * nu * 64 ** 2), rel=1e-12)
    # no step for a state without positive density
    Ubad = U.copy()
    Ubad[0].flat[7] = -0.1
    assert np.isnan(O.dt(P, Ubad, 0.5))


def _jacobian(O, P, U0, h=1e-7):
    u = U0.ravel().copy()
    J = np.zeros((u.size, u.size))
    for k in range(u.size):
        up, um = u.copy(), u.copy()
        up[k] += h
        um[k] -= h
        J[:, k] = (O.rhs(P, up.reshape(U0.shape)).ravel() - O.rhs(P, um.reshape(U0.shape)).ravel()) / (2 * h)
    return J


def _max_amplification(O, z):
    """Largest |R(z)| / max(1, exp(Re z)) over the eigenvalues: above 1, a
    numerical mode grows (or a physically growing mode grows too fast)."""
    g = O.lsrk_stability_poly()
    return (np.abs(np.polyval(g[::-1], z)) / np.maximum(1.0, np.exp(z.real))).max()


# (dim, elements per direction, N, alpha, kappa, state[, eps, beta]);
# beta = eps = 1e-3 unless given
DT_CASES = {
    # source and c-diffusion bounds equal to 0.5% (h = 1/73, N = 4, alpha = 200)
    "coinciding_liquid": (1, 73, 4, 200.0, 1e-4, "liquid"),
    "coinciding_vapour": (1, 73, 4, 200.0, 1e-4, "vapour"),
    "diffusion_limited": (1, 120, 4, 200.0, 1e-4, "liquid"),
    "source_limited_1d_workload": (1, 64, 3, 500.0, 1e-5, "liquid"),
    "source_limited_2d": (2, 6, 3, 200.0, 1e-4, "liquid"),
    "interface_moving": (1, 40, 4, 200.0, 1e-4, "interface"),
    # the planar-interface parameters of Sec. 4.1.1 (eps = beta = 0.01,
    # alpha = 100) in the vapour: the viscous momentum bound is the active one
    "viscous_limited_vapour": (1, 128, 3, 100.0, 1e-4, "vapour", 0.01, 0.01),
    # viscous momentum and c rates within 10% of each other: they act on
    # different variables, so the smallest of the two bounds suffices
    "viscous_and_c_coinciding": (1, 64, 3, 10.0, 1e-4, "vapour", 0.0024, 0.01),
    # 2D: the viscous rate (4/3)(eps/rho) sum_d 1/h_d^2 is the active one
    "viscous_limited_2d": (2, 6, 3, 100.0, 1e-4, "vapour", 0.2, 0.01),
}


def _dt_case(O, name):
    dim, E, N, alpha, kappa, state = DT_CASES[name][:6]
    eps, beta = DT_CASES[name][6:] if len(DT_CASES[name]) > 6 else (1e-3, 1e-3)
    P = O.Problem(dim=dim, N=N, nel=(E, E if dim > 1 else 1, 1), alpha=alpha, beta=beta, eps=eps, kappa=kappa)
    U = np.zeros(P.shape())
    if state == "interface":
        X = O.node_coords(P)[0]
        w = 2 * np.sqrt(kappa)
        rho = 0.32 + 0.5 * (1.81 - 0.32) * (np.tanh((X - 0.3) / w) - np.tanh((X - 0.7) / w))
        U[0] = rho
        U[1] = rho * 0.3 * np.sin(2 * np.pi * X)
        U[-1] = rho
    else:
        U[0] = 1.8 if state == "liquid" else 0.32
        U[-1] = U[0]
    return P, U


@pytest.mark.parametrize("case", sorted(DT_CASES))
def test_dt_rule_inside_stability_region(O, case):
    """Every eigenvalue z = dt lambda of the linearised model II operator
    satisfies |R(z)| <= max(1, exp(Re z)) for the LSRK4(5) polynomial R at CFL
    0.85 of the rule (the interface state has a physically growing mode); the
    workloads run at CFL 0.5."""
    P, U = _dt_case(O, case)
    lam = np.linalg.eigvals(_jacobian(O, P, U))
    assert _max_amplification(O, O.dt(P, U, 0.85) * lam) <= 1 + 1e-9


def test_dt_separate_bounds_leave_stability_region(O):
    """Where the c-diffusion and source bounds coincide, the smallest of the
    separate bounds at CFL 0.5 gives a step outside the stability region, so
    the rule must add the two rates (a mistake the test above would not see
    at the source-limited workloads)."""
    P, U = _dt_case(O, "coinciding_liquid")
    lam = np.linalg.eigvals(_jacobian(O, P, U))
    h, N2, zr = 1.0 / 73, 9.0, O.lsrk_real_limit()
    dt_sep = min(1.0 / (N2 ** 2 * max(P.eps, P.kappa / P.beta) / h ** 2), zr * P.beta / P.alpha)
    assert _max_amplification(O, 0.5 * dt_sep * lam) > 1.5
    assert _max_amplification(O, O.dt(P, U, 0.5) * lam) <= 1 + 1e-9


def test_dt_rule_convective_and_diffusive_together(O):
    """Where the convective bound (imaginary-axis eigenvalues) and the
    diffusion bounds (real ones) are about equal, eigenvalues with both parts
    near their separate limits leave the region at CFL 0.85 (2.8x
    amplification here), but at the workloads' CFL 0.5 each part is at half
    its limit and they stay inside."""
    P = O.Problem(dim=1, N=3, nel=(32, 1, 1), alpha=100.0, beta=0.01, eps=0.01, kappa=1e-4)
    U = np.zeros(P.shape())
    U[0] = 1.8
    U[-1] = 1.8
    lam = np.linalg.eigvals(_jacobian(O, P, U))
    assert _max_amplification(O, O.dt(P, U, 0.85) * lam) > 2.0
    assert _max_amplification(O, O.dt(P, U, 0.5) * lam) <= 1 + 1e-9


def test_dt_viscous_bound_takes_density_and_longitudinal_mode(O):
    """The viscous stress eps (grad v + grad v^T - (2/3) div v I) diffuses
    v = m / rho, so the momentum's largest viscous rate is (4/3) eps / rho,
    not eps: in the vapour (rho = 0.32) 4.2 times more.  With eps alone the
    bound leaves the stability region even at the workloads' CFL 0.5 on the
    planar-interface parameters (the 200-element planar interface went
    non-finite within 200 steps that way); with (4/3) eps / rho_min the rule
    holds."""
    P, U = _dt_case(O, "viscous_limited_vapour")
    lam = np.linalg.eigvals(_jacobian(O, P, U))
    h, N2, rho0 = 1.0 / 128, 7.0, 0.32
    a = np.sqrt(O.dpressure(T, rho0) + P.alpha * rho0)
    dtc = 1.0 / (N2 * a / h)
    dtk = 1.0 / (N2 ** 2 * (P.kappa / P.beta) / h ** 2 + P.alpha / (P.beta * O.lsrk_real_limit()))
    dtm = 1.0 / (N2 ** 2 * (4.0 / 3.0) * P.eps / rho0 / h ** 2)
    assert O.dt(P, U, 0.5) == pytest.approx(0.5 * min(dtc, dtm, dtk), rel=1e-12)
    assert dtm < min(dtc, dtk)  # the viscous bound is the active one
    dt_eps_only = min(dtc, 1.0 / (N2 ** 2 * P.eps / h ** 2), dtk)
    assert _max_amplification(O, 0.5 * dt_eps_only * lam) > 2.0
    assert _max_amplification(O, O.dt(P, U, 0.85) * lam) <= 1 + 1e-9


# --------------------------------------------------------------------------
# manufactured solution
# --------------------------------------------------------------------------
MMS = dict(eps=0.01, kappa=1e-3, alpha=10.0, beta=0.1)


def _mms(dim):
    X = sp.symbols(f"x0:{dim}")
    t = sp.Symbol("t")
    eps, kap, al, be = (sp.Float(MMS[k]) for k in ("eps", "kappa", "alpha", "beta"))
    ph = 2 * sp.pi * (sum(X) - t)
    rho = sp.Rational(9, 5) + sp.Rational(1, 20) * sp.sin(ph)
    v = [sp.Rational(1, 10) * sp.cos(ph + d) for d in range(dim)]
    c = rho + sp.Rational(1, 100) * sp.sin(ph)
    m = [rho * vi for vi in v]
    # the model II balance law written out from the paper: convective flux with
    # p_alpha = p + alpha rho^2/2, viscous flux (tau, (eps^2 gamma/beta) grad c),
    # source (0, alpha rho grad c, (alpha/beta)(rho - c))
    p = 8 * sp.Float(T) * rho / (3 - rho) - 3 * rho ** 2
    pa = p + al * rho ** 2 / 2
    div = sum(sp.diff(v[d], X[d]) for d in range(dim))
    tau = [[eps * (sp.diff(v[i], X[j]) + sp.diff(v[j], X[i])) - (sp.Rational(2, 3) * eps * div if i == j else 0)
            for j in range(dim)] for i in range(dim)]
    f = [sp.diff(rho, t) + sum(sp.diff(m[d], X[d]) for d in range(dim))]
    for i in range(dim):
        f.append(sp.diff(m[i], t) + sum(sp.diff(m[i] * v[d] + (pa if i == d else 0) - tau[i][d], X[d])
                                         for d in range(dim)) - al * rho * sp.diff(c, X[i]))
    f.append(sp.diff(c, t) - sum(sp.diff(kap / be * sp.diff(c, X[d]), X[d]) for d in range(dim))
             - al / be * (rho - c))
    return sp.lambdify((t,) + X, f, "numpy"), sp.lambdify((t,) + X, [rho] + m + [c], "numpy")


def _mms_error(O, dim, N, E, tend, flux=0):
    ff, uu = _mms(dim)
    m = I.Mesh(dim, N, (E,) * dim)
    P = _prob(O, m, flux=flux, **MMS)
    X = I.node_coords(m)

    def ev(fn, t):
        return np.array([np.broadcast_to(a, X.shape[1:]) for a in fn(t, *X)], dtype=float)

    U0 = ev(uu, 0.0)
    dt = O.dt(P, U0, 0.5)
    n = int(np.ceil(tend / dt))
    U = O.run(P, U0, tend / n, n, forcing=lambda t: ev(ff, t))
    b = O.basis(N)
    wq = np.ones(m.nnode)
    idx = np.arange(m.nnode)
    for d in range(dim):
        wq = wq * b.w[(idx // (N + 1) ** d) % (N + 1)] / (2 * E)
    return np.sqrt(np.sum(wq[None, :] * (U[0] - ev(uu, tend)[0]) ** 2))


@pytest.mark.parametrize("dim,N,Es", [
    (1, 1, (8, 16, 32)), (1, 2, (8, 16, 32)), (1, 3, (4, 8, 16)), (1, 4, (4, 8, 16)), (1, 5, (4, 8, 16)),
    (2, 2, (4, 8, 16)), (2, 3, (4, 8)), (3, 2, (4, 8)),
])
def test_mms_design_order(O, dim, N, Es):
    errs = [_mms_error(O, dim, N, E, 0.05) for E in Es]
    eoc = [np.log(errs[i] / errs[i + 1]) / np.log(Es[i + 1] / Es[i]) for i in range(len(errs) - 1)]
    assert eoc[-1] >= N + 0.5, (errs, eoc)


@pytest.mark.parametrize("dim,N,Es", [(1, 3, (4, 8, 16)), (2, 2, (4, 8, 16))])
def test_mms_design_order_hllc(O, dim, N, Es):
    errs = [_mms_error(O, dim, N, E, 0.05, flux=1) for E in Es]
    eoc = [np.log(errs[i] / errs[i + 1]) / np.log(Es[i + 1] / Es[i]) for i in range(len(errs) - 1)]
    assert eoc[-1] >= N + 0.5, (errs, eoc)


# --------------------------------------------------------------------------
# interface resolution: the limit behind the workloads' finite run lengths
# --------------------------------------------------------------------------
def _nonphysical_time(O, nel, kappa, tend):
    """The 1D slab (N = 3, alpha = 500, eps = beta = 1e-3) started from the
    equilibrium interface width 2 sqrt(kappa): the time at which a state
    leaves (0, 3) or turns non-finite, or None if it stays physical to tend."""
    m, U = I.slab_1d(nel=nel, N=3, width=2 * np.sqrt(kappa))
    P = _prob(O, m, alpha=500.0, beta=1e-3, eps=1e-3, kappa=kappa)
    dt = O.dt(P, U, 0.5)
    t, chunk = 0.0, 200
    while t < tend:
        U = O.run(P, U, dt, chunk)
        t += chunk * dt
        if not np.all(np.isfinite(U)) or U[0].min() <= 0.0 or U[0].max() >= 3.0:
            return t
    return None


def test_under_resolved_interface_goes_nonphysical(O):
    """Without shock capturing the DG scheme keeps an interface only if its
    width 2 sqrt(kappa) spans enough nodes (Sec. 3.2 motivates the FV
    sub-cells by this).  With N = 3 on [0, 1], kappa = 1e-5: 64 elements put
    1.6 mean node spacings across 2 sqrt(kappa) and the slab turns
    non-physical before t = 0.01; 128 elements (3.2 spacings) keep it
    physical, and so does kappa = 1e-4 on 64 elements (5.1 spacings)."""
    assert _nonphysical_time(O, 64, 1e-5, 0.01) is not None
    assert _nonphysical_time(O, 128, 1e-5, 0.01) is None
    assert _nonphysical_time(O, 64, 1e-4, 0.01) is None


# --------------------------------------------------------------------------
# planar interface: Maxwell densities, energy decay, surface tension
# --------------------------------------------------------------------------
def test_planar_interface_relaxes_to_maxwell(O):
    """Sec. 4.1.1 set-up (eps = 0.01, gamma = 1 so kappa = 1e-4, alpha = 100,
    beta = 0.01, N = 3, periodic (0, 1)) started from off-equilibrium phase
    densities 0.40 / 1.70.  At rest the model II equilibrium has equal
    chemical potential and equal pressure in the bulk phases for every alpha,
    so the bulk densities approach the Maxwell densities; the relaxation
    energy is non-increasing; the kinetic energy decays to O(1e-7) (the paper
    reports that order at t = 2); and kappa int c_x^2 over one interface tends
    to the gradient-theory surface tension sqrt(kappa) I(T)."""
    rv, rl, _, _ = O.maxwell(T)
    E, kap = 100, 1e-4
    P = O.Problem(dim=1, N=3, nel=(E, 1, 1), eps=0.01, kappa=kap, alpha=100.0, beta=0.01)
    X = O.node_coords(P)[0]
    w = 2 * np.sqrt(kap)
    rho = 0.40 + 0.5 * (1.70 - 0.40) * (np.tanh((X - 0.3) / w) - np.tanh((X - 0.7) / w))
    U = np.stack([rho, 0 * rho, rho.copy()])
    dt = O.dt(P, U, 0.5)
    chunk = 100
    nchunks = int(np.ceil(2.0 / (chunk * dt)))
    e_prev = O.diagnostics(P, U)["e_total"]
    for _ in range(nchunks):
        U = O.run(P, U, dt, chunk)
        e = O.diagnostics(P, U)["e_total"]
        assert e <= e_prev + 1e-12 * abs(e_prev)
        e_prev = e
    d = O.diagnostics(P, U)
    assert d["e_kin"] < 1e-6
    vap = U[0][np.abs(X - 0.0) < 0.06].mean()
    liq = U[0][np.abs(X - 0.5) < 0.06].mean()
    # 100 elements: 1.7e-4 and 4.1e-4 from Maxwell at t = 2, the same to two
    # digits as at 200 elements (measured), so resolution no longer limits it
    assert abs(vap - rv) < 1e-3 and abs(liq - rl) < 1e-3
    _, Q = O.rhs(P, U, return_Q=True)
    b = O.basis(3)
    wq = np.tile(b.w, E) / (2 * E)
    sigma_num = kap * np.sum(wq * Q[0, 1].ravel() ** 2) / 2
    assert sigma_num == pytest.approx(np.sqrt(kap) * O.surface_integral(T), rel=5e-3)


def test_energy_non_increasing_1d_config(O):
    m, U = I.slab_1d()
    P = _prob(O, m, alpha=500.0, beta=1e-3, eps=1e-3, kappa=1e-5)
    dt = O.dt(P, U, 0.5)
    e_prev = O.diagnostics(P, U)["e_total"]
    for _ in range(20):
        U = O.run(P, U, dt, 100)
        e = O.diagnostics(P, U)["e_total"]
        assert e <= e_prev + 1e-12 * abs(e_prev)
        e_prev = e


def test_diagnostics_closed_forms(O):
    """Quadrature diagnostics of states whose integrals are known exactly:
    a uniform state on the box [0,2]x[0,1]x[0,1] (volume 2) and a density
    polynomial of degree <= 2N+1 per direction (Gauss quadrature is exact)."""
    m = I.Mesh(3, 3, (4, 3, 2), lo=(0, 0, 0), hi=(2, 1, 1))
    P = _prob(O, m, alpha=200.0, beta=1e-3, eps=1e-3, kappa=1e-5)
    U = np.zeros(P.shape())
    rho, v, c = 1.4, (0.3, -0.2, 0.1), 1.35
    U[0] = rho
    for d in range(3):
        U[1 + d] = rho * v[d]
    U[4] = c
    dg = O.diagnostics(P, U)
    vol = 2.0
    np.testing.assert_allclose(dg["mass"], [rho * vol] + [rho * vd * vol for vd in v] + [c * vol], rtol=1e-12)
    ek = 0.5 * rho * sum(vd * vd for vd in v) * vol
    assert dg["e_kin"] == pytest.approx(ek, rel=1e-12)
    assert dg["e_total"] == pytest.approx(ek + vol * (O.W(T, rho) + 0.5 * 200.0 * (rho - c) ** 2), rel=1e-12)
    assert dg["l2_rho_minus_c"] == pytest.approx(abs(rho - c) * np.sqrt(vol), rel=1e-12)
    # polynomial density: int_0^2 x^3 dx * int_0^1 y^2 dy * int_0^1 (1+z) dz = 4 * 1/3 * 3/2
    X = I.node_coords(m)
    U[0] = 1.0 + X[0] ** 3 * X[1] ** 2 * (1 + X[2])
    assert O.diagnostics(P, U)["mass"][0] == pytest.approx(vol + 4.0 / 3.0 * 1.5, rel=1e-12)
    U[0, 5, 7] = np.nan
    assert O.diagnostics(P, U)["nonfinite"] == 1
