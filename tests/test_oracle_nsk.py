"""Pins of the oracle's DGSEM operator for the original NSK equations
(Sec. 2.2; discretisation of Sec. 3.1 with a second BR1 lifting for the
Laplacian of rho and the global Lax-Friedrichs flux):

- free-stream preservation;
- exact conservation of mass and momentum on the periodic grid (the Korteweg
  term enters as the divergence of its stress tensor);
- exactness of both liftings for C^1 piecewise cubic densities;
- design-order convergence on a manufactured solution whose forcing is
  written with the non-conservative Korteweg term kappa rho grad lap rho
  (an independent form of the same operator);
- the linear dispersion relation w^2 = p' k^2 + kappa rho k^4 with viscous
  damping, in a stable phase and in the spinodal interval (growth of long
  waves, capillary oscillation of short ones);
- stability of the time-step rule against the spectrum of the discrete
  operator;
- relaxation of a planar interface at rest to the Maxwell densities with
  non-increasing energy and the gradient-theory surface tension;
- closed-form diagnostics of a uniform state."""
import numpy as np
import pytest
import sympy as sp

from paper_1912_12059_amd import inputs as I

T = 0.85


def _prob(O, m, **kw):
    nel = tuple(m.nel) + (1,) * (3 - len(m.nel))
    lo = tuple(m.lo) + (0.0,) * (3 - len(m.lo))
    hi = tuple(m.hi) + (1.0,) * (3 - len(m.hi))
    return O.Problem(dim=m.dim, N=m.N, nel=nel, lo=lo, hi=hi, xbreaks=m.xbreaks, model=1, **kw)


def _quad_weights(O, P):
    """J_e omega_n per node, shape (nelem, nnode)."""
    b = O.basis(P.N)
    idx = np.arange(P.nnode)
    w = np.ones((P.nelem, P.nnode))
    e = np.arange(P.nelem)
    stride = 1
    for d in range(P.dim):
        h = np.diff(P.breaks(d))
        ed = (e // stride) % P.nel[d]
        stride *= P.nel[d]
        w = w * (0.5 * h[ed])[:, None] * b.w[(idx // (P.N + 1) ** d) % (P.N + 1)][None, :]
    return w


def _jittered(g, n):
    """Breakpoints of n elements on [0, 1], each within h/4 of uniform."""
    x = np.linspace(0.0, 1.0, n + 1)
    x[1:-1] += g.uniform(-0.25, 0.25, n - 1) / n
    return x


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("N", [1, 3, 4])
@pytest.mark.parametrize("uniform", [True, False])
def test_nsk_free_stream(O, dim, N, uniform):
    g = np.random.Generator(np.random.PCG64(100 + dim * 10 + N))
    nel = (4, 3, 3)[:dim]
    xb = None if uniform else [_jittered(g, nel[d]) for d in range(dim)]
    kap = 1e-4
    P = _prob(O, I.Mesh(dim, N, nel, xbreaks=xb), eps=1e-3, kappa=kap)
    U = np.zeros(P.shape())
    U[0] = 1.7
    for d in range(dim):
        U[1 + d] = 1.7 * (0.3 - 0.2 * d)
    R = O.rhs(P, U)
    # size of the largest terms summed into R: the convective one,
    # (2/h)(N+1)^2 (p + rho v^2), and the third-order Korteweg one, whose
    # round-off grows like kappa rho^2 ((2/h)(N+1)^2)^3
    k = 2.0 / min(np.diff(P.breaks(d)).min() for d in range(dim)) * (N + 1) ** 2
    scale = k * 10.0 + kap * 1.7 ** 2 * k ** 3
    assert np.abs(R).max() <= 1e-13 * scale


@pytest.mark.parametrize("dim,N", [(1, 3), (2, 2), (2, 4), (3, 2)])
def test_nsk_conserves_mass_and_momentum(O, dim, N):
    """The quadrature integral of every component of R vanishes on the
    periodic grid, for an arbitrary (here random, discontinuous) state: the
    convective, viscous and Korteweg terms are all in divergence form and the
    face fluxes are single-valued."""
    g = np.random.Generator(np.random.PCG64(7 + dim))
    nel = (5, 4, 3)[:dim]
    xb = [_jittered(g, nel[d]) for d in range(dim)]
    P = _prob(O, I.Mesh(dim, N, nel, xbreaks=xb), eps=1e-2, kappa=1e-3)
    U = np.zeros(P.shape())
    U[0] = g.uniform(0.3, 1.9, U[0].shape)
    for d in range(dim):
        U[1 + d] = U[0] * g.uniform(-0.5, 0.5, U[0].shape)
    R = O.rhs(P, U)
    w = _quad_weights(O, P)
    scale = (np.abs(R) * w[None]).sum(axis=(1, 2))
    integ = (R * w[None]).sum(axis=(1, 2))
    assert np.all(np.abs(integ) <= 1e-12 * scale.max()), (integ, scale)


def _hermite_periodic(xb, f, df, x):
    """C^1 periodic piecewise cubic through the values and slopes of f at the
    breakpoints; returns (value, first, second derivative) at x."""
    k = np.clip(np.searchsorted(xb, x, side="right") - 1, 0, len(xb) - 2)
    a, b = xb[k], xb[k + 1]
    h = b - a
    s = (x - a) / h
    y0, y1, m0, m1 = f(a), f(b), df(a) * h, df(b) * h
    h00, h10, h01, h11 = 2 * s**3 - 3 * s**2 + 1, s**3 - 2 * s**2 + s, -2 * s**3 + 3 * s**2, s**3 - s**2
    d00, d10, d01, d11 = 6 * s**2 - 6 * s, 3 * s**2 - 4 * s + 1, -6 * s**2 + 6 * s, 3 * s**2 - 2 * s
    e00, e10, e01, e11 = 12 * s - 6, 6 * s - 4, -12 * s + 6, 6 * s - 2
    val = h00 * y0 + h10 * m0 + h01 * y1 + h11 * m1
    d1 = (d00 * y0 + d10 * m0 + d01 * y1 + d11 * m1) / h
    d2 = (e00 * y0 + e10 * m0 + e01 * y1 + e11 * m1) / h**2
    return val, d1, d2


@pytest.mark.parametrize("dim,N", [(1, 3), (1, 5), (2, 3), (2, 4)])
def test_nsk_liftings_exact_for_c1_piecewise_cubics(O, dim, N):
    """For a density that is a C^1 piecewise cubic (separable products in 2D)
    the central traces of rho and of the lifted gradient are the true face
    values, so both BR1 liftings return the exact gradient and Laplacian at
    the nodes when N >= 3."""
    g = np.random.Generator(np.random.PCG64(31 + dim * 7 + N))
    nel = (6, 5)[:dim]
    xb = [_jittered(g, nel[d]) for d in range(dim)]
    P = _prob(O, I.Mesh(dim, N, nel, xbreaks=xb), eps=1e-2, kappa=1e-3)
    X = O.node_coords(P)
    parts = []
    for d in range(dim):
        k = 2 * np.pi * (d + 1)
        parts.append(_hermite_periodic(xb[d], lambda x, k=k: np.sin(k * x), lambda x, k=k: k * np.cos(k * x), X[d]))
    prod = np.ones_like(X[0])
    for p in parts:
        prod = prod * p[0]
    rho = 1.2 + 0.2 * prod
    grad, lap = [], np.zeros_like(rho)
    for d in range(dim):
        other = np.ones_like(rho)
        for dd in range(dim):
            if dd != d:
                other = other * parts[dd][0]
        grad.append(0.2 * parts[d][1] * other)
        lap += 0.2 * parts[d][2] * other
    U = np.stack([rho] + [0.1 * rho] * dim)
    _, Q, L = O.rhs(P, U, return_Q=True)
    for d in range(dim):
        np.testing.assert_allclose(Q[d, dim], grad[d], atol=1e-11 * np.abs(grad[d]).max())
    np.testing.assert_allclose(L, lap, atol=1e-10 * np.abs(lap).max())


@pytest.mark.parametrize("N", [1, 2, 4])
def test_nsk_piecewise_constant_reduces_to_lf_finite_volume(O, N):
    """With eps = kappa = 0 and a state constant in each element, the element
    mean of the DG right-hand side is the first-order finite-volume update
    (F*_- - F*_+)/h with the global Lax-Friedrichs flux
    F* = (F(uL) + F(uR))/2 - lam (uR - uL)/2, lam = max |v| + sqrt(max(p', 0))."""
    g = np.random.Generator(np.random.PCG64(55 + N))
    E = 8
    xb = _jittered(g, E)
    P = O.Problem(dim=1, N=N, nel=(E, 1, 1), xbreaks=[xb], model=1, eps=0.0, kappa=0.0)
    rho = g.uniform(0.3, 1.9, E)
    v = g.uniform(-0.5, 0.5, E)
    U = np.stack([np.repeat(rho[:, None], N + 1, 1), np.repeat((rho * v)[:, None], N + 1, 1)])
    R = O.rhs(P, U)
    b = O.basis(N)
    mean = (R * b.w[None, None, :]).sum(axis=2) / 2.0
    lam = max(abs(v[e]) + np.sqrt(max(O.dpressure(T, rho[e]), 0.0)) for e in range(E))

    def flux(e):
        return np.array([rho[e] * v[e], rho[e] * v[e] ** 2 + O.pressure(T, rho[e])])

    def u(e):
        return np.array([rho[e], rho[e] * v[e]])

    def lf(eL, eR):
        return 0.5 * (flux(eL) + flux(eR)) - 0.5 * lam * (u(eR) - u(eL))

    h = np.diff(xb)
    for e in range(E):
        fv = (lf((e - 1) % E, e) - lf(e, (e + 1) % E)) / h[e]
        np.testing.assert_allclose(mean[:, e], fv, rtol=1e-12, atol=1e-12 * np.abs(fv).max())


# --------------------------------------------------------------------------
# manufactured solution, forcing from the non-conservative Korteweg term
# --------------------------------------------------------------------------
MMS = dict(eps=0.01, kappa=1e-3)


def _mms(dim):
    X = sp.symbols(f"x0:{dim}")
    t = sp.Symbol("t")
    eps, kap = sp.Float(MMS["eps"]), sp.Float(MMS["kappa"])
    ph = 2 * sp.pi * (sum(X) - t)
    rho = sp.Rational(9, 5) + sp.Rational(1, 20) * sp.sin(ph)
    v = [sp.Rational(1, 10) * sp.cos(ph + d) for d in range(dim)]
    m = [rho * vi for vi in v]
    p = 8 * sp.Float(T) * rho / (3 - rho) - 3 * rho ** 2
    div = sum(sp.diff(v[d], X[d]) for d in range(dim))
    tau = [[eps * (sp.diff(v[i], X[j]) + sp.diff(v[j], X[i])) - (sp.Rational(2, 3) * eps * div if i == j else 0)
            for j in range(dim)] for i in range(dim)]
    lap = sum(sp.diff(rho, X[d], 2) for d in range(dim))
    f = [sp.diff(rho, t) + sum(sp.diff(m[d], X[d]) for d in range(dim))]
    for i in range(dim):
        f.append(sp.diff(m[i], t) + sum(sp.diff(m[i] * v[d] + (p if i == d else 0) - tau[i][d], X[d])
                                         for d in range(dim)) - kap * rho * sp.diff(lap, X[i]))
    return sp.lambdify((t,) + X, f, "numpy"), sp.lambdify((t,) + X, [rho] + m, "numpy")


def _mms_error(O, dim, N, E, tend):
    ff, uu = _mms(dim)
    m = I.Mesh(dim, N, (E,) * dim)
    P = _prob(O, m, **MMS)
    X = I.node_coords(m)

    def ev(fn, t):
        return np.array([np.broadcast_to(a, X.shape[1:]) for a in fn(t, *X)], dtype=float)

    U0 = ev(uu, 0.0)
    dt = O.dt(P, U0, 0.5)
    n = int(np.ceil(tend / dt))
    U = O.run(P, U0, tend / n, n, forcing=lambda t: ev(ff, t))
    w = _quad_weights(O, P)
    return np.sqrt(np.sum(w * (U[0] - ev(uu, tend)[0]) ** 2))


@pytest.mark.parametrize("dim,N,Es", [
    (1, 1, (8, 16, 32)), (1, 2, (8, 16, 32)), (1, 3, (4, 8, 16)), (1, 4, (4, 8, 16)), (1, 5, (4, 8, 16)),
    (2, 2, (4, 8, 16)), (2, 3, (4, 8)),
])
def test_nsk_mms_design_order(O, dim, N, Es):
    errs = [_mms_error(O, dim, N, E, 0.05) for E in Es]
    eoc = [np.log(errs[i] / errs[i + 1]) / np.log(Es[i + 1] / Es[i]) for i in range(len(errs) - 1)]
    assert eoc[-1] >= N + 0.5, (errs, eoc)


# --------------------------------------------------------------------------
# linear waves about a state at rest
# --------------------------------------------------------------------------
def _linear_amplitude(O, rho0, k, eps, kap, t):
    """rho = rho0 + delta A(t) cos(k x) with A'' + (4/3)(eps/rho0) k^2 A'
    + (p'(rho0) k^2 + kappa rho0 k^4) A = 0, A(0) = 1, A'(0) = 0."""
    b = 4.0 / 3.0 * eps / rho0 * k * k
    c = O.dpressure(T, rho0) * k * k + kap * rho0 * k ** 4
    s1, s2 = np.roots([1.0, b, c]).astype(complex)
    return ((s2 * np.exp(s1 * t) - s1 * np.exp(s2 * t)) / (s2 - s1)).real


@pytest.mark.parametrize("rho0,mode,kap,tend,E,kind", [
    (1.9, 2, 1e-2, 0.3, 16, "oscillates"),       # liquid: acoustic + capillary
    (1.0, 1, 1e-3, 0.5, 16, "grows"),            # spinodal, long wave: p' k^2 + kappa rho k^4 < 0
    (1.0, 6, 1e-3, 0.3, 32, "oscillates"),       # spinodal, short wave: stabilised by capillarity
])
def test_nsk_linear_dispersion(O, rho0, mode, kap, tend, E, kind):
    eps, delta, N = 1e-3, 1e-7, 4
    k = 2 * np.pi * mode
    P = O.Problem(dim=1, N=N, nel=(E, 1, 1), model=1, eps=eps, kappa=kap)
    X = O.node_coords(P)[0]
    U = np.stack([rho0 + delta * np.cos(k * X), 0 * X])
    dt = O.dt(P, U, 0.5)
    n = int(np.ceil(tend / dt))
    U = O.run(P, U, tend / n, n)
    A = _linear_amplitude(O, rho0, k, eps, kap, tend)
    assert (A > 2.0) == (kind == "grows")
    err = np.abs(U[0] - rho0 - delta * A * np.cos(k * X)).max() / (delta * max(1.0, abs(A)))
    assert err < 2e-5, err


# --------------------------------------------------------------------------
# time-step rule against the spectrum of the discrete operator
# --------------------------------------------------------------------------
def _jacobian(O, P, U0, h=1e-7):
    u = U0.ravel().copy()
    J = np.zeros((u.size, u.size))
    for k in range(u.size):
        up, um = u.copy(), u.copy()
        up[k] += h
        um[k] -= h
        J[:, k] = (O.rhs(P, up.reshape(U0.shape)).ravel() - O.rhs(P, um.reshape(U0.shape)).ravel()) / (2 * h)
    return J


@pytest.mark.parametrize("case", ["liquid_N2", "liquid_N5", "vapour_2d", "interface", "viscous_vapour"])
def test_nsk_dt_rule_inside_stability_region(O, case):
    """At CFL 1 every eigenvalue z = dt lambda of the linearised operator
    satisfies |R(z)| <= max(1, exp(Re z)) for the stability polynomial R of
    the Runge-Kutta scheme: numerical modes do not grow, and physically
    unstable modes (spinodal states) grow no faster than they should."""
    if case == "liquid_N2":
        P = O.Problem(dim=1, N=2, nel=(16, 1, 1), model=1, eps=1e-3, kappa=1e-3)
        U = np.zeros(P.shape())
        U[0] = 1.9
    elif case == "liquid_N5":
        P = O.Problem(dim=1, N=5, nel=(10, 1, 1), model=1, eps=1e-3, kappa=1e-5)
        U = np.zeros(P.shape())
        U[0] = 1.9
    elif case == "viscous_vapour":
        # eps = 0.02 in the vapour: the viscous bound, (4/3) eps / rho, is active
        P = O.Problem(dim=1, N=3, nel=(24, 1, 1), model=1, eps=0.02, kappa=1e-5)
        U = np.zeros(P.shape())
        U[0] = 0.32
    elif case == "vapour_2d":
        P = O.Problem(dim=2, N=3, nel=(4, 4, 1), model=1, eps=1e-3, kappa=1e-4)
        U = np.zeros(P.shape())
        U[0] = 0.3
    else:
        P = O.Problem(dim=1, N=4, nel=(20, 1, 1), model=1, eps=1e-2, kappa=1e-4)
        X = O.node_coords(P)[0]
        w = 2 * np.sqrt(1e-4)
        rho = 0.32 + 0.5 * (1.81 - 0.32) * (np.tanh((X - 0.3) / w) - np.tanh((X - 0.7) / w))
        U = np.stack([rho, rho * 0.3 * np.sin(2 * np.pi * X)])
    lam = np.linalg.eigvals(_jacobian(O, P, U))
    z = O.dt(P, U, 1.0) * lam
    g = O.lsrk_stability_poly()
    R = np.abs(np.polyval(g[::-1], z))
    assert np.all(R <= np.maximum(1.0, np.exp(z.real)) * (1 + 1e-6)), (z[np.argmax(R)], R.max())


# --------------------------------------------------------------------------
# Korteweg limit of the relaxation model
# --------------------------------------------------------------------------
def test_relaxation_model_approaches_nsk_as_alpha_grows(O):
    """Sec. 2.3 and 4.1.1: model II tends to the original NSK equations as
    alpha grows (c follows rho and alpha rho grad(rho - c) becomes the
    Korteweg force).  A slab at rest between the Maxwell densities, with the
    parameters of Sec. 4.1.1 (eps = 0.01, kappa = 1e-4, beta = 0.01, N = 3,
    50 elements), run to t = 0.5 with the two independently written right-hand
    sides: the density of model II at alpha = 100 is three times closer to
    the NSK density than at alpha = 10 (measured 1.6e-3 against 5.1e-3 in
    L2).  Larger alpha needs finer grids here: at alpha = 1000 on 100
    elements the gap is 1.7e-3, at alpha = 1e4 on 50 elements the relaxation
    is unresolved and the run blows up at t = 0.051 whatever the CFL."""
    rv, rl, _, _ = O.maxwell(0.85)
    E, kap, tend = 50, 1e-4, 0.5
    P1 = O.Problem(dim=1, N=3, nel=(E, 1, 1), model=1, eps=0.01, kappa=kap)
    X = O.node_coords(P1)[0]
    w = 2 * np.sqrt(kap)
    rho = rv + 0.5 * (rl - rv) * (np.tanh((X - 0.3) / w) - np.tanh((X - 0.7) / w))
    wq = np.tile(O.basis(3).w, E) / (2 * E)

    def run(P, U):
        n = int(np.ceil(tend / O.dt(P, U, 0.5)))
        return O.run(P, U, tend / n, n)

    r_nsk = run(P1, np.stack([rho, 0 * rho]))[0]
    gap = {}
    for alpha in (10.0, 100.0):
        P2 = O.Problem(dim=1, N=3, nel=(E, 1, 1), alpha=alpha, beta=0.01, eps=0.01, kappa=kap)
        r2 = run(P2, np.stack([rho, 0 * rho, rho.copy()]))[0]
        gap[alpha] = np.sqrt(np.sum(wq * (r2 - r_nsk).ravel() ** 2))
    assert gap[100.0] < 0.4 * gap[10.0], gap
    assert gap[100.0] < 2e-3, gap


# --------------------------------------------------------------------------
# planar interface and diagnostics
# --------------------------------------------------------------------------
def test_nsk_planar_interface_relaxes_to_maxwell(O):
    """Two planar interfaces at rest, started from off-equilibrium phase
    densities 0.40 / 1.70 (eps = 0.05, kappa = 1e-3, N = 3, periodic (0, 1)):
    the energy int (rho |v|^2/2 + W + kappa |grad rho|^2/2) does not increase,
    the bulk densities approach the Maxwell densities, and kappa int rho_x^2
    over one interface tends to the gradient-theory surface tension
    sqrt(kappa) I(T)."""
    rv, rl, _, _ = O.maxwell(T)
    E, kap = 24, 1e-3
    P = O.Problem(dim=1, N=3, nel=(E, 1, 1), model=1, eps=0.05, kappa=kap)
    X = O.node_coords(P)[0]
    w = 2 * np.sqrt(kap)
    rho = 0.40 + 0.5 * (1.70 - 0.40) * (np.tanh((X - 0.3) / w) - np.tanh((X - 0.7) / w))
    U = np.stack([rho, 0 * rho])
    dt = O.dt(P, U, 0.5)
    chunk = 100
    e_prev = O.diagnostics(P, U)["e_total"]
    for _ in range(int(np.ceil(3.0 / (chunk * dt)))):
        U = O.run(P, U, dt, chunk)
        e = O.diagnostics(P, U)["e_total"]
        assert e <= e_prev + 1e-12 * abs(e_prev)
        e_prev = e
    d = O.diagnostics(P, U)
    assert d["e_kin"] < 1e-6
    vap = U[0][np.abs(X - 0.0) < 0.06].mean()
    liq = U[0][np.abs(X - 0.5) < 0.06].mean()
    assert abs(vap - rv) < 2e-3 and abs(liq - rl) < 2e-3
    _, Q, _ = O.rhs(P, U, return_Q=True)
    b = O.basis(3)
    wq = np.tile(b.w, E) / (2 * E)
    sigma_num = kap * np.sum(wq * Q[0, 1].ravel() ** 2) / 2
    assert sigma_num == pytest.approx(np.sqrt(kap) * O.surface_integral(T), rel=5e-3)


def test_nsk_diagnostics_uniform_state(O):
    P = O.Problem(dim=3, N=2, nel=(3, 2, 2), lo=(0.0, 0.0, 0.0), hi=(2.0, 1.0, 1.0), model=1, kappa=1e-4)
    U = np.zeros(P.shape())
    rho, v = 1.8, (0.3, -0.2, 0.1)
    U[0] = rho
    for d in range(3):
        U[1 + d] = rho * v[d]
    d = O.diagnostics(P, U)
    vol = 2.0
    np.testing.assert_allclose(d["mass"], vol * np.array([rho] + [rho * x for x in v]), rtol=1e-13)
    ek = 0.5 * rho * sum(x * x for x in v)
    assert d["e_kin"] == pytest.approx(vol * ek, rel=1e-13)
    assert d["e_total"] == pytest.approx(vol * (ek + O.W(T, rho)), rel=1e-13)
    assert d["max_wavespeed"] == pytest.approx(0.3 + np.sqrt(O.dpressure(T, rho)), rel=1e-14)
    assert d["l2_rho_minus_c"] == 0.0
    # spinodal density: no real sound speed, the LF speed is the flow speed alone
    U[0] = 1.0
    for dd in range(3):
        U[1 + dd] = 1.0 * v[dd]
    assert O.lf_speed(P, U) == pytest.approx(0.3, rel=1e-14)
