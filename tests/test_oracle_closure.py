"""Pins of the closure oracle (network, training step, features, source,
nudging step) against closed forms, identities and finite differences."""
import numpy as np
import pytest

H = 64
OFF = {}
_o = 0
for _name, _size in (("W1", H * 4), ("b1", H), ("W2", H * H), ("b2", H), ("W3", H * H), ("b3", H),
                     ("W4", 2 * H), ("b4", 2)):
    OFF[_name] = (_o, _size)
    _o += _size
NPARAM = _o


def _block(w, name, shape):
    o, n = OFF[name]
    return w[o:o + n].reshape(shape)


def test_parameter_count(O):
    assert NPARAM == O.MLP_NPARAM == O.lib().or_mlp_nparam() == 8770


def test_relu_values_and_identity(O):
    assert O.relu(1.0) == 1.0 and O.relu(-1.0) == 0.0 and O.relu(0.0) == 0.0
    # the derivative at the kink is taken as 0, on both sides of the boundary
    assert O.relu_d(0.0) == 0.0 and O.relu_d(0.3) == 1.0 and O.relu_d(-0.3) == 0.0
    for z in (-3.2, -0.7, 0.1, 0.9, 2.5, 6.0):
        # g(z) - g(-z) = z, the identity the routing network below relies on
        assert O.relu(z) - O.relu(-z) == z
        h = 1e-5
        fd = (O.relu(z + h) - O.relu(z - h)) / (2 * h)
        assert O.relu_d(z) == pytest.approx(fd, rel=1e-8, abs=1e-10)


def routing_network():
    """Weights that pass inputs through all four layers using
    g(z) - g(-z) = z, so that y = (x0 + 1/4, x1 - x3 - 1/2) exactly.
    The units used are placed off the diagonal, so a transposed weight
    layout or a wrong block offset changes the result."""
    w = np.zeros(NPARAM)
    W1 = _block(w, "W1", (H, 4))
    W2 = _block(w, "W2", (H, H))
    W3 = _block(w, "W3", (H, H))
    W4 = _block(w, "W4", (2, H))
    b4 = _block(w, "b4", (2,))
    W1[3, 0], W1[7, 0] = 1.0, -1.0      # g(x0), g(-x0)
    W1[10, 1], W1[20, 1] = 1.0, -1.0    # g(x1), g(-x1)
    W1[30, 3], W1[40, 3] = 1.0, -1.0    # g(x3), g(-x3)
    W2[5, 3], W2[5, 7] = 1.0, -1.0      # z = x0
    W2[6, 3], W2[6, 7] = -1.0, 1.0      # z = -x0
    for u, s in ((50, 1.0), (51, -1.0)):  # z = +-(x1 - x3)
        W2[u, 10], W2[u, 20], W2[u, 30], W2[u, 40] = s, -s, -s, s
    W3[0, 5], W3[0, 6] = 1.0, -1.0
    W3[1, 5], W3[1, 6] = -1.0, 1.0
    W3[62, 50], W3[62, 51] = 1.0, -1.0
    W3[63, 50], W3[63, 51] = -1.0, 1.0
    W4[0, 0], W4[0, 1] = 1.0, -1.0
    W4[1, 62], W4[1, 63] = 1.0, -1.0
    b4[:] = (0.25, -0.5)
    return w


def test_forward_routing_network(O):
    w = routing_network()
    X = np.random.default_rng(0).uniform(-2, 2, (50, 4))
    Y = O.mlp_forward(w, X)
    np.testing.assert_allclose(Y[:, 0], X[:, 0] + 0.25, atol=1e-13)
    np.testing.assert_allclose(Y[:, 1], X[:, 1] - X[:, 3] - 0.5, atol=1e-13)


def test_loss_of_constant_network(O):
    w = np.random.default_rng(1).normal(0, 0.3, NPARAM)
    _block(w, "W4", (2, H))[:] = 0.0
    _block(w, "b4", (2,))[:] = (0.3, -1.1)
    rng = np.random.default_rng(2)
    X, T = rng.normal(size=(9, 4)), rng.normal(size=(9, 2))
    loss, g = O.mlp_loss_grad(w, X, T)
    assert loss == pytest.approx(0.5 / 9 * (((0.3 - T[:, 0]) ** 2).sum() + ((-1.1 - T[:, 1]) ** 2).sum()), rel=1e-14)
    # with W4 = 0 nothing below the output layer receives gradient
    assert np.all(g[: OFF["W4"][0]] == 0.0)
    np.testing.assert_allclose(_block(g, "b4", (2,)), [(0.3 - T[:, 0]).mean(), (-1.1 - T[:, 1]).mean()], rtol=1e-13)


def test_gradient_matches_central_differences(O):
    rng = np.random.default_rng(3)
    w = rng.normal(0, 0.25, NPARAM)
    X, T = rng.normal(size=(7, 4)), rng.normal(size=(7, 2))
    _, g = O.mlp_loss_grad(w, X, T)
    picks = []
    for name in OFF:
        o, n = OFF[name]
        picks += list(o + rng.choice(n, size=min(n, 12), replace=False))
    h = 1e-6
    for k in picks:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (O.mlp_loss_grad(wp, X, T)[0] - O.mlp_loss_grad(wm, X, T)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-10), k


def test_adam_first_two_steps_closed_form(O):
    rng = np.random.default_rng(4)
    w0 = rng.normal(size=100)
    g = rng.normal(size=100)
    w, m, v = w0.copy(), np.zeros(100), np.zeros(100)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    # bias-corrected moments of a constant gradient are g and g^2 at every step
    O.adam_step(w, m, v, g, lr, b1, b2, eps, 1)
    np.testing.assert_allclose(w, w0 - lr * g / (np.abs(g) + eps), rtol=1e-14)
    O.adam_step(w, m, v, g, lr, b1, b2, eps, 2)
    np.testing.assert_allclose(w, w0 - 2 * lr * g / (np.abs(g) + eps), rtol=1e-12)


NORM = dict(s0=1.06, k0=1.3, s1=0.9, k1=0.7, k2=0.02, k3=-0.003, g0=0.5, out_m=2.0, out_c=-3.0)


def _poly_problem(O, dim):
    # non-uniform breakpoints: the features must use each element's own width
    xb = [np.array([0.0, 0.3, 0.45, 0.8, 1.0]), np.array([0.0, 0.5, 0.6, 1.0]), np.array([0.0, 0.4, 1.0])]
    nel = tuple(len(b) - 1 for b in xb[:dim])
    return O.Problem(dim=dim, N=3, nel=nel, xbreaks=xb[:dim], alpha=300.0)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_features_exact_for_quadratics(O, dim):
    P = _poly_problem(O, dim)
    Xn = O.node_coords(P)
    x = Xn[0]
    y = Xn[1] if dim > 1 else 0 * x
    z = Xn[2] if dim > 2 else 0 * x
    rho = 1.1 + 0.3 * x - 0.2 * y ** 2 + 0.4 * x * z
    grad = [0.3 + 0.4 * z, -0.4 * y, 0.4 * x][:dim]
    lap = -0.4 if dim > 1 else 0.0
    c = rho + 0.01 * np.sin(3 * x)
    U = np.zeros(P.shape())
    U[0], U[-1] = rho, c
    U[1] = 0.1
    X, nv = O.closure_features(P, U, NORM)
    gn = np.sqrt(sum(gd ** 2 for gd in grad))
    np.testing.assert_allclose(X[:, 0], ((rho - NORM["s0"]) * NORM["k0"]).ravel(), atol=1e-14)
    np.testing.assert_allclose(X[:, 1], ((c - NORM["s1"]) * NORM["k1"]).ravel(), atol=1e-14)
    np.testing.assert_allclose(X[:, 2], (gn * NORM["k2"]).ravel(), atol=1e-13)
    np.testing.assert_allclose(X[:, 3], np.full(X.shape[0], lap * NORM["k3"]), atol=1e-12)
    den = np.sqrt(gn ** 2 + NORM["g0"] ** 2)
    for d in range(dim):
        np.testing.assert_allclose(nv[d], (grad[d] / den).ravel(), atol=1e-12)


def test_closure_source_constant_network(O):
    P = O.Problem(dim=2, N=3, nel=(3, 4), alpha=300.0)
    from paper_1912_12059_amd import inputs as I
    _, U = I.smooth_random(2, 3, (3, 4), seed=5)
    w = np.random.default_rng(6).normal(0, 0.2, NPARAM)
    _block(w, "W4", (2, H))[:] = 0.0
    _block(w, "b4", (2,))[:] = (0.7, -0.2)
    Sc = O.closure_source(P, U, w, NORM)
    _, nv = O.closure_features(P, U, NORM)
    S = P.nelem * P.nnode
    assert np.all(Sc[0] == 0.0)
    for d in range(2):
        np.testing.assert_allclose(Sc[1 + d].ravel(), NORM["out_m"] * 0.7 * nv[d], rtol=1e-15, atol=0)
    np.testing.assert_allclose(Sc[3].ravel(), np.full(S, NORM["out_c"] * -0.2), rtol=1e-15)


def test_nudge_step_closed_form(O):
    from paper_1912_12059_amd import inputs as I
    P = O.Problem(dim=2, N=3, nel=(4, 3), alpha=200.0)
    _, U = I.smooth_random(2, 3, (4, 3), seed=7)
    _, Ur = I.smooth_random(2, 3, (4, 3), seed=8)
    dt, tau, cmap = 1e-5, 4e-4, 10.0
    Un, X, Y = O.closure_nudge(P, U, Ur, dt, tau, cmap, NORM)
    Xf, nv = O.closure_features(P, U, NORM)
    np.testing.assert_array_equal(X, Xf)
    cstar = Ur[0] + cmap * (Ur[3] - Ur[0])
    np.testing.assert_array_equal(Un[0], U[0])
    for v in (1, 2):
        np.testing.assert_allclose(Un[v], U[v] + dt / tau * (Ur[v] - U[v]), rtol=1e-15, atol=1e-17)
    np.testing.assert_allclose(Un[3], U[3] + dt / tau * (cstar - U[3]), rtol=1e-15, atol=1e-17)
    dm = sum((Ur[1 + d] - U[1 + d]).ravel() * nv[d] for d in range(2))
    np.testing.assert_allclose(Y[:, 0], dm / tau, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(Y[:, 1], (cstar - U[3]).ravel() / tau, rtol=1e-13, atol=1e-12)
    # the reference itself (with c already in the model's frame) is a fixed point
    Ur2 = Ur.copy()
    Ur2[3] = Ur[0] + (Ur[3] - Ur[0]) / cmap
    Un2, _, Y2 = O.closure_nudge(P, Ur, Ur2, dt, tau, cmap, NORM)
    np.testing.assert_allclose(Un2, Ur, atol=1e-15)
    assert np.abs(Y2).max() < 1e-9
