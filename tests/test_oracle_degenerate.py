"""Degenerate periodic grids: with one element in a direction the element is
its own neighbour on both sides.  A state on such a grid is the same
periodic function as that state repeated three times on a grid three times
longer with the same element size, so the right-hand side of every copy
must equal the original's (both models, all three numerical fluxes)."""
import numpy as np
import pytest

from paper_1912_12059_amd import inputs as I


def _tile(U, nel, reps):
    """Repeat the element layout U[var][elem][node] reps[d] times along each
    direction (elements x-fastest)."""
    nv, E, nn = U.shape
    dim = len(nel)
    A = U.reshape((nv,) + tuple(reversed(nel)) + (nn,))  # [v][ez][ey][ex][n]
    for d in range(dim):
        A = np.concatenate([A] * reps[d], axis=1 + (dim - 1 - d))
    return np.ascontiguousarray(A.reshape(nv, -1, nn))


@pytest.mark.parametrize("model,flux", [(0, 0), (0, 1), (1, 0)])
@pytest.mark.parametrize("dim,N,nel,reps", [
    (1, 3, (1,), (3,)), (2, 2, (1, 1), (3, 2)), (2, 3, (1, 3), (3, 1)), (3, 2, (1, 1, 1), (2, 3, 2)),
    (3, 2, (2, 1, 2), (1, 3, 1)),
])
def test_one_element_directions_match_tiled_grid(O, model, flux, dim, N, nel, reps):
    m, U = I.smooth_random(dim, N, nel, seed=dim * 5 + N, rho_range=(1.5, 1.9))
    if model == 1:
        U = np.ascontiguousarray(U[:-1])
    kw = dict(eps=1e-2, kappa=1e-4, model=model, flux=flux)
    if model == 0:
        kw.update(alpha=500.0, beta=1e-2)
    pad = (1,) * (3 - dim)
    P1 = O.Problem(dim=dim, N=N, nel=tuple(nel) + pad, hi=(1.0,) * 3, **kw)
    big = tuple(n * r for n, r in zip(nel, reps))
    P3 = O.Problem(dim=dim, N=N, nel=big + pad, hi=tuple(float(r) for r in reps) + (1.0,) * (3 - dim), **kw)
    R1 = O.rhs(P1, U)
    R3 = O.rhs(P3, _tile(U, nel, reps))
    np.testing.assert_allclose(R3, _tile(R1, nel, reps), rtol=0, atol=1e-10 * np.abs(R1).max())
