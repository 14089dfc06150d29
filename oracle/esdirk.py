"""Oracle (test infrastructure only): implicit time stepping with the
six-stage, fourth-order explicit-first-stage singly diagonally implicit
Runge-Kutta scheme (ESDIRK4(6), Kennedy and Carpenter's ARK4(3)6L[2]SA
implicit tableau) named in Sec. 3.1 for the implicit runs of the paper.

For U' = R(U) one step from U_n:
  K_1 = R(U_n)
  stage i = 2..6: solve X - dt gamma R(X) = B_i,  B_i = U_n + dt sum_{j<i} a_ij K_j,
                  then K_i = (X - B_i) / (dt gamma)
  U_{n+1} = X_6 (the scheme is stiffly accurate: b is the last row of A).

Each stage equation is solved by Newton's method with a dense Jacobian of R
built column by column with central differences, to machine precision; this
is only for small systems, and it is the plain reference that the GPU's
matrix-free Newton-Krylov solver is compared with.  R is the oracle's
weak-form right-hand side (either model).
"""
from __future__ import annotations

from fractions import Fraction as F

import numpy as np

from . import oracle as O

GAMMA = F(1, 4)


def tableau():
    """(A, b, bhat, c) as Fractions: Kennedy and Carpenter's ESDIRK
    ARK4(3)6L[2]SA implicit part, gamma = 1/4; bhat is the embedded
    third-order solution."""
    g = GAMMA
    A = [[F(0)] * 6 for _ in range(6)]
    A[1][:2] = [F(1, 4), g]
    A[2][:3] = [F(8611, 62500), F(-1743, 31250), g]
    A[3][:4] = [F(5012029, 34652500), F(-654441, 2922500), F(174375, 388108), g]
    A[4][:5] = [F(15267082809, 155376265600), F(-71443401, 120774400), F(730878875, 902184768),
                F(2285395, 8070912), g]
    A[5] = [F(82889, 524892), F(0), F(15625, 83664), F(69875, 102672), F(-2260, 8211), g]
    b = list(A[5])
    bhat = [F(4586570599, 29645900160), F(0), F(178811875, 945068544), F(814220225, 1159782912),
            F(-3700637, 11593932), F(61727, 225920)]
    c = [sum(row) for row in A]
    return A, b, bhat, c


def _jacobian(fun, X, h_rel=1e-7):
    n = X.size
    J = np.zeros((n, n))
    x = X.ravel()
    for k in range(n):
        h = h_rel * max(1.0, abs(x[k]))
        xp, xm = x.copy(), x.copy()
        xp[k] += h
        xm[k] -= h
        J[:, k] = (fun(xp) - fun(xm)) / (2.0 * h)
    return J


def solve_stage(fun, B, dtg, X0, tol=1e-14, max_iter=30):
    """Newton for X - dtg fun(X) = B (flat arrays); returns (X, iterations).
    Converged when the Newton update is below tol relative to |X|."""
    X = X0.copy()
    J = None
    for it in range(1, max_iter + 1):
        G = X - dtg * fun(X) - B
        if J is None:
            J = np.eye(X.size) - dtg * _jacobian(fun, X)
        dX = np.linalg.solve(J, -G)
        X = X + dX
        if np.linalg.norm(dX) <= tol * max(1.0, np.linalg.norm(X)):
            return X, it
    raise RuntimeError("stage Newton iteration did not converge")


def step_fun(fun, U, dt, tol=1e-14):
    """One ESDIRK4(6) step of U' = fun(U) for a flat state U."""
    A, b, _, c = tableau()
    Af = [[float(x) for x in row] for row in A]
    dtg = dt * float(GAMMA)
    K = [fun(U)]
    X = U.copy()
    for i in range(1, 6):
        B = U + dt * sum(Af[i][j] * K[j] for j in range(i))
        X, _ = solve_stage(fun, B, dtg, X, tol)
        K.append((X - B) / dtg)
    return X


def run(P, U, dt, nsteps, tol=1e-14):
    """nsteps ESDIRK4(6) steps of the oracle's semi-discretisation for the
    problem P (oracle.Problem, either model)."""
    shape = P.shape()
    fun = lambda x: O.rhs(P, x.reshape(shape)).ravel()
    x = np.ascontiguousarray(U, dtype=np.float64).ravel().copy()
    for _ in range(nsteps):
        x = step_fun(fun, x, dt, tol)
    return x.reshape(shape)
