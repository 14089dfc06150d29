"""Round-off scale of the DGSEM right-hand side, per variable.

Each R value is a sum of O(10) terms whose size is bounded by
    (2/h_min) * C_D * (|F_v| + lambda |U_v|),
with C_D the larger of the max row sum of |Dhat| and max(|L+|+|L-|)/w_min,
F_v the physical flux of variable v (rho: m; momentum: m v + p_alpha; c: its
viscous flux, small) and lambda the largest Rusanov wave speed.  Two FP64
evaluations in different summation orders differ by a few ulps of that size;
the parity bound used by the tests is RHS_ULPS times 2^-53 times it."""
import os

import numpy as np

RHS_ULPS = 100
MIXED_ULPS = 200  # FP32 ulps of the term scale (mixed-precision right-hand sides)

# (test, quantity) -> [largest achieved value, bound]; printed at the end of
# the run by the terminal-summary hook in conftest.py
RECORDS = {}


def record(quantity: str, achieved: float, bound: float) -> None:
    """Keep the largest achieved error of a check next to its bound."""
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").rsplit(" (", 1)[0]
    key = (test, quantity)
    prev = RECORDS.get(key)
    if prev is None or float(achieved) > prev[0]:
        RECORDS[key] = [float(achieved), float(bound)]


def term_scales(O, N, h_min, U, alpha, T=0.85):
    b = O.basis(N)
    cD = max(np.abs(b.Dhat).sum(axis=1).max(), (np.abs(b.Lp) + np.abs(b.Lm)).max() / b.w.min())
    rho = U[0]
    nv = U.shape[0]
    dim = nv - 2
    rmax = float(np.abs(rho).max())
    pa = max(abs(O.pressure(T, r)) for r in (float(rho.min()), rmax, 1.0)) + 0.5 * alpha * rmax ** 2
    vmax = max(float(np.abs(U[1 + d] / rho).max()) for d in range(dim))
    lam = vmax + np.sqrt(max(O.dpressure(T, r) + alpha * r for r in (float(rho.min()), rmax)))
    mmax = max(float(np.abs(U[1 + d]).max()) for d in range(dim))
    F = [mmax] + [mmax * vmax + pa] * dim + [0.0]
    return np.array([2.0 / h_min * cD * (F[v] + lam * float(np.abs(U[v]).max())) for v in range(nv)])


def rhs_err_ulps(R_test, R_ref, scales):
    """max over variables of max|R_test - R_ref| / (2^-53 scale_v) (recorded
    against RHS_ULPS)."""
    R_test = np.asarray(R_test).reshape(R_ref.shape)
    d = np.abs(R_test - R_ref).reshape(R_ref.shape[0], -1).max(axis=1)
    ulps = float(np.max(d / (2.0 ** -53 * scales)))
    record("rhs, ulps of term scale", ulps, RHS_ULPS)
    return ulps


def mixed_traj_bound(O, N, h_min, U, alpha, t_end, growth=2.0):
    """Bound on the relative L2 error of rho of a mixed-precision run after
    time t_end, against an FP64 run from the same state.

    Every mixed right-hand side lies within MIXED_ULPS FP32 ulps of the rho
    term scale s of the FP64 one at every node (the bound the mixed RHS
    tests check).  A Runge-Kutta step of size dt adds at most dt times that
    per node, and at a step inside the stability region of the linearised
    operator earlier differences are not amplified beyond physical growth,
    allowed for by the factor `growth` (exp(Re lambda t_end) stays near 1 for
    the growth rates of these states and t_end <= 1e-2).  Summed over the run
    and divided by the RMS of rho:
        |rho_mixed - rho_fp64|_2 / |rho_fp64|_2
            <= growth * t_end * MIXED_ULPS * 2^-24 * s / rms(rho)."""
    s = term_scales(O, N, h_min, U, alpha)[0]
    rms = float(np.sqrt(np.mean(np.asarray(U[0]) ** 2)))
    return growth * t_end * MIXED_ULPS * 2.0 ** -24 * s / rms


def term_scales_nsk(O, P, U, kappa, eps, T=0.85):
    """The same bound for the original NSK path (state rho, m; P a model-1
    oracle problem).  The momentum flux adds the second-order stress
    Sigma = eps tau + kappa ((rho lap + |g|^2/2) I - g g^T), g = grad rho,
    sized from the oracle's liftings, and the round-off of the two liftings
    grows through the third-order term: an error of one ulp in rho becomes
    K ulps in g and K (|g| + K rho) in lap rho, K = (2/h_min) C_D."""
    b = O.basis(P.N)
    cD = max(np.abs(b.Dhat).sum(axis=1).max(), (np.abs(b.Lp) + np.abs(b.Lm)).max() / b.w.min())
    h_min = min(float(np.diff(P.breaks(d)).min()) for d in range(P.dim))
    K = 2.0 / h_min * cD
    dim = P.dim
    rho = U[0]
    rmax = float(np.abs(rho).max())
    vmax = max(float(np.abs(U[1 + d] / rho).max()) for d in range(dim))
    mmax = max(float(np.abs(U[1 + d]).max()) for d in range(dim))
    pmax = max(abs(O.pressure(T, r)) for r in (float(rho.min()), rmax, 1.0))
    lam = O.lf_speed(P, U)
    _, Q, lap = O.rhs(P, U, return_Q=True)
    gmax = float(np.abs(Q[:, dim]).max())
    dvmax = float(np.abs(Q[:, :dim]).max())
    sig = 2.0 * eps * dvmax * dim + kappa * (rmax * float(np.abs(lap).max()) + 1.5 * dim * gmax ** 2)
    lift_err = kappa * rmax * K * (gmax + K * rmax) + kappa * gmax * K * rmax
    s_rho = K * (mmax + lam * rmax)
    s_m = K * (mmax * vmax + pmax + lam * mmax + sig + lift_err)
    return np.array([s_rho] + [s_m] * dim)
