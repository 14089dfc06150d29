"""Round-off scale of the DGSEM right-hand side, per variable.

Each R value is a sum of O(10) terms whose size is bounded by
    (2/h_min) * C_D * (|F_v| + lambda |U_v|),
with C_D the larger of the max row sum of |Dhat| and max(|L+|+|L-|)/w_min,
F_v the physical flux of variable v (rho: m; momentum: m v + p_alpha; c: its
viscous flux, small) and lambda the largest Rusanov wave speed.  Two FP64
evaluations in different summation orders differ by a few ulps of that size;
the parity bound used by the tests is RHS_ULPS times 2^-53 times it."""
import numpy as np

RHS_ULPS = 100


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
    """max over variables of max|R_test - R_ref| / (2^-53 scale_v)."""
    R_test = np.asarray(R_test).reshape(R_ref.shape)
    d = np.abs(R_test - R_ref).reshape(R_ref.shape[0], -1).max(axis=1)
    return float(np.max(d / (2.0 ** -53 * scales)))
