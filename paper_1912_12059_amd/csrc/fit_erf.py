"""Coefficients of the standard normal CDF used by the closure kernels'
GELU, g(z) = z Phi(z) (closure.hpp).

Phi(z) - 1/2 = erf(z / sqrt 2) / 2 is approximated on |z| <= Z by z Q(z^2),
Q of degree DEG, fitted by least squares at Chebyshev nodes of [0, Z]
(z is clamped to [-Z, Z] before the evaluation, where Phi is within 1.2e-4
of 0 or 1).  Run this file to print the coefficients (lowest degree first)
and the maximum error of Phi in FP64 and with FP32 Horner evaluation; both
are far below the 2^-9 relative rounding of the BF16 activations the GELU
feeds."""
import numpy as np
from scipy.special import erf

Z, DEG, NODES = 3.7, 6, 4000


def phi(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0)))


def coefficients() -> np.ndarray:
    k = np.arange(NODES)
    z = Z * 0.5 * (1.0 - np.cos(np.pi * (k + 0.5) / NODES))
    V = np.vander(z * z, DEG + 1, increasing=True) * z[:, None]
    c, *_ = np.linalg.lstsq(V, phi(z) - 0.5, rcond=None)
    return c


def max_error(c, dtype):
    zt = np.linspace(-8.0, 8.0, 400001)
    zc = np.clip(zt, -Z, Z).astype(dtype)
    u = (zc * zc).astype(dtype)
    q = dtype(c[-1])
    for j in range(DEG - 1, -1, -1):
        q = (q * u + dtype(c[j])).astype(dtype)
    approx = (dtype(0.5) + zc * q).astype(dtype)
    return float(np.abs(approx.astype(np.float64) - phi(zt)).max())


if __name__ == "__main__":
    c = coefficients()
    print(", ".join(f"{v:.9e}f" for v in c))
    print(f"max |Phi error|: fp64 {max_error(c, np.float64):.2e}, fp32 {max_error(c, np.float32):.2e}")
