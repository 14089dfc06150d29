"""Seeded synthetic inputs shared by the GPU path, the oracle tests and the
benchmark.

This module holds none of the method's arithmetic.  It places the samples of
the analytic initial conditions at the Gauss-Legendre nodes (numpy's
Gauss-Legendre rule) in the state layout U[var][elem][node], and reads the
thermodynamic constants (Maxwell and Young-Laplace densities, surface-tension
integral) from ``case_constants.json``, which a script under ``oracle/``
writes.  Random numbers come from numpy's PCG64 with fixed seeds.

Workloads (all periodic boxes, reduced Van-der-Waals fluid at T = 0.85):
- ``slab_1d``:   liquid slab on [0.3, 0.7] in vapour, tanh interfaces of width
                 0.02, seeded uniform noise 1e-3 on rho, c = rho (the 1D
                 static-interface set-up of Sec. 4.1.1 with two interfaces).
- ``droplets_2d``: two droplets in vapour (initial condition of Sec. 4.2 with
                 n = 2), radius 0.12 at (0.36, 0.5) and (0.64, 0.5).
- ``collision_3d``: two droplets of radius R moving head-on (initial condition
                 of Sec. 4.3.1), Young-Laplace densities, speed U from a
                 Weber number We = rho_l (2U)^2 (2R) / sigma.
- ``smooth_random``: smooth periodic random states for parity tests.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SEED_NOISE = 1912
SEED_SWEEP = 12059


def constants() -> dict:
    with open(os.path.join(HERE, "case_constants.json")) as f:
        return json.load(f)


@dataclass
class Mesh:
    dim: int
    N: int
    nel: tuple
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    xbreaks: list | None = None

    @property
    def nelem(self) -> int:
        return int(np.prod(self.nel[: self.dim]))

    @property
    def nnode(self) -> int:
        return (self.N + 1) ** self.dim

    @property
    def nvar(self) -> int:
        return self.dim + 2

    def breaks(self, d: int) -> np.ndarray:
        if self.xbreaks is not None and self.xbreaks[d] is not None:
            return np.asarray(self.xbreaks[d], dtype=np.float64)
        return self.lo[d] + (self.hi[d] - self.lo[d]) * np.arange(self.nel[d] + 1) / self.nel[d]


def node_coords(m: Mesh) -> np.ndarray:
    """X[d][elem][node] of the Gauss-Legendre nodes of every element."""
    xi = np.polynomial.legendre.leggauss(m.N + 1)[0]
    np1 = m.N + 1
    X = np.empty((m.dim, m.nelem, m.nnode))
    # element index per direction and node index per direction
    e = np.arange(m.nelem)
    n = np.arange(m.nnode)
    eidx = [e % m.nel[0]]
    if m.dim > 1:
        eidx.append((e // m.nel[0]) % m.nel[1])
    if m.dim > 2:
        eidx.append(e // (m.nel[0] * m.nel[1]))
    nidx = [(n // np1 ** d) % np1 for d in range(m.dim)]
    for d in range(m.dim):
        b = m.breaks(d)
        left = b[eidx[d]][:, None]
        h = (b[eidx[d] + 1] - b[eidx[d]])[:, None]
        X[d] = left + 0.5 * (xi[nidx[d]][None, :] + 1.0) * h
    return X


def _pack(rho, mom, c) -> np.ndarray:
    return np.ascontiguousarray(np.stack([rho] + list(mom) + [c]))


def slab_1d(nel: int = 64, N: int = 3, width: float = 0.02, noise: float = 1e-3, seed: int = SEED_NOISE):
    """Liquid slab in vapour on periodic [0, 1]."""
    k = constants()["maxwell"]
    rv, rl = k["rho_v"], k["rho_l"]
    m = Mesh(1, N, (nel,))
    x = node_coords(m)[0]
    rho = rv + 0.5 * (rl - rv) * (np.tanh((x - 0.3) / width) - np.tanh((x - 0.7) / width))
    if noise:
        rho = rho + np.random.Generator(np.random.PCG64(seed)).uniform(-noise, noise, rho.shape)
    return m, _pack(rho, [np.zeros_like(rho)], rho.copy())


def _min_image(dx, L):
    return dx - L * np.round(dx / L)


def droplets_2d(nel: int = 96, N: int = 4, radius: float = 0.12, centres=((0.36, 0.5), (0.64, 0.5)),
                width: float = 0.02, noise: float = 1e-3, seed: int = SEED_NOISE):
    """Droplets at rest in vapour on periodic [0, 1]^2 (n-droplet initial
    condition of Sec. 4.2)."""
    k = constants()["maxwell"]
    rv, rl = k["rho_v"], k["rho_l"]
    m = Mesh(2, N, (nel, nel))
    X = node_coords(m)
    n = len(centres)
    rho = 0.5 * (n * rl - (n - 2) * rv) * np.ones(X.shape[1:])
    for cx, cy in centres:
        dist = np.hypot(_min_image(X[0] - cx, 1.0), _min_image(X[1] - cy, 1.0))
        rho = rho + 0.5 * (rv - rl) * np.tanh((dist - radius) / width)
    if noise:
        rho = rho + np.random.Generator(np.random.PCG64(seed)).uniform(-noise, noise, rho.shape)
    z = np.zeros_like(rho)
    return m, _pack(rho, [z, z.copy()], rho.copy())


def collision_speed(We: float, radius: float, rho_l: float, sigma: float) -> float:
    """U from We = rho_l (2U)^2 (2R) / sigma."""
    return math.sqrt(We * sigma / (rho_l * 4.0 * 2.0 * radius))


def collision_3d(nel=(96, 48, 48), N: int = 4, We: float = 40.0, radius: float = 0.2,
                 lo=(0.0, 0.0, 0.0), hi=(2.0, 1.0, 1.0), centres=None, width: float = 0.02,
                 impact: float = 0.0, noise: float = 0.0, seed: int = SEED_NOISE, dtype=np.float64,
                 device=None):
    """Two droplets of radius R approaching head-on along x (initial
    condition of Sec. 4.3.1, density written as rho_v + (rho_l - rho_v)/2
    sum_i [1 - tanh((d_i - R)/w)]).  ``impact`` offsets the droplets by
    -+impact/2 in y.  With ``device`` (a torch device string) the same state
    is built there with torch and returned as a torch tensor (no noise)."""
    kc = constants()
    yl = kc["young_laplace"][f"{radius:.3f}"]
    rl, rv = yl["rho_l"], yl["rho_v"]
    U = collision_speed(We, radius, rl, kc["sigma"])
    Lx = hi[0] - lo[0]
    if centres is None:
        xm = lo[0] + 0.5 * Lx
        cy, cz = 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])
        centres = ((xm - 0.15 * Lx, cy - 0.5 * impact, cz), (xm + 0.15 * Lx, cy + 0.5 * impact, cz))
    m = Mesh(3, N, tuple(nel), tuple(lo), tuple(hi))
    X = node_coords(m)
    if device is not None:
        import torch as xp

        X = xp.from_numpy(X).to(device)
        minimg = lambda dx, L: dx - L * xp.round(dx / L)
    else:
        xp = np
        minimg = _min_image
    L = [hi[d] - lo[d] for d in range(3)]
    prof = []
    for c in centres:
        dist = xp.sqrt(sum(minimg(X[d] - c[d], L[d]) ** 2 for d in range(3)))
        prof.append(1.0 - xp.tanh((dist - radius) / width))
    rho = rv + 0.5 * (rl - rv) * (prof[0] + prof[1])
    xm = 0.5 * (centres[0][0] + centres[1][0])
    vx = xp.where(X[0] < xm, 0.5 * U * prof[0], -0.5 * U * prof[1])
    del X
    if noise and device is None:
        rho = rho + np.random.Generator(np.random.PCG64(seed)).uniform(-noise, noise, rho.shape)
    if device is not None:
        out = xp.zeros((5,) + tuple(rho.shape), dtype=xp.float64, device=device)
    else:
        out = np.zeros((5,) + rho.shape, dtype=dtype)
    out[0] = rho
    out[1] = rho * vx
    out[4] = rho
    return m, out


def smooth_random(dim: int, N: int, nel, seed: int = 7, rho_range=(0.45, 1.75), vmax: float = 0.2,
                  dc: float = 0.02, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), xbreaks=None):
    """Smooth periodic random state: a few random Fourier modes per field.
    rho spans both phases and the spinodal region."""
    g = np.random.Generator(np.random.PCG64(seed))
    m = Mesh(dim, N, tuple(nel), tuple(lo), tuple(hi), xbreaks)
    X = node_coords(m)

    def field():
        f = np.zeros(X.shape[1:])
        for _ in range(3):
            kvec = g.integers(-2, 3, size=dim)
            ph = g.uniform(0, 2 * np.pi)
            amp = g.uniform(0.5, 1.0)
            arg = sum(2 * np.pi * kvec[d] * (X[d] - lo[d]) / (hi[d] - lo[d]) for d in range(dim))
            f = f + amp * np.sin(arg + ph)
        return f / 3.0

    r0, r1 = rho_range
    rho = 0.5 * (r0 + r1) + 0.5 * (r1 - r0) * np.clip(field(), -1, 1)
    vel = [vmax * field() for _ in range(dim)]
    c = rho + dc * field()
    return m, _pack(rho, [rho * v for v in vel], c)


def batched_sweep(n: int = 24, seed: int = SEED_SWEEP):
    """Instance list of the batched collision sweep: x-length n_x/32 with
    n_x in {32, 40, 48, 56, 64}, 32 x 32 cross-section, degree N in {3,4,5},
    R = 0.1 L_x, We ~ U[5, 150], impact parameter ~ U[0, 0.5] R."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        nx = int(g.choice([32, 40, 48, 56, 64]))
        N = int(g.choice([3, 4, 5]))
        Lx = nx / 32.0
        R = round(0.1 * Lx, 3)
        We = float(g.uniform(5.0, 150.0))
        b = float(g.uniform(0.0, 0.5)) * R
        out.append({"nel": (nx, 32, 32), "N": N, "lo": (0.0, 0.0, 0.0), "hi": (Lx, 1.0, 1.0),
                    "radius": R, "We": We, "impact": b})
    return out
