"""ctypes binding of the plain FP64 CPU oracle (``oracle/liboracle.so``).

TEST INFRASTRUCTURE ONLY: the checker the GPU path is compared against.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the HIP library.

Each wrapper names the C function it calls; the C sources cite the passages of
the paper they follow.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = ["basis.c", "thermo.c", "lsrk.c", "dg_weak.c", "dg_strong.c", "nsk_orig.c", "subcell.c", "mlp.c",
           "closure.c"]


def build(force: bool = True, path: str = LIB_PATH, native: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP over elements).  The checker the
    tests load is built -O2 for any x86-64 host, since the library travels
    between machines; native=True builds an -O3 -march=native copy for the
    host it is built on (the CPU baseline's timing build, same sources)."""
    if not force and os.path.exists(path):
        return path
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    tmp = path + ".tmp"
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = ["gcc", "-std=c11"] + opt + ["-fopenmp", "-fPIC", "-shared", "-o", tmp] + srcs + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, path)
    return path


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def use(path: str) -> None:
    """Load the oracle from another build of the same sources (before any
    other call of this module)."""
    global _lib
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    _lib = C.CDLL(path)
    _declare(_lib)


class _Basis(C.Structure):
    _fields_ = [
        ("N", C.c_int),
        ("xi", C.c_double * 13),
        ("w", C.c_double * 13),
        ("D", (C.c_double * 13) * 13),
        ("Dhat", (C.c_double * 13) * 13),
        ("Lm", C.c_double * 13),
        ("Lp", C.c_double * 13),
    ]


class _Prob(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("N", C.c_int),
        ("nel", C.c_int * 3),
        ("xb", C.POINTER(C.c_double) * 3),
        ("T", C.c_double),
        ("eps", C.c_double),
        ("kappa", C.c_double),
        ("alpha", C.c_double),
        ("beta", C.c_double),
        ("diss_c", C.c_int),
        ("flux", C.c_int),
    ]


FORCING = C.CFUNCTYPE(None, C.c_double, C.POINTER(C.c_double), C.c_void_p)
_dp = C.POINTER(C.c_double)


def _declare(L):
    L.or_make_basis.argtypes = [C.c_int, C.POINTER(_Basis)]
    for name in ("or_W", "or_dW", "or_p", "or_dp", "or_d2W"):
        getattr(L, name).argtypes = [C.c_double, C.c_double]
        getattr(L, name).restype = C.c_double
    L.or_maxwell.argtypes = [C.c_double, _dp, _dp, _dp, _dp]
    L.or_spinodal.argtypes = [C.c_double, _dp, _dp]
    L.or_surface_integral.argtypes = [C.c_double]
    L.or_surface_integral.restype = C.c_double
    L.or_young_laplace.argtypes = [C.c_double, C.c_double, C.c_double, _dp, _dp]
    L.or_lsrk45.argtypes = [_dp, _dp, _dp]
    L.or_lsrk_stability_poly.argtypes = [_dp]
    L.or_lsrk_real_limit.restype = C.c_double
    L.or_rhs_weak.argtypes = [C.POINTER(_Prob), _dp, _dp, _dp]
    L.or_rhs_strong.argtypes = [C.POINTER(_Prob), _dp, _dp]
    L.or_run.argtypes = [C.POINTER(_Prob), _dp, C.c_double, C.c_int, C.c_double, FORCING, C.c_void_p]
    L.or_dt.argtypes = [C.POINTER(_Prob), _dp, C.c_double]
    L.or_dt.restype = C.c_double
    L.or_diagnostics.argtypes = [C.POINTER(_Prob), _dp, _dp]
    L.or_node_coords.argtypes = [C.POINTER(_Prob), _dp]
    L.or_numflux.argtypes = [C.POINTER(_Prob), C.c_int, _dp, _dp, _dp]
    L.or_nsk_rhs.argtypes = [C.POINTER(_Prob), _dp, _dp, _dp, _dp]
    L.or_nsk_rhs_lam.argtypes = [C.POINTER(_Prob), _dp, C.c_double, _dp, _dp, _dp]
    L.or_nsk_run.argtypes = [C.POINTER(_Prob), _dp, C.c_double, C.c_int, C.c_double, FORCING, C.c_void_p]
    L.or_nsk_lf_speed.argtypes = [C.POINTER(_Prob), _dp]
    L.or_nsk_lf_speed.restype = C.c_double
    L.or_nsk_dt.argtypes = [C.POINTER(_Prob), _dp, C.c_double]
    L.or_nsk_dt.restype = C.c_double
    L.or_nsk_diagnostics.argtypes = [C.POINTER(_Prob), _dp, _dp]
    L.or_subcell_matrices.argtypes = [C.c_int, _dp, _dp]
    L.or_persson.argtypes = [C.POINTER(_Prob), _dp, _dp]
    L.or_rhs_subcell.argtypes = [C.POINTER(_Prob), _dp, C.c_double, _dp, C.POINTER(C.c_int)]
    L.or_relu.argtypes = [C.c_double]
    L.or_relu.restype = C.c_double
    L.or_relu_d.argtypes = [C.c_double]
    L.or_relu_d.restype = C.c_double
    L.or_mlp_nparam.restype = C.c_long
    L.or_mlp_forward.argtypes = [_dp, _dp, C.c_long, _dp]
    L.or_mlp_loss_grad.argtypes = [_dp, _dp, _dp, C.c_long, _dp]
    L.or_mlp_loss_grad.restype = C.c_double
    L.or_adam_step.argtypes = [_dp, _dp, _dp, _dp, C.c_long, C.c_double, C.c_double, C.c_double, C.c_double,
                               C.c_int]
    L.or_closure_features.argtypes = [C.POINTER(_Prob), _dp, _dp, _dp, _dp]
    L.or_closure_source.argtypes = [C.POINTER(_Prob), _dp, _dp, _dp, _dp]
    L.or_closure_nudge.argtypes = [C.POINTER(_Prob), _dp, _dp, C.c_double, C.c_double, C.c_double, _dp, _dp,
                                   _dp]


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


# --------------------------------------------------------------------------
# basis, thermodynamics, time integration
# --------------------------------------------------------------------------
@dataclass
class Basis:
    N: int
    xi: np.ndarray
    w: np.ndarray
    D: np.ndarray
    Dhat: np.ndarray
    Lm: np.ndarray
    Lp: np.ndarray


def basis(N: int) -> Basis:
    b = _Basis()
    if lib().or_make_basis(N, C.byref(b)) != 0:
        raise ValueError(f"bad degree {N}")
    n = N + 1
    D = np.array([[b.D[i][j] for j in range(n)] for i in range(n)])
    Dh = np.array([[b.Dhat[i][j] for j in range(n)] for i in range(n)])
    return Basis(N, np.array(b.xi[:n]), np.array(b.w[:n]), D, Dh, np.array(b.Lm[:n]), np.array(b.Lp[:n]))


def W(T, rho):
    return lib().or_W(T, rho)


def dW(T, rho):
    return lib().or_dW(T, rho)


def d2W(T, rho):
    return lib().or_d2W(T, rho)


def pressure(T, rho):
    return lib().or_p(T, rho)


def dpressure(T, rho):
    return lib().or_dp(T, rho)


def maxwell(T: float):
    v, l, p, m = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    if lib().or_maxwell(T, C.byref(v), C.byref(l), C.byref(p), C.byref(m)):
        raise ValueError("Maxwell construction failed")
    return v.value, l.value, p.value, m.value


def spinodal(T: float):
    a, b = C.c_double(), C.c_double()
    if lib().or_spinodal(T, C.byref(a), C.byref(b)):
        raise ValueError("no spinodal")
    return a.value, b.value


def surface_integral(T: float) -> float:
    return lib().or_surface_integral(T)


def young_laplace(T: float, sigma: float, r: float):
    l, v = C.c_double(), C.c_double()
    if lib().or_young_laplace(T, sigma, r, C.byref(l), C.byref(v)):
        raise ValueError("Young-Laplace inversion failed")
    return l.value, v.value


def lsrk45():
    A, B, Cc = (np.zeros(5) for _ in range(3))
    lib().or_lsrk45(_ptr(A), _ptr(B), _ptr(Cc))
    return A, B, Cc


def lsrk_stability_poly():
    g = np.zeros(6)
    lib().or_lsrk_stability_poly(_ptr(g))
    return g


def lsrk_real_limit() -> float:
    return lib().or_lsrk_real_limit()


# --------------------------------------------------------------------------
# DG operator
# --------------------------------------------------------------------------
@dataclass
class Problem:
    dim: int
    N: int
    nel: tuple
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    T: float = 0.85
    eps: float = 1e-3
    kappa: float = 1e-5
    alpha: float = 500.0
    beta: float = 1e-3
    diss_c: int = 1
    flux: int = 0  # 0: Rusanov, 1: HLLC
    model: int = 0  # 0: relaxation model II, 1: original NSK (state rho, rho v)
    xbreaks: list | None = None  # optional per-direction breakpoints
    _keep: list = field(default_factory=list, repr=False)

    def breaks(self, d: int) -> np.ndarray:
        if self.xbreaks is not None and self.xbreaks[d] is not None:
            return np.ascontiguousarray(self.xbreaks[d], dtype=np.float64)
        return np.linspace(self.lo[d], self.hi[d], self.nel[d] + 1)

    @property
    def nelem(self) -> int:
        return int(np.prod(self.nel[: self.dim]))

    @property
    def nnode(self) -> int:
        return (self.N + 1) ** self.dim

    @property
    def nvar(self) -> int:
        return self.dim + 2 if self.model == 0 else self.dim + 1

    def shape(self):
        return (self.nvar, self.nelem, self.nnode)

    def c(self) -> _Prob:
        p = _Prob()
        p.dim, p.N = self.dim, self.N
        self._keep = []
        for d in range(3):
            p.nel[d] = int(self.nel[d]) if d < self.dim else 1
            if d < self.dim:
                xb = self.breaks(d)
                self._keep.append(xb)
                p.xb[d] = _ptr(xb)
        p.T, p.eps, p.kappa, p.alpha, p.beta = self.T, self.eps, self.kappa, self.alpha, self.beta
        p.diss_c = self.diss_c
        p.flux = self.flux
        return p


def _state(P: Problem, U) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    if U.size != P.nvar * P.nelem * P.nnode:
        raise ValueError("state size does not match the problem")
    return U


def rhs(P: Problem, U, return_Q: bool = False, lf_speed: float | None = None):
    """Weak-form DGSEM right-hand side (or_rhs_weak; or_nsk_rhs for the
    original NSK equations, where return_Q also returns the lifted Laplacian
    of rho and lf_speed, if given, replaces the global Lax-Friedrichs speed
    of U: or_nsk_rhs_lam)."""
    U = _state(P, U)
    R = np.zeros_like(U)
    if P.model == 1:
        Q = np.zeros((P.dim, P.dim + 1, P.nelem, P.nnode)) if return_Q else None
        lap = np.zeros((P.nelem, P.nnode)) if return_Q else None
        pc = P.c()
        qp, lp = (_ptr(Q) if return_Q else None), (_ptr(lap) if return_Q else None)
        if lf_speed is None:
            rc = lib().or_nsk_rhs(C.byref(pc), _ptr(U), _ptr(R), qp, lp)
        else:
            rc = lib().or_nsk_rhs_lam(C.byref(pc), _ptr(U), float(lf_speed), _ptr(R), qp, lp)
        if rc != 0:
            raise RuntimeError("or_nsk_rhs failed")
        R = R.reshape(P.shape())
        return (R, Q, lap) if return_Q else R
    Q = np.zeros((P.dim, P.dim + 1, P.nelem, P.nnode)) if return_Q else None
    pc = P.c()
    if lib().or_rhs_weak(C.byref(pc), _ptr(U), _ptr(R), _ptr(Q) if return_Q else None) != 0:
        raise RuntimeError("or_rhs_weak failed")
    R = R.reshape(P.shape())
    return (R, Q) if return_Q else R


def numflux(P: Problem, d: int, uL, uR) -> np.ndarray:
    """Convective numerical flux of the weak form between two point states."""
    uL = np.ascontiguousarray(uL, dtype=np.float64)
    uR = np.ascontiguousarray(uR, dtype=np.float64)
    F = np.zeros(P.nvar)
    pc = P.c()
    if lib().or_numflux(C.byref(pc), d, _ptr(uL), _ptr(uR), _ptr(F)) != 0:
        raise RuntimeError("or_numflux failed")
    return F


def rhs_strong(P: Problem, U):
    """Strong-form DGSEM right-hand side (or_rhs_strong)."""
    U = _state(P, U)
    R = np.zeros_like(U)
    pc = P.c()
    if lib().or_rhs_strong(C.byref(pc), _ptr(U), _ptr(R)) != 0:
        raise RuntimeError("or_rhs_strong failed")
    return R.reshape(P.shape())


def run(P: Problem, U, dt: float, nsteps: int, t0: float = 0.0, forcing=None):
    """LSRK4(5) integration (or_run).  ``forcing(t) -> array of U's shape``."""
    U = _state(P, U).copy()
    pc = P.c()
    if forcing is None:
        cb = FORCING()
    else:
        size = U.size

        def _f(t, out, _user):
            arr = np.ctypeslib.as_array(out, shape=(size,))
            arr[:] = np.ascontiguousarray(forcing(t), dtype=np.float64).ravel()

        cb = FORCING(_f)
    fn = lib().or_nsk_run if P.model == 1 else lib().or_run
    if fn(C.byref(pc), _ptr(U), dt, nsteps, t0, cb, None) != 0:
        raise RuntimeError("or_run failed")
    return U.reshape(P.shape())


def dt(P: Problem, U, cfl: float) -> float:
    U = _state(P, U)
    pc = P.c()
    if P.model == 1:
        return lib().or_nsk_dt(C.byref(pc), _ptr(U), cfl)
    return lib().or_dt(C.byref(pc), _ptr(U), cfl)


def subcell_matrices(N: int):
    """(M, M^{-1}): sub-cell averaging of the Lagrange basis (or_subcell_matrices)."""
    n = N + 1
    M, Mi = np.zeros(n * n), np.zeros(n * n)
    if lib().or_subcell_matrices(N, _ptr(M), _ptr(Mi)) != 0:
        raise RuntimeError("or_subcell_matrices failed")
    return M.reshape(n, n), Mi.reshape(n, n)


def persson(P: Problem, U) -> np.ndarray:
    """Persson-Peraire indicator of rho per element (or_persson)."""
    U = _state(P, U)
    ind = np.zeros(P.nelem)
    pc = P.c()
    if lib().or_persson(C.byref(pc), _ptr(U), _ptr(ind)) != 0:
        raise RuntimeError("or_persson failed")
    return ind


def rhs_subcell(P: Problem, U, threshold: float):
    """Right-hand side with FV sub-cells in troubled elements
    (or_rhs_subcell); returns (R, flags)."""
    U = _state(P, U)
    R = np.zeros_like(U)
    flags = np.zeros(P.nelem, dtype=np.int32)
    pc = P.c()
    if lib().or_rhs_subcell(C.byref(pc), _ptr(U), float(threshold), _ptr(R),
                            flags.ctypes.data_as(C.POINTER(C.c_int))) != 0:
        raise RuntimeError("or_rhs_subcell failed")
    return R.reshape(P.shape()), flags.astype(bool)


def lf_speed(P: Problem, U) -> float:
    """Global Lax-Friedrichs speed of the original NSK path (or_nsk_lf_speed)."""
    U = _state(P, U)
    pc = P.c()
    return lib().or_nsk_lf_speed(C.byref(pc), _ptr(U))


DIAG_KEYS = ["mass", "e_kin", "e_total", "l2_rho_minus_c", "rho_min", "rho_max", "max_wavespeed", "nonfinite"]


def diagnostics(P: Problem, U) -> dict:
    U = _state(P, U)
    out = np.zeros(16)
    pc = P.c()
    fn = lib().or_nsk_diagnostics if P.model == 1 else lib().or_diagnostics
    if fn(C.byref(pc), _ptr(U), _ptr(out)) != 0:
        raise RuntimeError("or_diagnostics failed")
    return {
        "mass": out[: P.nvar].copy(),
        "e_kin": out[7],
        "e_total": out[8],
        "l2_rho_minus_c": out[9],
        "rho_min": out[10],
        "rho_max": out[11],
        "max_wavespeed": out[12],
        "nonfinite": int(out[13]),
    }


def node_coords(P: Problem) -> np.ndarray:
    X = np.zeros((P.dim, P.nelem, P.nnode))
    pc = P.c()
    lib().or_node_coords(C.byref(pc), _ptr(X))
    return X


# --------------------------------------------------------------------------
# learned closure: network, training step, features, nudging
# --------------------------------------------------------------------------
MLP_NPARAM = 8770
CLOSURE_NORM_KEYS = ("s0", "k0", "s1", "k1", "k2", "k3", "g0", "out_m", "out_c")


def relu(z: float) -> float:
    return lib().or_relu(z)


def relu_d(z: float) -> float:
    return lib().or_relu_d(z)


def mlp_forward(w, X) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 4)
    Y = np.zeros((X.shape[0], 2))
    lib().or_mlp_forward(_ptr(w), _ptr(X), X.shape[0], _ptr(Y))
    return Y


def mlp_loss_grad(w, X, Yt):
    w = np.ascontiguousarray(w, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 4)
    Yt = np.ascontiguousarray(Yt, dtype=np.float64).reshape(-1, 2)
    g = np.zeros(MLP_NPARAM)
    loss = lib().or_mlp_loss_grad(_ptr(w), _ptr(X), _ptr(Yt), X.shape[0], _ptr(g))
    return loss, g


def adam_step(w, m, v, g, lr, b1, b2, eps, t):
    """In place on w, m, v (float64 arrays)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().or_adam_step(_ptr(w), _ptr(m), _ptr(v), _ptr(g), w.size, lr, b1, b2, eps, t)


def _norm(norm) -> np.ndarray:
    if isinstance(norm, dict):
        norm = [norm[k] for k in CLOSURE_NORM_KEYS]
    return np.ascontiguousarray(norm, dtype=np.float64)


def closure_features(P: Problem, U, norm):
    U = _state(P, U)
    S = P.nelem * P.nnode
    X = np.zeros((S, 4))
    nv = np.zeros((P.dim, S))
    nm = _norm(norm)
    pc = P.c()
    if lib().or_closure_features(C.byref(pc), _ptr(U), _ptr(nm), _ptr(X), _ptr(nv)) != 0:
        raise RuntimeError("or_closure_features failed")
    return X, nv


def closure_source(P: Problem, U, w, norm):
    U = _state(P, U)
    w = np.ascontiguousarray(w, dtype=np.float64)
    Sc = np.zeros_like(U).reshape(P.shape())
    nm = _norm(norm)
    pc = P.c()
    if lib().or_closure_source(C.byref(pc), _ptr(U), _ptr(w), _ptr(nm), _ptr(Sc)) != 0:
        raise RuntimeError("or_closure_source failed")
    return Sc


def closure_nudge(P: Problem, U, Uref, dt, tau, cmap, norm):
    """Returns (U_new, X, Y); U is not modified."""
    Un = _state(P, U).copy()
    Ur = _state(P, Uref)
    S = P.nelem * P.nnode
    X = np.zeros((S, 4))
    Y = np.zeros((S, 2))
    nm = _norm(norm)
    pc = P.c()
    if lib().or_closure_nudge(C.byref(pc), _ptr(Un), _ptr(Ur), dt, tau, cmap, _ptr(nm), _ptr(X), _ptr(Y)) != 0:
        raise RuntimeError("or_closure_nudge failed")
    return Un.reshape(P.shape()), X, Y
