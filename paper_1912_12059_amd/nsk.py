"""Python binding of libnsk (include/nsk.h): argument marshalling only.

Every function here forwards to the C entry point of the same name.  All
arithmetic of the method runs in the HIP kernels of ``csrc/``; PyTorch only
provides device memory and the stream.  Importing this module fails loudly when
the compiled library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnsk.so")

NSK_OK = 0
NSK_EINVAL = -1
NSK_ENONPHYS = -2
NSK_EHIP = -3
NSK_EUNBOUND = -4
NSK_EUNSUPPORTED = -5
NSK_ENOCONV = -6
NSK_ESCRATCH = -7
NSK_NOALLOC_SCRATCH_BYTES = 128 << 20
NSK_GMRES_MAX = 64


class NskError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {nsk_strerror(code)} ({code})")
        self.code = code


class nsk_mesh(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("N", C.c_int),
        ("nel", C.c_int * 3),
        ("lo", C.c_double * 3),
        ("hi", C.c_double * 3),
        ("xbreaks", C.POINTER(C.c_double) * 3),
    ]


class nsk_params(C.Structure):
    _fields_ = [
        ("T", C.c_double),
        ("eps", C.c_double),
        ("kappa", C.c_double),
        ("alpha", C.c_double),
        ("beta", C.c_double),
        ("flux", C.c_int),
        ("diss_c", C.c_int),
        ("precision", C.c_int),
        ("closure", C.c_int),
        ("model", C.c_int),
        ("subcell", C.c_int),
        ("subcell_threshold", C.c_double),
    ]


class nsk_closure_norm(C.Structure):
    _fields_ = [(k, C.c_float) for k in ("s0", "k0", "s1", "k1", "k2", "k3", "g0", "out_m", "out_c")]


NSK_MLP_NPARAM = 8770
NSK_CLOSURE_KEPT, NSK_CLOSURE_PARAMS, NSK_CLOSURE_NONPHYS, NSK_CLOSURE_ENERGY = 0, 1, 2, 3


class nsk_closure_report(C.Structure):
    _fields_ = [("fell_back", C.c_int), ("reason", C.c_int), ("closure_steps", C.c_longlong),
                ("fallback_steps", C.c_longlong), ("e_start", C.c_double), ("e_last", C.c_double)]


class nsk_implicit_opts(C.Structure):
    _fields_ = [
        ("newton_tol", C.c_double),
        ("newton_max", C.c_int),
        ("gmres_rtol", C.c_double),
        ("gmres_m", C.c_int),
        ("precond", C.c_int),
        ("basis_fp32", C.c_int),
        ("reorth_tol", C.c_double),
    ]


class nsk_implicit_stats(C.Structure):
    _fields_ = [
        ("steps", C.c_longlong),
        ("rhs_evals", C.c_longlong),
        ("newton_iters", C.c_longlong),
        ("gmres_iters", C.c_longlong),
        ("reorth", C.c_longlong),
        ("max_residual", C.c_double),
        ("converged", C.c_int),
    ]


class nsk_diag(C.Structure):
    _fields_ = [
        ("mass", C.c_double * 5),
        ("e_kin", C.c_double),
        ("e_total", C.c_double),
        ("l2_rho_minus_c", C.c_double),
        ("rho_min", C.c_double),
        ("rho_max", C.c_double),
        ("max_wavespeed", C.c_double),
        ("nonfinite", C.c_longlong),
        ("status", C.c_int),
    ]


_lib = None


def load() -> C.CDLL:
    """Load libnsk.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        L.nsk_create.argtypes = [C.POINTER(nsk_mesh), C.POINTER(nsk_params), C.POINTER(vp)]
        L.nsk_destroy.argtypes = [vp]
        L.nsk_destroy.restype = None
        L.nsk_state_size.argtypes = [vp]
        L.nsk_state_size.restype = C.c_size_t
        L.nsk_workspace_bytes.argtypes = [vp]
        L.nsk_workspace_bytes.restype = C.c_size_t
        L.nsk_bind.argtypes = [vp, vp, vp, vp, vp]
        L.nsk_set_state.argtypes = [vp, vp]
        L.nsk_get_state.argtypes = [vp, vp]
        L.nsk_rhs.argtypes = [vp, vp, vp, C.c_double]
        L.nsk_rhs_noalloc.argtypes = [vp, vp, vp, vp]
        L.nsk_dt_estimate.argtypes = [vp, C.c_double, dp]
        L.nsk_rk_step.argtypes = [vp, C.c_double, C.c_int]
        L.nsk_diagnostics.argtypes = [vp, C.POINTER(nsk_diag)]
        L.nsk_set_params.argtypes = [vp, C.POINTER(nsk_params)]
        L.nsk_set_tile.argtypes = [vp, C.c_int, C.c_int]
        L.nsk_autotune.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), dp]
        ip = C.POINTER(C.c_int)
        L.nsk_batch_create.argtypes = [C.POINTER(nsk_mesh), C.c_int, C.POINTER(nsk_params), C.POINTER(vp)]
        L.nsk_batch_destroy.argtypes = [vp]
        L.nsk_batch_destroy.restype = None
        L.nsk_batch_state_size.argtypes = [vp]
        L.nsk_batch_state_size.restype = C.c_size_t
        L.nsk_batch_state_offset.argtypes = [vp, C.c_int]
        L.nsk_batch_state_offset.restype = C.c_size_t
        L.nsk_batch_workspace_bytes.argtypes = [vp]
        L.nsk_batch_workspace_bytes.restype = C.c_size_t
        L.nsk_batch_bind.argtypes = [vp, vp, vp, vp, vp]
        L.nsk_batch_ctx.argtypes = [vp, C.c_int, C.POINTER(vp)]
        L.nsk_batch_dt_estimate.argtypes = [vp, C.c_double, dp]
        L.nsk_batch_rk_step.argtypes = [vp, C.c_double, C.c_int]
        L.nsk_batch_autotune.argtypes = [vp, C.c_int, dp]
        L.nsk_batch_groups.argtypes = [vp, ip, ip, ip, ip, ip, C.c_int]
        L.nsk_batch_set_group.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.nsk_timing_enable.argtypes = [vp, C.c_int]
        L.nsk_timing_read.argtypes = [vp, dp]
        L.nsk_subcell_flags.argtypes = [vp, vp]
        L.nsk_implicit_workspace_bytes.argtypes = [vp, C.c_int]
        L.nsk_implicit_workspace_bytes.restype = C.c_size_t
        L.nsk_esdirk_step.argtypes = [vp, vp, C.c_double, C.c_int, C.POINTER(nsk_implicit_opts),
                                      C.POINTER(nsk_implicit_stats)]
        fp = C.POINTER(C.c_float)
        L.nsk_closure_set.argtypes = [vp, vp, C.POINTER(nsk_closure_norm), C.c_int]
        L.nsk_closure_nudge.argtypes = [vp, C.POINTER(nsk_closure_norm), vp, C.c_double, C.c_double, C.c_double, vp,
                                        vp]
        L.nsk_closure_run.argtypes = [vp, vp, C.c_double, C.c_int, C.c_int, C.c_int, C.c_double,
                                      C.POINTER(nsk_closure_report)]
        L.nsk_mlp_forward.argtypes = [vp, vp, C.c_longlong, vp, vp]
        L.nsk_mlp_workspace_bytes.argtypes = [C.c_longlong]
        L.nsk_mlp_workspace_bytes.restype = C.c_size_t
        L.nsk_mlp_loss_grad.argtypes = [vp, vp, vp, vp, C.c_longlong, C.c_float, C.c_float, vp, vp, vp, vp]
        L.nsk_mlp_adam.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, vp]
        L.nsk_mlp_moments.argtypes = [vp, C.c_longlong, C.c_int, vp, vp, vp]
        del fp
        L.nsk_strerror.argtypes = [C.c_int]
        L.nsk_strerror.restype = C.c_char_p
        _lib = L
    return _lib


def _check(fn: str, rc: int) -> int:
    if rc != NSK_OK:
        raise NskError(fn, rc)
    return rc


def nsk_strerror(code: int) -> str:
    return load().nsk_strerror(code).decode()


def make_mesh(dim, N, nel, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), xbreaks=None):
    """Fill an nsk_mesh.  The returned keep-alive list must outlive the call
    to nsk_create (the library copies the breakpoints)."""
    m = nsk_mesh()
    m.dim, m.N = dim, N
    keep = []
    for d in range(3):
        m.nel[d] = int(nel[d]) if d < len(nel) else 1
        m.lo[d] = float(lo[d]) if d < len(lo) else 0.0
        m.hi[d] = float(hi[d]) if d < len(hi) else 1.0
        if xbreaks is not None and d < len(xbreaks) and xbreaks[d] is not None:
            arr = (C.c_double * len(xbreaks[d]))(*[float(v) for v in xbreaks[d]])
            keep.append(arr)
            m.xbreaks[d] = C.cast(arr, C.POINTER(C.c_double))
    return m, keep


def make_params(T=0.85, eps=1e-3, kappa=1e-5, alpha=500.0, beta=1e-3, diss_c=1, precision=0, flux=0, closure=0,
                model=0, subcell=0, subcell_threshold=0.0):
    """model 0: relaxation model II; model 1: the original NSK equations
    (flux 2, the global Lax-Friedrichs flux, is then the default)."""
    p = nsk_params()
    p.T, p.eps, p.kappa, p.alpha, p.beta = T, eps, kappa, alpha, beta
    if model == 1 and flux == 0:
        flux = 2
    p.flux, p.diss_c, p.precision, p.closure, p.model = flux, diss_c, precision, closure, model
    p.subcell, p.subcell_threshold = subcell, subcell_threshold
    return p


# ---- thin forwards, one per C entry point ---------------------------------
def nsk_create(mesh: nsk_mesh, params: nsk_params) -> int:
    h = C.c_void_p()
    _check("nsk_create", load().nsk_create(C.byref(mesh), C.byref(params), C.byref(h)))
    return h.value


def nsk_destroy(ctx: int) -> None:
    load().nsk_destroy(ctx)


def nsk_state_size(ctx: int) -> int:
    return load().nsk_state_size(ctx)


def nsk_workspace_bytes(ctx: int) -> int:
    return load().nsk_workspace_bytes(ctx)


def nsk_bind(ctx: int, d_U: int, d_dU: int, d_work: int, stream: int) -> None:
    _check("nsk_bind", load().nsk_bind(ctx, d_U, d_dU, d_work, stream))


def nsk_set_state(ctx: int, d_src: int) -> None:
    _check("nsk_set_state", load().nsk_set_state(ctx, d_src))


def nsk_get_state(ctx: int, d_dst: int) -> None:
    _check("nsk_get_state", load().nsk_get_state(ctx, d_dst))


def nsk_rhs(ctx: int, d_U: int, d_R: int, t: float = 0.0) -> None:
    _check("nsk_rhs", load().nsk_rhs(ctx, d_U, d_R, t))


def nsk_rhs_noalloc(ctx: int, d_U: int, d_R: int, stream: int = 0) -> None:
    _check("nsk_rhs_noalloc", load().nsk_rhs_noalloc(ctx, d_U, d_R, stream))


def nsk_dt_estimate(ctx: int, cfl: float) -> float:
    out = C.c_double()
    _check("nsk_dt_estimate", load().nsk_dt_estimate(ctx, cfl, C.byref(out)))
    return out.value


def nsk_rk_step(ctx: int, dt: float, nsteps: int) -> None:
    _check("nsk_rk_step", load().nsk_rk_step(ctx, dt, nsteps))


def nsk_diagnostics(ctx: int) -> tuple[int, nsk_diag]:
    d = nsk_diag()
    rc = load().nsk_diagnostics(ctx, C.byref(d))
    if rc not in (NSK_OK, NSK_ENONPHYS):
        raise NskError("nsk_diagnostics", rc)
    return rc, d


def nsk_set_params(ctx: int, params: nsk_params) -> None:
    _check("nsk_set_params", load().nsk_set_params(ctx, C.byref(params)))


def nsk_set_tile(ctx: int, variant: int, order: int) -> None:
    _check("nsk_set_tile", load().nsk_set_tile(ctx, variant, order))


def nsk_autotune(ctx: int, reps: int = 3) -> tuple[int, int, list]:
    v, r = C.c_int(), C.c_int()
    ms = (C.c_double * 12)()
    _check("nsk_autotune", load().nsk_autotune(ctx, reps, C.byref(v), C.byref(r), ms))
    return v.value, r.value, list(ms)


def nsk_timing_enable(ctx: int, enable: int) -> None:
    _check("nsk_timing_enable", load().nsk_timing_enable(ctx, enable))


def nsk_timing_read(ctx: int) -> tuple[float, float, int, float]:
    """(summed ms of the lifting kernel, of the right-hand-side kernel,
    number of stages timed, summed ms of the closure kernel)."""
    out = (C.c_double * 4)()
    _check("nsk_timing_read", load().nsk_timing_read(ctx, out))
    return out[0], out[1], int(out[2]), out[3]


def nsk_subcell_flags(ctx: int, d_flags_ptr: int) -> None:
    _check("nsk_subcell_flags", load().nsk_subcell_flags(ctx, d_flags_ptr))


def make_implicit_opts(newton_tol=1e-10, newton_max=20, gmres_rtol=1e-3, gmres_m=20, precond=0, basis_fp32=0,
                       reorth_tol=0.5):
    o = nsk_implicit_opts()
    o.newton_tol, o.newton_max, o.gmres_rtol, o.gmres_m = newton_tol, newton_max, gmres_rtol, gmres_m
    o.precond, o.basis_fp32, o.reorth_tol = precond, basis_fp32, reorth_tol
    return o


def nsk_implicit_workspace_bytes(ctx: int, gmres_m: int) -> int:
    return load().nsk_implicit_workspace_bytes(ctx, gmres_m)


def nsk_esdirk_step(ctx: int, iwork_ptr: int, dt: float, nsteps: int, opts: nsk_implicit_opts) -> dict:
    """Runs the steps; returns the statistics (raises NskError on failure,
    with the statistics in its .stats attribute)."""
    st = nsk_implicit_stats()
    rc = load().nsk_esdirk_step(ctx, iwork_ptr, dt, nsteps, C.byref(opts), C.byref(st))
    stats = {k: getattr(st, k) for k, _ in nsk_implicit_stats._fields_}
    if rc != NSK_OK:
        err = NskError("nsk_esdirk_step", rc)
        err.stats = stats
        raise err
    return stats


def nsk_batch_create(meshes: list, params: nsk_params) -> int:
    arr = (nsk_mesh * len(meshes))(*meshes)
    h = C.c_void_p()
    _check("nsk_batch_create", load().nsk_batch_create(arr, len(meshes), C.byref(params), C.byref(h)))
    return h.value


def nsk_batch_destroy(b: int) -> None:
    load().nsk_batch_destroy(b)


def nsk_batch_state_size(b: int) -> int:
    return load().nsk_batch_state_size(b)


def nsk_batch_state_offset(b: int, inst: int) -> int:
    return load().nsk_batch_state_offset(b, inst)


def nsk_batch_workspace_bytes(b: int) -> int:
    return load().nsk_batch_workspace_bytes(b)


def nsk_batch_bind(b: int, d_U: int, d_dU: int, d_work: int, stream: int) -> None:
    _check("nsk_batch_bind", load().nsk_batch_bind(b, d_U, d_dU, d_work, stream))


def nsk_batch_ctx(b: int, inst: int) -> int:
    h = C.c_void_p()
    _check("nsk_batch_ctx", load().nsk_batch_ctx(b, inst, C.byref(h)))
    return h.value


def nsk_batch_dt_estimate(b: int, cfl: float) -> float:
    out = C.c_double()
    _check("nsk_batch_dt_estimate", load().nsk_batch_dt_estimate(b, cfl, C.byref(out)))
    return out.value


def nsk_batch_rk_step(b: int, dt: float, nsteps: int) -> None:
    _check("nsk_batch_rk_step", load().nsk_batch_rk_step(b, dt, nsteps))


BATCH_TUNE_SLOTS = 12  # timings per group written by nsk_batch_autotune


def nsk_batch_autotune(b: int, reps: int = 2) -> list:
    ng = load().nsk_batch_groups(b, None, None, None, None, None, 0)
    ms = (C.c_double * (BATCH_TUNE_SLOTS * max(ng, 1)))()
    _check("nsk_batch_autotune", load().nsk_batch_autotune(b, reps, ms))
    return list(ms)


def nsk_batch_set_group(b: int, group: int, variant: int, gridmul: int, order: int, chunk_mib: int) -> None:
    _check("nsk_batch_set_group", load().nsk_batch_set_group(b, group, variant, gridmul, order, chunk_mib))


def nsk_batch_groups(b: int) -> list:
    n = load().nsk_batch_groups(b, None, None, None, None, None, 0)
    Ns, vs, gm, od, ch = ((C.c_int * n)() for _ in range(5))
    load().nsk_batch_groups(b, Ns, vs, gm, od, ch, n)
    return [{"N": Ns[i], "variant": vs[i], "gridmul": gm[i], "order": od[i], "chunk_mib": ch[i]} for i in range(n)]


def nsk_closure_set(ctx: int, d_w: int, norm: dict, every_stage: int = 1) -> None:
    nm = _norm_struct(norm)
    _check("nsk_closure_set", load().nsk_closure_set(ctx, d_w, C.byref(nm), every_stage))


def _norm_struct(norm: dict) -> nsk_closure_norm:
    full = {k: 0.0 for k in ("s0", "k0", "s1", "k1", "k2", "k3", "g0", "out_m", "out_c")}
    full.update(norm)
    return nsk_closure_norm(**{k: float(v) for k, v in full.items()})


def nsk_closure_run(cl: int, ref: int, dt: float, nsteps: int, ratio: int, check_every: int,
                    energy_tol: float = -1.0) -> dict:
    rep = nsk_closure_report()
    _check("nsk_closure_run", load().nsk_closure_run(cl, ref, dt, nsteps, ratio, check_every, energy_tol,
                                                     C.byref(rep)))
    return {k: getattr(rep, k) for k, _ in nsk_closure_report._fields_}


def nsk_closure_nudge(ctx: int, norm: dict, d_Uref: int, dt: float, tau: float, cmap: float, d_X: int,
                      d_Y: int) -> None:
    nm = _norm_struct(norm)
    _check("nsk_closure_nudge",
           load().nsk_closure_nudge(ctx, C.byref(nm), d_Uref, dt, tau, cmap, d_X or None, d_Y or None))


def nsk_mlp_forward(d_w: int, d_X: int, n: int, d_Y: int, stream: int) -> None:
    _check("nsk_mlp_forward", load().nsk_mlp_forward(d_w, d_X, n, d_Y, stream))


def nsk_mlp_workspace_bytes(batch: int) -> int:
    return load().nsk_mlp_workspace_bytes(batch)


def nsk_mlp_loss_grad(d_w: int, d_X: int, d_Y: int, d_idx: int, n: int, tscale0: float, tscale1: float, d_ws: int,
                      d_grad: int, d_loss: int, stream: int) -> None:
    _check("nsk_mlp_loss_grad",
           load().nsk_mlp_loss_grad(d_w, d_X, d_Y, d_idx or None, n, tscale0, tscale1, d_ws, d_grad, d_loss or None,
                                    stream))


def nsk_mlp_adam(d_master: int, d_w: int, d_m: int, d_v: int, d_grad: int, t: int, lr: float, beta1: float,
                 beta2: float, eps: float, stream: int) -> None:
    _check("nsk_mlp_adam", load().nsk_mlp_adam(d_master, d_w, d_m, d_v, d_grad, t, lr, beta1, beta2, eps, stream))


def nsk_mlp_moments(d_Y: int, n: int, ncol: int, d_ws: int, d_out: int, stream: int) -> None:
    _check("nsk_mlp_moments", load().nsk_mlp_moments(d_Y, n, ncol, d_ws, d_out, stream))


# ---- convenience owner of the device buffers (torch) ----------------------
@dataclass
class Solver:
    """Owns a context plus torch-allocated state, register and workspace."""

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
    precision: int = 0
    flux: int = 0
    closure: int = 0
    model: int = 0  # 0: relaxation model II, 1: original NSK (state rho, rho v)
    subcell: int = 0  # 1: FV sub-cells in elements whose indicator exceeds subcell_threshold
    subcell_threshold: float = 0.0
    xbreaks: list | None = None
    device: str = "cuda:0"
    stream: object = None
    ctx: int = field(default=0, init=False)

    def __post_init__(self):
        import torch

        mesh, keep = make_mesh(self.dim, self.N, self.nel, self.lo, self.hi, self.xbreaks)
        params = make_params(self.T, self.eps, self.kappa, self.alpha, self.beta, self.diss_c, self.precision,
                             flux=self.flux, closure=self.closure, model=self.model, subcell=self.subcell,
                             subcell_threshold=self.subcell_threshold)
        self.ctx = nsk_create(mesh, params)
        del keep
        n = nsk_state_size(self.ctx)
        self.nvar = self.dim + (1 if self.model == 1 else 2)
        self.nnode = (self.N + 1) ** self.dim
        self.nelem = n // (self.nvar * self.nnode)
        dev = torch.device(self.device)
        self.U = torch.zeros(n, dtype=torch.float64, device=dev)
        self.dU = torch.zeros(n, dtype=torch.float64, device=dev)
        self.work = torch.zeros(nsk_workspace_bytes(self.ctx) + 256, dtype=torch.uint8, device=dev)
        base = self.work.data_ptr()
        self._work_ptr = (base + 255) // 256 * 256
        if self.stream is None:
            self.stream = torch.cuda.current_stream(dev)
        self._after_torch()  # the zero fills above run on torch's current stream
        nsk_bind(self.ctx, self.U.data_ptr(), self.dU.data_ptr(), self._work_ptr, self.stream.cuda_stream)

    def _after_torch(self) -> None:
        """Order the bound stream after the work torch has enqueued on its
        current stream (allocation fills, host copies of inputs): torch's side
        streams do not synchronise with the null stream by themselves."""
        import torch

        cur = torch.cuda.current_stream(self.U.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    @property
    def shape(self):
        return (self.nvar, self.nelem, self.nnode)

    def set_state(self, U) -> None:
        import torch

        t = torch.as_tensor(U, dtype=torch.float64).reshape(-1).to(self.U.device).contiguous()
        if t.numel() != self.U.numel():
            raise ValueError("state size mismatch")
        self._after_torch()
        nsk_set_state(self.ctx, t.data_ptr())
        self.stream.synchronize()

    def get_state(self):
        import torch

        out = torch.empty_like(self.U)
        self._after_torch()
        nsk_get_state(self.ctx, out.data_ptr())
        self.stream.synchronize()
        return out.reshape(self.shape)

    def rhs(self, U):
        import torch

        t = torch.as_tensor(U, dtype=torch.float64).reshape(-1).to(self.U.device).contiguous()
        R = torch.empty_like(t)
        self._after_torch()
        nsk_rhs(self.ctx, t.data_ptr(), R.data_ptr(), 0.0)
        self.stream.synchronize()
        return R.reshape(self.shape)

    def rk_step(self, dt: float, nsteps: int = 1) -> None:
        nsk_rk_step(self.ctx, dt, nsteps)

    def dt_estimate(self, cfl: float) -> float:
        return nsk_dt_estimate(self.ctx, cfl)

    def subcell_flags(self):
        """Troubled-element flags of the last right-hand side (numpy bool)."""
        import torch

        f = torch.zeros(self.nelem, dtype=torch.int32, device=self.U.device)
        self._after_torch()
        nsk_subcell_flags(self.ctx, f.data_ptr())
        self.stream.synchronize()
        return f.cpu().numpy().astype(bool)

    def esdirk_step(self, dt: float, nsteps: int = 1, **opts) -> dict:
        """Implicit ESDIRK4(6) steps (nsk_esdirk_step); the Krylov workspace
        is allocated with torch on first use and kept for the same size."""
        import torch

        o = make_implicit_opts(**opts)
        need = nsk_implicit_workspace_bytes(self.ctx, o.gmres_m)
        if getattr(self, "_iwork", None) is None or self._iwork.numel() < need + 256:
            self._iwork = None
            self._iwork = torch.empty(need + 256, dtype=torch.uint8, device=self.U.device)
        ptr = (self._iwork.data_ptr() + 255) // 256 * 256
        self._after_torch()
        return nsk_esdirk_step(self.ctx, ptr, dt, nsteps, o)

    def diagnostics(self) -> dict:
        rc, d = nsk_diagnostics(self.ctx)
        return {
            "mass": list(d.mass)[: self.nvar],
            "e_kin": d.e_kin,
            "e_total": d.e_total,
            "l2_rho_minus_c": d.l2_rho_minus_c,
            "rho_min": d.rho_min,
            "rho_max": d.rho_max,
            "max_wavespeed": d.max_wavespeed,
            "nonfinite": d.nonfinite,
            "status": d.status,
        }

    def close(self) -> None:
        if self.ctx:
            nsk_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owns a batch of 3D instances plus torch-allocated packed state,
    register and workspace, and a dedicated stream (the step graph is
    captured on it)."""

    def __init__(self, meshes: list, T=0.85, eps=1e-3, kappa=1e-5, alpha=1000.0, beta=1e-3, diss_c=1,
                 precision=1, device="cuda:0"):
        import torch

        keep, cm = [], []
        for m in meshes:
            mm, k = make_mesh(3, m["N"], m["nel"], m.get("lo", (0.0, 0.0, 0.0)), m.get("hi", (1.0, 1.0, 1.0)))
            cm.append(mm)
            keep.append(k)
        params = make_params(T, eps, kappa, alpha, beta, diss_c, precision)
        self.b = nsk_batch_create(cm, params)
        self.ninst = len(meshes)
        dev = torch.device(device)
        self.stream = torch.cuda.Stream(dev)
        n = nsk_batch_state_size(self.b)
        self.U = torch.zeros(n, dtype=torch.float64, device=dev)
        self.dU = torch.zeros(n, dtype=torch.float64, device=dev)
        self.work = torch.zeros(nsk_batch_workspace_bytes(self.b) + 256, dtype=torch.uint8, device=dev)
        wp = (self.work.data_ptr() + 255) // 256 * 256
        torch.cuda.synchronize(dev)
        nsk_batch_bind(self.b, self.U.data_ptr(), self.dU.data_ptr(), wp, self.stream.cuda_stream)
        self.meshes = meshes
        self.sizes = []
        for i, m in enumerate(meshes):
            nn = (m["N"] + 1) ** 3
            self.sizes.append(5 * int(m["nel"][0]) * int(m["nel"][1]) * int(m["nel"][2]) * nn)

    def view(self, i: int):
        o = nsk_batch_state_offset(self.b, i)
        return self.U[o:o + self.sizes[i]]

    def set_state(self, i: int, U) -> None:
        import torch

        t = torch.as_tensor(U, dtype=torch.float64).reshape(-1)
        self.stream.synchronize()
        self.view(i).copy_(t.to(self.U.device))
        torch.cuda.synchronize(self.U.device)

    def get_state(self, i: int):
        self.stream.synchronize()
        return self.view(i).clone()

    def ctx(self, i: int) -> int:
        return nsk_batch_ctx(self.b, i)

    def dt_estimate(self, cfl: float) -> float:
        return nsk_batch_dt_estimate(self.b, cfl)

    def rk_step(self, dt: float, nsteps: int) -> None:
        nsk_batch_rk_step(self.b, dt, nsteps)

    def close(self) -> None:
        if self.b:
            nsk_batch_destroy(self.b)
            self.b = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

