"""Learned closure for relaxation model II: parameters, training pairs and
training, driven through the C ABI of libnsk.  Every arithmetic step
(features, nudging, network, loss gradient, Adam, moments, the closure source
in the right-hand side) runs in the library's kernels; this module allocates
device buffers with torch, draws the seeded random numbers (initial weights,
minibatch indices) and sequences the calls.

The closure (the paper has none) lets a run at a moderate relaxation
parameter alpha follow a run at a large alpha_ref.  Training pairs come from
a nudged run: the alpha run is pulled towards the alpha_ref run on a time
scale tau, with the reference c mapped into the alpha frame,
c* = rho_ref + (alpha_ref / alpha)(c_ref - rho_ref) (the relaxation
equilibrium alpha (c - rho) = kappa lap c does not depend on alpha), and the
pull per unit time is the target the network learns from the element-local
features of the alpha run's own state.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs, nsk

NPARAM = nsk.NSK_MLP_NPARAM
LAYOUT = (("W1", (64, 4)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 64)), ("b3", (64,)),
          ("W4", (2, 64)), ("b4", (2,)))


def to_bf16_bits(a) -> np.ndarray:
    """IEEE binary32 -> BF16 bit patterns, rounded to nearest even."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_bits_to_f64(b) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights for the layers followed by a ReLU (limit
    sqrt(6 / fan_in)), Glorot-uniform for the output layer, zero biases
    (numpy PCG64)."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for name, shape in LAYOUT:
        if name.startswith("W"):
            lim = math.sqrt(6.0 / (shape[0] + shape[1])) if name == "W4" else math.sqrt(6.0 / shape[1])
            out.append(g.uniform(-lim, lim, size=shape).ravel())
        else:
            out.append(np.zeros(shape[0]))
    p = np.concatenate(out).astype(np.float32)
    assert p.size == NPARAM
    return p


def default_norm(kappa: float) -> dict:
    """Feature scaling from the Maxwell densities and the equilibrium
    interface width 2 sqrt(kappa); output scales 1 until set from the
    targets."""
    k = inputs.constants()["maxwell"]
    rv, rl = k["rho_v"], k["rho_l"]
    dr, rm = rl - rv, 0.5 * (rl + rv)
    w0 = 2.0 * math.sqrt(kappa)
    return dict(s0=rm, k0=2.0 / dr, s1=rm, k1=2.0 / dr, k2=w0 / dr, k3=w0 * w0 / dr, g0=0.01 * dr / w0,
                out_m=1.0, out_c=1.0)


class Network:
    """FP32 master parameters, their BF16 copy (what the kernels read) and
    the Adam moments, on the device."""

    def __init__(self, params=None, seed: int = 0, device: str = "cuda:0"):
        import torch

        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        self.device = torch.device(device)
        self.master = torch.from_numpy(p.copy()).to(self.device)
        self.w = torch.from_numpy(to_bf16_bits(p).view(np.int16)).to(self.device)
        self.m = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.t = 0
        self.stream = torch.cuda.current_stream(self.device)

    @property
    def w_ptr(self) -> int:
        return self.w.data_ptr()

    def bf16_values(self) -> np.ndarray:
        """The parameters the network evaluates with, as float64."""
        self.stream.synchronize()
        return bf16_bits_to_f64(self.w.cpu().numpy().view(np.uint16))

    def forward(self, X):
        import torch

        X = X.contiguous()
        Y = torch.empty((X.shape[0], 2), dtype=torch.float32, device=self.device)
        nsk.nsk_mlp_forward(self.w_ptr, X.data_ptr(), X.shape[0], Y.data_ptr(), self.stream.cuda_stream)
        return Y

    def loss_grad(self, X, Y, idx=None, tscale=(1.0, 1.0), ws=None):
        import torch

        n = X.shape[0] if idx is None else idx.shape[0]
        if ws is None:
            ws = torch.empty(nsk.nsk_mlp_workspace_bytes(n), dtype=torch.uint8, device=self.device)
        grad = torch.empty(NPARAM, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        nsk.nsk_mlp_loss_grad(self.w_ptr, X.data_ptr(), Y.data_ptr(), 0 if idx is None else idx.data_ptr(), n,
                              tscale[0], tscale[1], ws.data_ptr(), grad.data_ptr(), loss.data_ptr(),
                              self.stream.cuda_stream)
        return loss, grad

    def adam(self, grad, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        self.t += 1
        nsk.nsk_mlp_adam(self.master.data_ptr(), self.w_ptr, self.m.data_ptr(), self.v.data_ptr(), grad.data_ptr(),
                         self.t, lr, beta1, beta2, eps, self.stream.cuda_stream)

    def train(self, X, Y, steps: int, batch: int = 32768, lr: float = 2e-3, lr_final: float = 2e-4,
              tscale=(1.0, 1.0), seed: int = 0, log_every: int = 0, chunk: int = 256):
        """Adam on random minibatches; learning rate decays geometrically
        from lr to lr_final.  The minibatch indices are drawn on the host
        (numpy PCG64 with the given seed) and uploaded `chunk` steps at a
        time.  Returns the sampled losses."""
        import torch

        g = np.random.Generator(np.random.PCG64(seed))
        ws = torch.empty(nsk.nsk_mlp_workspace_bytes(batch), dtype=torch.uint8, device=self.device)
        n = X.shape[0]
        losses = []
        idx_all = None
        for k in range(steps):
            if k % chunk == 0:
                m = min(chunk, steps - k)
                draw = g.integers(0, n, size=(m, batch), dtype=np.int32)
                idx_all = torch.from_numpy(draw).to(self.device)
            idx = idx_all[k % chunk]
            loss, grad = self.loss_grad(X, Y, idx, tscale, ws)
            rate = lr * (lr_final / lr) ** (k / max(steps - 1, 1))
            self.adam(grad, rate)
            if log_every and (k % log_every == 0 or k == steps - 1):
                losses.append((k, float(loss.item())))
        return losses

    def save(self, path: str) -> None:
        self.stream.synchronize()
        np.savez(path, master=self.master.cpu().numpy(), w=self.w.cpu().numpy())

    @classmethod
    def load(cls, path: str, device: str = "cuda:0") -> "Network":
        import torch

        with np.load(path, allow_pickle=False) as z:
            net = cls(params=z["master"], device=device)
            net.w.copy_(torch.from_numpy(z["w"]).to(net.device))
        return net


def moments(Y):
    """(means, standard deviations) of the columns of a device array."""
    import torch

    ncol = Y.shape[1]
    ws = torch.empty(nsk.nsk_mlp_workspace_bytes(1), dtype=torch.uint8, device=Y.device)
    out = torch.empty(2 * ncol, dtype=torch.float64, device=Y.device)
    nsk.nsk_mlp_moments(Y.data_ptr(), Y.shape[0], ncol, ws.data_ptr(), out.data_ptr(),
                        torch.cuda.current_stream(Y.device).cuda_stream)
    o = out.cpu().numpy()
    return o[:ncol], o[ncol:]


def nudged_pairs(mesh: dict, U0, alpha_ref: float, alpha: float, kappa: float, tend: float, norm: dict,
                 tau_steps: float = 100.0, record_every: int = 40, cfl: float = 0.5, progress=None, **phys):
    """Training pairs from one nudged run.  mesh: Solver mesh keywords (dim,
    N, nel, lo, hi); U0: initial state.  The alpha run takes its own time
    step dt; the alpha_ref run takes M = ceil(dt / dt_ref) steps of dt / M
    (within its own limit dt_ref) per alpha step, and the alpha run is nudged
    after every step toward the reference at the same time, with
    tau = tau_steps * dt.  Returns (X, Y) on the device, one row per node of
    every recorded step, and the step sizes (info["dt_ref"] = dt / M). progress(step, nsteps), if given, is called after every
    recorded step."""
    import torch

    ref = nsk.Solver(alpha=alpha_ref, kappa=kappa, **mesh, **phys)
    mod = nsk.Solver(alpha=alpha, kappa=kappa, **mesh, **phys)
    ref.set_state(U0)
    mod.set_state(U0)
    dt = mod.dt_estimate(cfl)
    M = max(1, math.ceil(dt / ref.dt_estimate(cfl) * (1.0 - 1e-12)))
    dt_ref = dt / M
    nsteps = int(round(tend / dt))
    S = ref.nelem * ref.nnode
    nrec = nsteps // record_every
    X = torch.empty((nrec * S, 4), dtype=torch.float32, device=ref.U.device)
    Y = torch.empty((nrec * S, 2), dtype=torch.float32, device=ref.U.device)
    tau = tau_steps * dt
    cmap = alpha_ref / alpha
    k = 0
    for step in range(1, nsteps + 1):
        ref.rk_step(dt_ref, M)
        mod.rk_step(dt, 1)
        rec = step % record_every == 0 and k < nrec
        xp = X[k * S:].data_ptr() if rec else 0
        yp = Y[k * S:].data_ptr() if rec else 0
        nsk.nsk_closure_nudge(mod.ctx, norm, ref.U.data_ptr(), dt, tau, cmap, xp, yp)
        k += int(rec)
        if rec and progress is not None:
            torch.cuda.synchronize()
            progress(step, nsteps)
    torch.cuda.synchronize()
    info = {"dt_ref": dt_ref, "dt": dt, "M": M, "steps": nsteps, "records": nrec}
    ref.close()
    mod.close()
    return X, Y, info


def closure_solver(net: Network, norm: dict, every_stage: int = 1, **kw) -> "nsk.Solver":
    """A Solver with the closure switched on and this network set, evaluated
    in every stage or once per step (every_stage = 0)."""
    s = nsk.Solver(closure=1, **kw)
    nsk.nsk_closure_set(s.ctx, net.w_ptr, norm, every_stage)
    s._closure_net = net  # keep the parameters alive while the solver steps
    return s
