"""Benchmark: DOF-stage updates per second of the explicit DGSEM right-hand
side plus low-storage Runge-Kutta update for relaxation model II, on one GPU.

A step is one full five-stage Runge-Kutta step over the whole mesh (lifting,
volume and surface integrals, source and update in every stage).  The default
workload is the 3D head-on droplet collision: periodic box [0,2]x[0,1]^2,
96x48x48 elements, N = 4 (27,648,000 nodes, 5 variables), alpha = 1000,
beta = 1e-3, eps = 1e-3, kappa = 1e-5, We = 100, FP64.  Inputs are generated
once on the host and are resident in HBM before the timed region starts.

Prints ONE JSON line.  Fields beyond the common contract:
  roofline      dominant kernel (right-hand side + stage update): algorithmic
                bytes per launch / its mean duration from HIP events recorded
                on the bound stream during the timed steps, against 8 TB/s
  cpu_baseline  the CPU oracle timed on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

REPO = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, REPO)

METRIC = "DOF-stage updates/s (DG RHS+RK) plain FP64 vs closure/mixed at fixed L2 error"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (builder kwargs, physics)
    "3d-collision": dict(dim=3, nel=(96, 48, 48), N=4, lo=(0.0, 0.0, 0.0), hi=(2.0, 1.0, 1.0), We=100.0,
                         alpha=1000.0),
    "2d-droplets": dict(dim=2, nel=(96, 96), N=4, lo=(0.0, 0.0), hi=(1.0, 1.0), alpha=2000.0),
}


KERNEL_SOURCES = ("dg_kernels.hpp", "host_common.hpp", "nsk.hip")


def counter_traffic(workload: str, precision: str, tile) -> dict | None:
    """HBM bytes per launch of the right-hand-side kernel from the committed
    rocprofv3 counter summary, if that summary was taken on the kernel
    sources as they are now, on this workload, precision and tile."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(REPO, "paper_1912_12059_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()
    for path in sorted(glob.glob(os.path.join(REPO, "profiles", "*hbm_traffic.md"))):
        with open(path) as fh:
            text = fh.read()
        if "```json" not in text:
            continue
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        if (rec.get("source_sha256") == sha and rec.get("workload", "").split()[0] == workload
                and rec.get("precision") == precision and list(rec.get("tile", [])) == list(tile)):
            return {"bytes": rec["traffic_bytes_per_launch"], "lift_bytes": rec.get("lift_traffic_bytes_per_launch"),
                    "source": os.path.relpath(path, REPO)}
    return None


def bytes_per_node(dim: int, stage_first: bool, mixed: bool) -> dict:
    """Algorithmic HBM bytes per node of each kernel of one stage.
    lift: read U (nvar words), write G (tau + grad c: dim(dim+1)/2 + dim).
    rhs : read U and G, read the register dU (not in the first stage, whose
          coefficient A is zero), write U_new and dU."""
    nvar = dim + 2
    ng = dim * (dim + 1) // 2 + dim
    gw = 4 if mixed else 8
    lift = 8 * nvar + gw * ng
    rhs = 8 * nvar + gw * ng + (0 if stage_first else 8 * nvar) + 16 * nvar
    return {"lift": lift, "rhs": rhs}


def build_state(name: str):
    from paper_1912_12059_amd import inputs as I

    w = WORKLOADS[name]
    if w["dim"] == 3:
        return I.collision_3d(nel=w["nel"], N=w["N"], We=w["We"], lo=w["lo"], hi=w["hi"])
    return I.droplets_2d(nel=w["nel"][0], N=w["N"])


def sample_block(U, nel, block):
    """Elements of the sub-box [x0, x0+bx) x [y0, y0+by) x [z0, z0+bz) of a
    state U[var][elem][node] (x-fastest element order), as a new state."""
    import numpy as np

    dim = len(nel)
    rng = [np.arange(b0, b0 + nb) for b0, nb in block]
    if dim == 3:
        ez, ey, ex = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
        idx = (ex + nel[0] * (ey + nel[1] * ez)).reshape(-1)
    else:
        ey, ex = np.meshgrid(rng[1], rng[0], indexing="ij")
        idx = (ex + nel[0] * ey).reshape(-1)
    return np.ascontiguousarray(U[:, idx, :])


_ORACLE = None


def oracle():
    """The CPU oracle for the timing legs: its sources built -O3
    -march=native for this host (the checker the tests load is a portable
    -O2 build of the same sources)."""
    global _ORACLE
    if _ORACLE is None:
        import tempfile

        from oracle import oracle as O

        path = os.path.join(tempfile.mkdtemp(prefix="nsk_oracle_"), "liboracle_native.so")
        O.build(path=path, native=True)
        O.use(path)
        _ORACLE = O
    return _ORACLE


def host_record() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "omp_num_threads": os.environ.get("OMP_NUM_THREADS"), "cpu_model": model,
            "oracle_build": "gcc -O3 -march=native -fopenmp (built on this host)"}


def _oracle_rate_one_thread(P_kw: dict, sample, dt: float, steps: int) -> float | None:
    """DOF-stage/s of the oracle on one thread: the same sample timed in a
    child process started with OMP_NUM_THREADS=1."""
    import subprocess
    import tempfile

    import numpy as np

    O = oracle()
    d = tempfile.mkdtemp(prefix="nsk_cpu1_")
    np.save(os.path.join(d, "U.npy"), sample)
    with open(os.path.join(d, "job.json"), "w") as fh:
        json.dump({"P": P_kw, "dt": dt, "steps": steps, "lib": O._lib._name}, fh)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-one-thread", d], env=env,
                           capture_output=True, text=True, timeout=300)
        el = float(json.loads(r.stdout.strip().splitlines()[-1])["seconds"])
    except Exception:  # the 1-thread figure is informative only
        return None
    return sample.shape[1] * sample.shape[2] * 5 * steps / el


def cpu_one_thread_child(d: str) -> int:
    import numpy as np

    from oracle import oracle as O

    with open(os.path.join(d, "job.json")) as fh:
        job = json.load(fh)
    O.use(job["lib"])
    P = O.Problem(**{k: (tuple(v) if isinstance(v, list) else v) for k, v in job["P"].items()})
    U = np.load(os.path.join(d, "U.npy"))
    t0 = time.perf_counter()
    O.run(P, U, job["dt"], job["steps"])
    print(json.dumps({"seconds": time.perf_counter() - t0}))
    return 0


def cpu_baseline(name: str, sample, sub, budget_s: float = 20.0):
    """Time the CPU oracle (as it stands) on a bounded sample: a block of
    elements cut out of the same initial state, treated as a periodic box with
    the same element size, degree and physics; full LSRK4(5) steps; rate in
    DOF-stage updates per second."""
    O = oracle()

    w = WORKLOADS[name]
    dim = w["dim"]
    h = [(w["hi"][d] - w["lo"][d]) / w["nel"][d] for d in range(dim)]
    nel3 = tuple(sub) + (1,) * (3 - dim)
    hi3 = tuple(sub[d] * h[d] for d in range(dim)) + (1.0,) * (3 - dim)
    P_kw = dict(dim=dim, N=w["N"], nel=nel3, lo=(0, 0, 0), hi=hi3, alpha=w["alpha"], beta=1e-3, eps=1e-3,
                kappa=1e-5)
    P = O.Problem(**P_kw)
    dt = O.dt(P, sample, 0.5)
    t0 = time.perf_counter()
    O.run(P, sample, dt, 1)
    first = time.perf_counter() - t0
    steps = int(min(60, max(1, budget_s // max(first, 1e-3))))
    t0 = time.perf_counter()
    O.run(P, sample, dt, steps)
    el = time.perf_counter() - t0
    dofs = sample.shape[1] * sample.shape[2]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # one thread: about 10 s of work
    steps1 = int(max(1, min(steps, 10.0 // max(first * threads, 1e-3))))
    return {
        "value": dofs * 5 * steps / el,
        "unit": "DOF-stage/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{'x'.join(map(str, sub))}-element block of the same initial state (periodic, same "
                  f"element size, N={w['N']} and physics), {steps} LSRK4(5) steps in {el:.1f} s",
        "value_one_thread": _oracle_rate_one_thread(P_kw, sample, dt, steps1),
        "one_thread_steps": steps1,
        "host": host_record(),
    }


def run_form(nsk, m, U0, w, precision: int, steps: int, warmup: int, tile: str, flux: int = 0, model: int = 0,
             subcell_threshold=None):
    """Time `steps` LSRK4(5) steps of one form (precision, numerical flux,
    model) from the resident state U0 (torch, device).  Returns timings, the
    stage-kernel means from HIP events on the bound stream, and the final
    state (device)."""
    import torch

    sc = {} if subcell_threshold is None else dict(subcell=1, subcell_threshold=subcell_threshold)
    s = nsk.Solver(dim=m.dim, N=m.N, nel=tuple(m.nel), lo=tuple(m.lo), hi=tuple(m.hi), alpha=w["alpha"],
                   beta=1e-3, eps=1e-3, kappa=1e-5, precision=precision, flux=flux, model=model, **sc)
    s.set_state(U0)
    dt = s.dt_estimate(0.5)
    if tile == "auto":
        variant, order, tune_ms = nsk.nsk_autotune(s.ctx, 3)
    else:
        variant, order = (int(x) for x in tile.split(","))
        nsk.nsk_set_tile(s.ctx, variant, order)
        tune_ms = None
    print(f"[bench] precision={precision} tile variant={variant} order={order} dt={dt:.4e}", file=sys.stderr,
          flush=True)
    # warm-up from the initial state, then restart from it for the timed steps
    s.rk_step(dt, warmup)
    s.set_state(U0)
    torch.cuda.synchronize()
    nsk.nsk_timing_enable(s.ctx, 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    t0 = time.perf_counter()
    s.rk_step(dt, steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_lift, ms_rhs, nst, ms_mid = nsk.nsk_timing_read(s.ctx)
    nsk.nsk_timing_enable(s.ctx, 0)
    troubled = float(s.subcell_flags().mean()) if subcell_threshold is not None else None
    diag = s.diagnostics()
    final = s.get_state()
    s.close()
    return {"ms": ms, "wall": wall, "ms_lift": ms_lift / max(nst, 1), "ms_rhs": ms_rhs / max(nst, 1),
            "ms_mid": ms_mid / max(nst, 1), "dt": dt, "variant": variant, "order": order, "tune_ms": tune_ms,
            "diag": diag, "final": final, "troubled": troubled}


def nsk_bytes_per_node(dim: int, stage_first: bool) -> dict:
    """Algorithmic HBM bytes per node of each kernel of one stage of the
    original NSK path (FP64, nvar = dim + 1 words of state).
    lift: read U, write G (tau and grad rho: dim(dim+1)/2 + dim).
    lap : read grad rho, tau and rho, write Sigma (dim(dim+1)/2).
    rhs : read U and Sigma, read dU (not in the first stage), write U, dU."""
    nvar = dim + 1
    nt = dim * (dim + 1) // 2
    lift = 8 * (nvar + nt + dim)
    lap = 8 * (dim + nt + 1 + nt)
    rhs = 8 * (nvar + nt) + (0 if stage_first else 8 * nvar) + 16 * nvar
    return {"lift": lift, "lap": lap, "rhs": rhs}


def run_nsk_form(nsk, m, U0, w, steps: int, warmup: int, tile: str, ref: dict):
    """The original NSK equations (Korteweg stress, second lifting, global
    Lax-Friedrichs flux) on the same workload, FP64: rate, kernel times and
    roofline fractions, and the simulated time per wall-clock second against
    the relaxation model (ref: the FP64 model II run)."""
    nsk_U0 = U0.reshape(m.nvar, -1)[: m.dim + 1].contiguous()
    r = run_form(nsk, m, nsk_U0, w, 0, steps, warmup, tile, flux=2, model=1)
    dofs = m.nelem * m.nnode
    b1, b = nsk_bytes_per_node(m.dim, True), nsk_bytes_per_node(m.dim, False)
    rhs_bytes = dofs * (b1["rhs"] + 4 * b["rhs"]) / 5.0
    frac = lambda nbytes, ms: nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS if ms > 0 else None
    ms_step = r["ms"] / steps
    return {
        "value": dofs * 5 * steps / (r["ms"] * 1e-3), "unit": "DOF-stage/s", "ms_per_step": ms_step,
        "lift_ms": r["ms_lift"], "lap_and_reduce_ms": r["ms_mid"], "rhs_ms": r["ms_rhs"],
        "rhs_roofline_frac": frac(rhs_bytes, r["ms_rhs"]),
        "lift_roofline_frac": frac(dofs * b["lift"], r["ms_lift"]),
        "lap_roofline_frac": frac(dofs * b["lap"], r["ms_mid"]),
        "stage_bytes_per_node": b["lift"] + b["lap"] + b["rhs"],
        "dt": r["dt"], "dt_model2_alpha": {"alpha": w["alpha"], "dt": ref["dt"]},
        "sim_time_per_wall_s": r["dt"] / (ms_step * 1e-3),
        "sim_time_per_wall_s_model2": ref["dt"] / (ref["ms"] / steps * 1e-3),
        "status_after": r["diag"]["status"],
        "tile": {"variant": r["variant"], "order": r["order"]},
        "physics": "kappa=1e-5, eps=1e-3, no alpha/beta; state (rho, rho v) of the same collision",
    }


def run_subcell_form(nsk, m, U0, w, ref: dict, thresholds=(-7.5, -9.0, -12.0, -1e9), steps: int = 10,
                     warmup: int = 2):
    """FV sub-cell shock capturing (model II, FP64) on the same workload at
    several indicator thresholds (the last one troubles every element): rate
    against the FP64 DG run, the troubled fraction at the last stage, and the
    stage time split into the lifting, the indicator/means kernels and the DG
    right-hand side plus the FV sub-cell kernel."""
    dofs = m.nelem * m.nnode
    out = []
    for thr in thresholds:
        r = run_form(nsk, m, U0, w, 0, steps, warmup, "0,4", subcell_threshold=thr)
        out.append({"threshold": thr, "troubled_fraction": r["troubled"],
                    "value": dofs * 5 * steps / (r["ms"] * 1e-3), "unit": "DOF-stage/s",
                    "ms_per_step": r["ms"] / steps, "rel_to_dg_fp64": (ref["ms"] / ref["steps"]) / (r["ms"] / steps),
                    "lift_ms": r["ms_lift"], "indicator_and_means_ms": r["ms_mid"],
                    "dg_rhs_plus_fv_ms": r["ms_rhs"], "status_after": r["diag"]["status"]})
        print(f"[bench] subcell threshold {thr:g}: troubled {r['troubled']:.4f}, {r['ms'] / steps:.2f} ms/step",
              file=sys.stderr, flush=True)
    return out


def run_implicit_form(nsk, m, U0, w, factors=(100, 200), reference: bool = True):
    """Implicit ESDIRK4(6) steps (Jacobian-free Newton-GMRES with the
    node-local source preconditioner, an FP32 Krylov basis and a second
    Gram-Schmidt pass only when 99.5% of a vector's norm cancels; state,
    right-hand sides and Newton residuals FP64) on the same workload, one step
    each of `factor` times the explicit step, against the explicit LSRK4(5)
    over the same simulated time: wall time, solver counts, and the relative
    L2 difference of rho between the two integrators."""
    import torch

    s = nsk.Solver(dim=m.dim, N=m.N, nel=tuple(m.nel), lo=tuple(m.lo), hi=tuple(m.hi), alpha=w["alpha"],
                   beta=1e-3, eps=1e-3, kappa=1e-5)
    s.set_state(U0)
    nsk.nsk_autotune(s.ctx, 3)
    dte = s.dt_estimate(0.5)
    opts = dict(precond=1, gmres_m=40, newton_tol=1e-8, gmres_rtol=1e-3, newton_max=20, basis_fp32=1,
                reorth_tol=0.01)
    out = {"dt_explicit": dte, "opts": opts, "steps": []}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for fac in factors:
        ms_exp, ref = float("nan"), None
        if reference:
            s.set_state(U0)
            torch.cuda.synchronize()
            e0.record(s.stream)
            s.rk_step(dte, fac)
            e1.record(s.stream)
            torch.cuda.synchronize()
            ms_exp = e0.elapsed_time(e1)
            ref = s.get_state()[0].clone()
        s.set_state(U0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.esdirk_step(fac * dte, 1, **opts)
        torch.cuda.synchronize()
        ms_imp = (time.perf_counter() - t0) * 1e3
        got = s.get_state()[0]
        l2 = float(torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref)) if reference else None
        print(f"[bench] implicit x{fac}: {ms_imp:.0f} ms vs explicit {ms_exp:.0f} ms", file=sys.stderr, flush=True)
        out["steps"].append({"factor": fac, "dt": fac * dte, "implicit_ms": ms_imp, "explicit_ms": ms_exp,
                             "speedup_vs_explicit": ms_exp / ms_imp, "l2_rel_rho_vs_explicit": l2, **st})
        del ref, got
    s.close()
    return out


def run_batched(nsk, steps: int, warmup: int, compare_steps: int = 20):
    """The batched collision sweep: 24 3D head-on collisions (n_x x 32 x 32
    elements, n_x in 32..64, N in {3,4,5}, We ~ U[5,150], impact ~ U[0,0.5] R,
    alpha = 1000) in mixed precision, advanced as one batch (per-degree
    persistent kernels, two steps per graph replay) for `steps` steps,
    against the same 24 instances run one after another, mixed and plain
    FP64, for the first compare_steps of them (rates, and the L2 of rho
    against FP64 at that step)."""
    import torch

    from paper_1912_12059_amd import inputs as I

    sweep = I.batched_sweep()
    steps += steps % 2  # whole graph replays
    meshes = [{"nel": s["nel"], "N": s["N"], "lo": s["lo"], "hi": s["hi"]} for s in sweep]
    print(f"[bench] batched sweep: {len(sweep)} instances", file=sys.stderr, flush=True)
    init = []
    for s in sweep:
        _, U = I.collision_3d(nel=s["nel"], N=s["N"], We=s["We"], radius=s["radius"], lo=s["lo"], hi=s["hi"],
                              impact=s["impact"], device="cuda:0")
        init.append(U.reshape(-1))
    dofs = [u.numel() // 5 for u in init]
    b = nsk.Batch(meshes, alpha=1000.0, beta=1e-3, eps=1e-3, kappa=1e-5, precision=1)
    for i, u in enumerate(init):
        b.set_state(i, u)
    dt = b.dt_estimate(0.5)
    tune_ms = nsk.nsk_batch_autotune(b.b, 2)
    groups = nsk.nsk_batch_groups(b.b)
    b.rk_step(dt, warmup + warmup % 2)
    for i, u in enumerate(init):
        b.set_state(i, u)
    compare_steps = min(compare_steps + compare_steps % 2, steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(b.stream)
    b.rk_step(dt, compare_steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms_batch = e0.elapsed_time(e1)
    finals = [b.get_state(i) for i in range(len(sweep))]
    if steps > compare_steps:
        e0.record(b.stream)
        b.rk_step(dt, steps - compare_steps)
        e1.record(b.stream)
        torch.cuda.synchronize()
        ms_batch += e0.elapsed_time(e1)
    physical = True
    for i in range(len(sweep)):
        rho = b.get_state(i).reshape(5, -1)[0]
        physical &= bool(torch.isfinite(rho).all()) and float(rho.min()) > 0.0 and float(rho.max()) < 3.0
    b.close()
    del b
    # the same instances one after another (single-mesh launches), same
    # states and dt: mixed for what batching gains, FP64 as the reference
    ms_seq, l2max = {0: 0.0, 1: 0.0}, 0.0
    for i, s in enumerate(sweep):
        for prec in (1, 0):
            sv = nsk.Solver(dim=3, N=s["N"], nel=s["nel"], lo=s["lo"], hi=s["hi"], alpha=1000.0, beta=1e-3,
                            eps=1e-3, kappa=1e-5, precision=prec)
            sv.set_state(init[i])
            nsk.nsk_autotune(sv.ctx, 2)
            sv.rk_step(dt, 1)
            sv.set_state(init[i])
            torch.cuda.synchronize()
            e0.record(sv.stream)
            sv.rk_step(dt, compare_steps)
            e1.record(sv.stream)
            torch.cuda.synchronize()
            ms_seq[prec] += e0.elapsed_time(e1)
            if prec == 0:
                ref = sv.get_state().reshape(-1)
                n = dofs[i]  # rho is the first variable
                l2 = float(torch.linalg.vector_norm(finals[i].reshape(-1)[:n] - ref[:n])
                           / torch.linalg.vector_norm(ref[:n]))
                l2max = max(l2max, l2)
            sv.close()
    work = sum(dofs) * 5 * steps
    seq_work = sum(dofs) * 5 * compare_steps
    return {
        "instances": len(sweep),
        "dofs": sum(dofs),
        "steps": steps,
        "dt": dt,
        "precision": "mixed (FP32 volume/surface, FP64 state, RK, source, near-spinodal EoS)",
        "value": work / (ms_batch * 1e-3),
        "unit": "DOF-stage/s",
        "ms_per_step": ms_batch / steps,
        "all_physical_after_steps": physical,
        "compare_steps": compare_steps,
        "sequential_mixed_value": seq_work / (ms_seq[1] * 1e-3),
        "sequential_fp64_value": seq_work / (ms_seq[0] * 1e-3),
        "speedup_vs_sequential_mixed": (work / (ms_batch * 1e-3)) / (seq_work / (ms_seq[1] * 1e-3)),
        "speedup_vs_sequential_fp64": (work / (ms_batch * 1e-3)) / (seq_work / (ms_seq[0] * 1e-3)),
        "max_l2_rel_rho_vs_fp64": l2max,
        "l2_note": f"relative L2 of rho, batched mixed against sequential FP64, after {compare_steps} steps",
        "groups": groups,
        "autotune_ms": tune_ms[: nsk.BATCH_TUNE_SLOTS * len(groups)],
    }


def run_batched_small(nsk, steps: int = 20, n: int = 64):
    """Launch-bound case beside the sweep: n small collisions (8x8x8
    elements, N = 3, 32,768 nodes each) in mixed precision, batched (one
    graph replay per two steps) against the same instances run one after
    another."""
    import torch

    from paper_1912_12059_amd import inputs as I

    mesh = {"nel": (8, 8, 8), "N": 3, "lo": (0.0, 0.0, 0.0), "hi": (1.0, 1.0, 1.0)}
    meshes = [dict(mesh) for _ in range(n)]
    init = []
    for i in range(n):
        _, U = I.collision_3d(nel=(8, 8, 8), N=3, We=5.0 + 2.0 * i, radius=0.1, hi=(1.0, 1.0, 1.0),
                              impact=0.001 * i, device="cuda:0")
        init.append(U.reshape(-1))
    dofs = init[0].numel() // 5
    b = nsk.Batch(meshes, alpha=1000.0, beta=1e-3, eps=1e-3, kappa=1e-5, precision=1)
    for i, u in enumerate(init):
        b.set_state(i, u)
    dt = b.dt_estimate(0.5)
    nsk.nsk_batch_autotune(b.b, 2)
    b.rk_step(dt, 2)
    for i, u in enumerate(init):
        b.set_state(i, u)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(b.stream)
    b.rk_step(dt, steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    b.close()
    solvers = [nsk.Solver(dim=3, N=3, nel=(8, 8, 8), alpha=1000.0, beta=1e-3, eps=1e-3, kappa=1e-5, precision=1)
               for _ in range(n)]
    for s, u in zip(solvers, init):
        s.set_state(u)
        nsk.nsk_autotune(s.ctx, 2)
        s.set_state(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for s in solvers:
        s.rk_step(dt, steps)
    e1.record()
    torch.cuda.synchronize()
    ms_s = e0.elapsed_time(e1)
    wall_s = (time.perf_counter() - t0) * 1e3
    for s in solvers:
        s.close()
    work = n * dofs * 5 * steps
    return {"instances": n, "mesh": "8x8x8 N=3", "dofs": n * dofs, "steps": steps,
            "value": work / (ms_b * 1e-3), "unit": "DOF-stage/s",
            "sequential_value": work / (ms_s * 1e-3), "speedup_vs_sequential": ms_s / ms_b,
            "sequential_host_ms": wall_s}


def run_closure_form(nsk, tend: float = 0.01, timing_steps: int = 20, full_mesh: bool = False,
                     train_full: bool = False):
    """Closure form, kappa = 1e-4 (interface width 2 sqrt(kappa) = 0.02).
    A network is trained here, from seeded initial weights, on nudged
    alpha = 200 / 2000 pairs of two 3D collisions on [0,1]x[0,0.5]^2 with
    48x24x24 elements, N = 4 (the element size of the full collision mesh),
    R = 0.1, to t_end.

    Accuracy: a held-out collision runs to t_end at alpha = 2000 (the reference),
    1000, 400 and 200, and at alpha = 200 with the closure (every stage, and
    once per step; FP64 and mixed-precision right-hand sides) through
    nsk_closure_run, whose fallback is the FP64 alpha = 2000 run.  By default the held-out collision is a 48x24x24 one (We = 70,
    impact 0.03); with full_mesh it is the benchmark collision itself on
    96x48x48 (We = 100), and every run's time to t_end is measured.  Errors
    of rho against the alpha = 2000 run: the quadrature-weighted L2 over
    the weighted L2 of rho_ref, and over that of rho_ref's change from the
    initial state.  Speed-ups are times to t_end against the alpha = 2000
    run; on the 48x24x24 collision they are the full mesh's measured time
    per step times each run's step count.

    train_full (with full_mesh): the training pairs come from two collisions
    on the full 96x48x48 mesh instead (R = 0.2: We = 40 head-on and We = 150
    with impact 0.1 R; the benchmark's We = 100 head-on collision stays held
    out), and the plain alpha = 1000 and 2000 runs are not repeated to t_end
    (their times to t_end come from timed steps)."""
    import numpy as np
    import torch

    from paper_1912_12059_amd import closure as CL
    from paper_1912_12059_amd import inputs as I

    kappa, N = 1e-4, 4
    small = dict(dim=3, N=N, nel=(48, 24, 24), hi=(1.0, 0.5, 0.5))
    w = WORKLOADS["3d-collision"]
    full = dict(dim=3, N=N, nel=w["nel"], lo=w["lo"], hi=w["hi"])
    norm = CL.default_norm(kappa)

    def small_ic(We, b):
        _, U = I.collision_3d(nel=small["nel"], N=N, We=We, radius=0.1, hi=small["hi"], impact=b, device="cuda:0")
        return U.reshape(-1)

    def full_ic(We, b):
        _, U = I.collision_3d(nel=w["nel"], N=N, We=We, lo=w["lo"], hi=w["hi"], impact=b, device="cuda:0")
        return U.reshape(-1)

    def progress(step, nsteps):
        print(f"[bench] closure pairs: step {step}/{nsteps}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    Xs, Ys = [], []
    pairs = ((full, full_ic, ((40.0, 0.0), (150.0, 0.02)), 200) if train_full else
             (small, small_ic, ((40.0, 0.0), (100.0, 0.05)), 100))
    for We, b in pairs[2]:
        X, Y, info = CL.nudged_pairs(pairs[0], pairs[1](We, b), 2000.0, 200.0, kappa, tend, norm,
                                     record_every=pairs[3], progress=progress)
        Xs.append(X)
        Ys.append(Y)
    X, Y = torch.cat(Xs), torch.cat(Ys)
    del Xs, Ys
    _, std = CL.moments(Y)
    norm.update(out_m=float(std[0]), out_c=float(std[1]))
    net = CL.Network(seed=0)
    net.train(X, Y, steps=3000, batch=32768, lr=2e-3, lr_final=2e-4, tscale=(1.0 / std[0], 1.0 / std[1]))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    nsamp = X.shape[0]
    del X, Y
    print(f"[bench] closure trained on {nsamp} samples in {train_s:.1f} s", file=sys.stderr, flush=True)

    # the alpha = 200 runs take their own step dt and the alpha = 2000 reference
    # M steps of dt / M per step (within its own limit dt_ref_own)
    dt_mod, M = info["dt"], info["M"]
    dt_ref = dt_mod / M
    n_mod = int(round(tend / dt_mod))
    n_ref = M * n_mod
    tend_run = n_mod * dt_mod
    if full_mesh:
        mesh = full
        _, U0 = I.collision_3d(nel=w["nel"], N=N, We=w["We"], lo=w["lo"], hi=w["hi"], device="cuda:0")
        U0 = U0.reshape(-1)
    else:
        mesh = small
        U0 = small_ic(70.0, 0.03)
    wq = np.polynomial.legendre.leggauss(N + 1)[1]
    wn = torch.from_numpy(np.einsum("i,j,k->kji", wq, wq, wq).reshape(-1)).cuda()  # node weights, i fastest
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def run(fn, s):
        torch.cuda.synchronize()
        e0.record(s.stream)
        extra = fn()
        e1.record(s.stream)
        torch.cuda.synchronize()
        return s.get_state()[0].reshape(-1, wn.numel()).clone(), e0.elapsed_time(e1), extra

    def plain(alpha, reference=False):
        """The plain run at alpha to t_end: as the reference, the alpha = 2000 run
        in the steps of the closure runs' fallback (dt / M); otherwise in the
        fewest equal steps within its own limit."""
        s = nsk.Solver(alpha=alpha, kappa=kappa, **mesh)
        s.set_state(U0)
        n = n_ref if reference else int(math.ceil(tend_run / s.dt_estimate(0.5) - 1e-9))
        dt = dt_ref if reference else tend_run / n

        def steps():
            for k in range(0, n, 2000):  # a progress line per 2000 steps
                s.rk_step(dt, min(2000, n - k))
                s.stream.synchronize()
                print(f"[bench] closure form: plain alpha={alpha:g} {min(k + 2000, n)}/{n} steps", file=sys.stderr,
                      flush=True)

        rho, ms, _ = run(steps, s)
        s.close()
        return rho, ms, n

    def with_closure(every_stage, precision=0):
        s = CL.closure_solver(net, norm, every_stage=every_stage, alpha=200.0, kappa=kappa, precision=precision,
                              **mesh)
        fb = nsk.Solver(alpha=2000.0, kappa=kappa, **mesh)
        s.set_state(U0)
        fb.set_state(U0)
        rho, ms, rep = run(lambda: nsk.nsk_closure_run(s.ctx, fb.ctx, dt_mod, n_mod, M, 200), s)
        s.close()
        fb.close()
        return rho, ms, rep

    rho0 = U0.reshape(5, -1)[0].reshape(-1, wn.numel())
    rho_ref, ms_ref, _ = plain(2000.0, reference=True)

    def wl2(a):
        return float(torch.sqrt(torch.sum(wn * a * a)))

    ref_norm, change_norm = wl2(rho_ref), wl2(rho_ref - rho0)

    def errors(rho):
        e = wl2(rho - rho_ref)
        return {"l2_rho_rel_to_ref": e / ref_norm, "l2_rho_rel_to_ref_change": e / change_norm}

    results = {}
    for alpha in (2000.0, 1000.0, 400.0, 200.0):
        if train_full and alpha in (2000.0, 1000.0):
            # time 200 steps at the run's own limit; its error is not needed
            s = nsk.Solver(alpha=alpha, kappa=kappa, stream=torch.cuda.Stream(), **mesh)
            s.set_state(U0)
            n = int(math.ceil(tend_run / s.dt_estimate(0.5) - 1e-9))
            ms200 = _timed_steps(s, tend_run / n, 200)
            s.close()
            results[f"plain_alpha{int(alpha)}"] = dict(alpha=alpha, steps=n, ms_to_tend=ms200 / 200 * n,
                                                      note="time to t_end from 200 timed steps")
            continue
        rho, ms, n = plain(alpha)
        results[f"plain_alpha{int(alpha)}"] = dict(errors(rho), alpha=alpha, steps=n, ms_to_tend=ms)
        print(f"[bench] closure form: plain alpha={alpha:g} done", file=sys.stderr, flush=True)
    # the closure with FP64 and with mixed-precision right-hand sides (the
    # alpha = 2000 fallback and reference stay FP64)
    closure_runs = ((1, 0, "closure_alpha200"), (0, 0, "closure_alpha200_once_per_step"),
                    (1, 1, "closure_alpha200_mixed"), (0, 1, "closure_alpha200_once_per_step_mixed"))
    for every_stage, precision, name in closure_runs:
        rho, ms, rep = with_closure(every_stage, precision)
        results[name] = dict(errors(rho), alpha=200.0, steps=n_mod, ms_to_tend=ms, fallback_report=rep,
                             precision="mixed" if precision else "fp64")
        print(f"[bench] closure form: {name} done (fell back: {rep['fell_back']})", file=sys.stderr, flush=True)

    # time per step on the full mesh (the speed-ups of the 48x24x24 runs)
    per_step = {}
    if not full_mesh:
        _, Uf = I.collision_3d(nel=w["nel"], N=N, We=w["We"], lo=w["lo"], hi=w["hi"], device="cuda:0")
        Uf = Uf.reshape(-1)

        def ms_per_step(s, dt):
            s.set_state(Uf)
            nsk.nsk_autotune(s.ctx, 2)
            s.rk_step(dt, 2)
            s.set_state(Uf)
            return _timed_steps(s, dt, timing_steps) / timing_steps

        for alpha in (2000.0, 1000.0, 400.0, 200.0):
            s = nsk.Solver(alpha=alpha, kappa=kappa, stream=torch.cuda.Stream(), **full)
            per_step[f"plain_alpha{int(alpha)}"] = ms_per_step(s, dt_mod if alpha == 200.0 else dt_ref)
            s.close()
        for every_stage, precision, name in closure_runs:
            s = CL.closure_solver(net, norm, every_stage=every_stage, alpha=200.0, kappa=kappa, precision=precision,
                                  stream=torch.cuda.Stream(), **full)
            per_step[name] = ms_per_step(s, dt_mod)
            if every_stage and not precision:
                s.set_state(Uf)
                nsk.nsk_timing_enable(s.ctx, 1)
                _timed_steps(s, dt_mod, timing_steps)
                ms_lift, ms_rhs, nst, ms_cls = nsk.nsk_timing_read(s.ctx)
                nsk.nsk_timing_enable(s.ctx, 0)
                per_step["closure_kernel_ms_per_stage"] = ms_cls / max(nst, 1)
            s.close()
    # the cost to beat: the plain alpha = 2000 run at its own step limit
    n2000 = results["plain_alpha2000"]["steps"]
    if not full_mesh:
        ms_ref_full = per_step["plain_alpha2000"] * n2000
    else:
        ms_ref_full = results["plain_alpha2000"]["ms_to_tend"]
    dofs_full = int(np.prod(w["nel"])) * (N + 1) ** 3
    for name, r in results.items():
        if full_mesh:
            t = r["ms_to_tend"]
        else:
            t = per_step[name] * r["steps"]
            r["ms_per_step_full_mesh"] = per_step[name]
        r["speedup_vs_alpha2000"] = ms_ref_full / t
        r["value"] = dofs_full * 5 * n2000 / (t * 1e-3)
    out = {
        "workload": (f"3d-collision {'x'.join(map(str, w['nel']))} N={N} kappa={kappa:g} t_end={tend_run:.4g}; "
                     + ("every run on the full mesh" if full_mesh else
                        "accuracy on a held-out 48x24x24 collision (same element size), speed on the full mesh")),
        "alpha": 200.0, "alpha_ref": 2000.0, "dt": dt_mod, "ratio": M, "dt_reference": dt_ref,
        "steps": n_mod, "steps_reference": n_ref,
        "reference_note": "errors are against the alpha = 2000 run in steps dt / ratio (the closure runs' fallback); "
                      "speed-ups against the plain alpha = 2000 run at its own step limit (plain_alpha2000)",
        **results,
        "value_note": "effective DOF-stage/s of the 96x48x48 mesh: DOF-stages of the plain alpha = 2000 run to "
                      "t_end / time to t_end",
        "error_note": "quadrature-weighted L2 of rho - rho_ref (alpha = 2000, same t_end) over that of rho_ref "
                      "(rel_to_ref) and of rho_ref - rho_initial (rel_to_ref_change)",
        "training": {"samples": nsamp, "seconds": train_s, "steps": 3000, "batch": 32768,
                     "pairs": ("nudged alpha=200 toward alpha=2000 (tau = 100 steps), collisions "
                               + ("R=0.2 We=40 b=0 and We=150 b=0.1R on 96x48x48" if train_full else
                                  "R=0.1 We=40 b=0 and We=100 b=0.05R on 48x24x24"))},
    }
    if per_step:
        out["closure_kernel_ms_per_stage"] = per_step.get("closure_kernel_ms_per_stage")
    return out


def _timed_steps(s, dt: float, steps: int) -> float:
    """Milliseconds of `steps` steps on the solver's stream (HIP events)."""
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.rk_step(dt, steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def dof_stage_rate(dofs: int, steps: int, seconds: float) -> float:
    """DOF-stage updates per second of `steps` five-stage steps over `dofs`
    nodes taking `seconds`."""
    return dofs * 5 * steps / seconds


def run_small_configs(nsk, with_oracle: bool = True) -> dict:
    """The 1D slab workload (64 elements, N = 3, alpha = 500: a launch-latency
    case, 256 nodes) in microseconds per step over its 2000 steps: all steps
    in one launch (the mesh fits one workgroup of the first tile variant; the
    default), and, on the second variant (two workgroups), replayed as a
    captured graph (non-null stream) and launched stage by stage; and the 2D
    droplet workload (96^2, N = 4, 230,400 nodes) rate at alpha = 500 and
    2000 over 200 steps.  The oracle is timed beside each: the full 2000 1D
    steps, 40 steps in 2D."""
    import torch

    from paper_1912_12059_amd import inputs as I

    out = {}
    m, U = I.slab_1d()
    res = {"workload": "1d-slab 64 N=3 alpha=500 beta=1e-3 eps=1e-3 kappa=1e-5, 2000 steps", "dofs": 256}
    for name, variant, stream in (("one_launch", 0, torch.cuda.Stream()), ("graph", 1, torch.cuda.Stream()),
                                  ("stagewise", 1, None)):
        s = nsk.Solver(dim=1, N=3, nel=(64,), alpha=500.0, beta=1e-3, eps=1e-3, kappa=1e-5, stream=stream)
        nsk.nsk_set_tile(s.ctx, variant, 0)
        s.set_state(U)
        dt = s.dt_estimate(0.5)
        _timed_steps(s, dt, 200)
        s.set_state(U)
        ms = _timed_steps(s, dt, 2000)
        res[f"us_per_step_{name}"] = 1e3 * ms / 2000
        res["dt"] = dt
        s.close()
    res["value"] = dof_stage_rate(256, 1, 1e-6 * res["us_per_step_one_launch"])
    res["unit"] = "DOF-stage/s"
    if with_oracle:
        O = oracle()
        P = O.Problem(dim=1, N=3, nel=(64, 1, 1), alpha=500.0, beta=1e-3, eps=1e-3, kappa=1e-5)
        t0 = time.perf_counter()
        O.run(P, U, res["dt"], 2000)
        el = time.perf_counter() - t0
        res["oracle"] = {"us_per_step": 1e6 * el / 2000, "value": dof_stage_rate(256, 2000, el),
                         "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))}
    out["1d_slab"] = res
    m, U = I.droplets_2d()
    U0 = torch.from_numpy(U.reshape(-1)).to("cuda:0")
    dofs = m.nelem * m.nnode
    for alpha in (500.0, 2000.0):
        s = nsk.Solver(dim=2, N=4, nel=(96, 96), alpha=alpha, beta=1e-3, eps=1e-3, kappa=1e-5,
                       stream=torch.cuda.Stream())
        s.set_state(U0)
        dt = s.dt_estimate(0.5)
        variant, order, _ = nsk.nsk_autotune(s.ctx, 3)
        _timed_steps(s, dt, 20)
        s.set_state(U0)
        ms = _timed_steps(s, dt, 200)
        r = {"workload": f"2d-droplets 96x96 N=4 alpha={alpha:g} beta=1e-3 eps=1e-3 kappa=1e-5", "dofs": dofs,
             "value": dof_stage_rate(dofs, 200, ms * 1e-3), "unit": "DOF-stage/s", "ms_per_step": ms / 200, "dt": dt,
             "tile": {"variant": variant, "order": order}}
        s.close()
        if with_oracle:
            O = oracle()
            P = O.Problem(dim=2, N=4, nel=(96, 96, 1), alpha=alpha, beta=1e-3, eps=1e-3, kappa=1e-5)
            t0 = time.perf_counter()
            O.run(P, U, dt, 40)
            el = time.perf_counter() - t0
            r["oracle"] = {"value": dof_stage_rate(dofs, 40, el), "steps": 40,
                           "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))}
        out[f"2d_droplets_alpha{int(alpha)}"] = r
    return out


def _long_run(nsk, s, U0, steps: int, chunk: int) -> dict:
    """Steps in chunks with diagnostics after each, stopping at the first
    non-physical state; returns how far the run got and its rate."""
    s.set_state(U0)
    dt = s.dt_estimate(0.5)
    done, ms = 0, 0.0
    while done < steps:
        k = min(chunk, steps - done)
        ms += _timed_steps(s, dt, k)
        done += k
        d = s.diagnostics()
        if d["status"] != 0:
            return {"finite_steps": done - k, "nonphysical_by_step": done, "t_finite": (done - k) * dt, "dt": dt}
    return {"finite_steps": done, "t_finite": done * dt, "dt": dt, "ms_per_step": ms / done,
            "rho_range": [d["rho_min"], d["rho_max"]], "e_kin": d["e_kin"]}


def run_long_runs(nsk, U0_3d) -> dict:
    """Run lengths the workloads reach.  2D droplets (96^2, N = 4): the
    stated 20k steps at alpha = 500 and 2000 as configured (kappa = 1e-5, no
    shock capturing), with FV sub-cells at kappa = 1e-5 (indicator threshold
    -9) and with kappa = 1e-4 (the equilibrium interface width 2 sqrt(kappa)
    equal to the initial 0.02).  3D collision (96x48x48, N = 4, kappa =
    1e-5): FP64 and mixed over 2000 steps, and the relative L2 of rho between
    them at the end.  Diagnostics every 1000 (2D) or 500 (3D) steps; a run
    stops at its first non-physical state."""
    import torch

    from paper_1912_12059_amd import inputs as I

    out = {}
    m, U = I.droplets_2d()
    U0 = torch.from_numpy(U.reshape(-1)).to("cuda:0")
    for label, kappa, sc in (("kappa1e-5", 1e-5, None), ("kappa1e-5_subcells", 1e-5, -9.0),
                             ("kappa1e-4", 1e-4, None)):
        for alpha in (500.0, 2000.0):
            kw = {} if sc is None else dict(subcell=1, subcell_threshold=sc)
            s = nsk.Solver(dim=2, N=4, nel=(96, 96), alpha=alpha, beta=1e-3, eps=1e-3, kappa=kappa,
                           stream=torch.cuda.Stream(), **kw)
            r = _long_run(nsk, s, U0, 20000, 1000)
            s.close()
            if "ms_per_step" in r:
                r["value"] = m.nelem * m.nnode * 5 / (r["ms_per_step"] * 1e-3)
            out[f"2d_droplets_{label}_alpha{int(alpha)}"] = r
            print(f"[bench] long run 2D {label} alpha={alpha:g}: {r['finite_steps']} finite steps", file=sys.stderr,
                  flush=True)
    del U0
    fin = {}
    for prec in (0, 1):
        s = nsk.Solver(dim=3, N=4, nel=(96, 48, 48), lo=(0, 0, 0), hi=(2, 1, 1), alpha=1000.0, beta=1e-3, eps=1e-3,
                       kappa=1e-5, precision=prec, stream=torch.cuda.Stream())
        r = _long_run(nsk, s, U0_3d, 2000, 500)
        if r["finite_steps"] == 2000:
            fin[prec] = s.get_state()[0].reshape(-1).clone()
        s.close()
        out[f"3d_collision_{'fp64' if prec == 0 else 'mixed'}"] = r
        print(f"[bench] long run 3D precision={prec}: {r['finite_steps']} finite steps", file=sys.stderr, flush=True)
    if len(fin) == 2:
        out["3d_collision_mixed_vs_fp64_l2_rel_rho"] = float(
            torch.linalg.vector_norm(fin[1] - fin[0]) / torch.linalg.vector_norm(fin[0]))
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="3d-collision", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="form reported as value; the other one is measured beside it unless --no-forms")
    ap.add_argument("--no-forms", action="store_true", help="skip the second precision form and the batch")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched collision sweep")
    ap.add_argument("--no-implicit", action="store_true", help="skip the implicit ESDIRK form")
    ap.add_argument("--no-closure", action="store_true", help="skip the closure form")
    ap.add_argument("--only-closure", action="store_true", help="run only the closure form (prints its block)")
    ap.add_argument("--closure-full-mesh", action="store_true",
                    help="with --only-closure: run every accuracy run of the closure form on the full mesh")
    ap.add_argument("--closure-tend", type=float, default=0.01, help="t_end of the closure form")
    ap.add_argument("--closure-kernel-steps", type=int, default=0, metavar="K",
                    help="only K closure steps (every stage) on the full collision with a seeded untrained network "
                         "(profiling the closure kernel)")
    ap.add_argument("--closure-train-full", action="store_true",
                    help="with --closure-full-mesh: train on two full-mesh collisions (the benchmark's held out)")
    ap.add_argument("--only-implicit", action="store_true",
                    help="run only one implicit step of 100x the explicit step, no explicit reference (profiling)")
    ap.add_argument("--only-subcell", type=float, default=None, metavar="THRESHOLD",
                    help="run only the FV sub-cell form at this indicator threshold (profiling)")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched collision sweep and the 64 small collisions (prints their blocks)")
    ap.add_argument("--only-nsk", action="store_true",
                    help="run only the original NSK form on the workload (prints its block)")
    ap.add_argument("--no-long-runs", action="store_true", help="skip the run-length form")
    ap.add_argument("--only-long-runs", action="store_true", help="run only the run-length form")
    ap.add_argument("--only-small-configs", action="store_true",
                    help="run only the 1D latency and 2D rate form (with the oracle beside them)")
    ap.add_argument("--cpu-one-thread", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", default="auto", help="auto (autotuner) or 'variant,order', e.g. 0,4")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of MIB MiB (to scale HBM byte counters)")
    args = ap.parse_args()
    if args.cpu_one_thread:
        return cpu_one_thread_child(args.cpu_one_thread)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (sharding across GPUs is designed, not implemented)", file=sys.stderr)
        return 2
    if args.copy_calibration:
        import torch

        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 8, "copies": 4}))
        return 0

    import torch

    from paper_1912_12059_amd import nsk

    if args.closure_kernel_steps:
        from paper_1912_12059_amd import closure as CL

        w = WORKLOADS["3d-collision"]
        m, U = build_state("3d-collision")
        net = CL.Network(seed=0)
        norm = dict(CL.default_norm(1e-4), out_m=1e-3, out_c=1e-3)  # small outputs keep the state physical
        s = CL.closure_solver(net, norm, alpha=200.0, kappa=1e-4, dim=3, N=w["N"], nel=w["nel"], lo=w["lo"],
                              hi=w["hi"])
        s.set_state(U)
        dt = s.dt_estimate(0.5)
        ms = _timed_steps(s, dt, args.closure_kernel_steps)
        s.close()
        print(json.dumps({"closure_kernel_steps": args.closure_kernel_steps, "ms_per_step": ms / args.closure_kernel_steps}))
        return 0
    if args.only_closure:
        print(json.dumps({"closure": run_closure_form(nsk, tend=args.closure_tend,
                                                      full_mesh=args.closure_full_mesh or args.closure_train_full,
                                                      train_full=args.closure_train_full)}))
        return 0
    if args.only_batched:
        print(json.dumps({"batched": run_batched(nsk, 200, 2), "batched_small": run_batched_small(nsk)}))
        return 0
    if args.only_small_configs:
        print(json.dumps({"configs_small": run_small_configs(nsk, not args.no_cpu_baseline)}))
        return 0
    w = WORKLOADS[args.workload]
    print(f"[bench] building {args.workload} state", file=sys.stderr, flush=True)
    m, U = build_state(args.workload)
    U0 = torch.from_numpy(U.reshape(-1)).to("cuda:0")
    if args.only_subcell is not None:
        del U
        r = run_form(nsk, m, U0, w, 0, args.steps, args.warmup, args.tile, subcell_threshold=args.only_subcell)
        dofs = m.nelem * m.nnode
        print(json.dumps({"subcell": {"threshold": args.only_subcell, "troubled_fraction": r["troubled"],
                                      "value": dofs * 5 * args.steps / (r["ms"] * 1e-3),
                                      "ms_per_step": r["ms"] / args.steps, "lift_ms": r["ms_lift"],
                                      "indicator_and_means_ms": r["ms_mid"], "dg_rhs_plus_fv_ms": r["ms_rhs"]}}))
        return 0
    if args.only_implicit:
        del U
        print(json.dumps({"implicit_esdirk": run_implicit_form(nsk, m, U0, w, (100,), reference=False)}))
        return 0
    if args.only_long_runs:
        del U
        print(json.dumps({"long_runs": run_long_runs(nsk, U0)}))
        return 0
    if args.only_nsk:
        del U
        s2 = nsk.Solver(dim=m.dim, N=m.N, nel=tuple(m.nel), lo=tuple(m.lo), hi=tuple(m.hi), alpha=w["alpha"],
                        beta=1e-3, eps=1e-3, kappa=1e-5)
        s2.set_state(U0)
        ref = {"dt": s2.dt_estimate(0.5), "ms": float("nan")}
        s2.close()
        print(json.dumps({"nsk_original_fp64": run_nsk_form(nsk, m, U0, w, args.steps, args.warmup, args.tile,
                                                            ref)}))
        return 0
    if m.dim == 3:
        sub = (16, 16, 16)
        block = ((24, 16), (16, 16), (16, 16))  # around the first droplet's interface
    else:
        sub = (32, 32)
        block = ((16, 32), (32, 32))
    sample = None if args.no_cpu_baseline else sample_block(U, m.nel, block)
    del U
    dofs = m.nelem * m.nnode
    main_prec = 1 if args.precision == "mixed" else 0
    forms = {}
    order = [main_prec] if args.no_forms else [main_prec, 1 - main_prec]
    for prec in order:
        forms[prec] = run_form(nsk, m, U0, w, prec, args.steps, args.warmup, args.tile)
    r = forms[main_prec]
    mixed = main_prec == 1
    rate = dofs * 5 * args.steps / (r["ms"] * 1e-3)
    bp_first = bytes_per_node(m.dim, True, mixed)
    bp = bytes_per_node(m.dim, False, mixed)
    # average algorithmic bytes per launch of the rhs kernel over the 5 stages
    rhs_bytes = dofs * (bp_first["rhs"] + 4 * bp["rhs"]) / 5.0
    lift_bytes = dofs * bp["lift"]
    achieved = rhs_bytes / (r["ms_rhs"] * 1e-3) / 1e9
    diag = r["diag"]
    tr = counter_traffic(args.workload, args.precision, (r["variant"], r["order"]))
    out = {
        "metric": METRIC,
        "value": rate,
        "unit": "DOF-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if not mixed else "f64-state/f32-flux",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload} {'x'.join(map(str, m.nel))} N={m.N} alpha={w['alpha']:g} beta=1e-3 "
                        f"eps=1e-3 kappa=1e-5" + (f" We={w['We']:g}" if "We" in w else ""),
            "dofs": dofs,
            "nvar": m.nvar,
            "precision": args.precision,
            "dt": r["dt"],
            "tile": {"variant": r["variant"], "order": r["order"], "autotune_ms": r["tune_ms"]},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "rhs_kernel (volume+surface+source+RK stage)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": tr["bytes"] if tr else None,
            "traffic_over_algorithmic": tr["bytes"] / rhs_bytes if tr else None,
            "traffic_source": tr["source"] if tr else None,
            "avg_ms": r["ms_rhs"],
            "bytes_per_launch": rhs_bytes,
            "lift_avg_ms": r["ms_lift"],
            "lift_achieved_GBs": lift_bytes / (r["ms_lift"] * 1e-3) / 1e9 if r["ms_lift"] > 0 else None,
            "stage_bytes_per_node": (bp["lift"] + bp["rhs"]),
            "stage_GBs": dofs * (bp["lift"] + bp["rhs"]) / ((r["ms_rhs"] + r["ms_lift"]) * 1e-3) / 1e9,
        },
        "diag_after": {"mass_rho": diag["mass"][0], "e_total": diag["e_total"], "status": diag["status"]},
        "wall_s": r["wall"],
    }
    if len(forms) == 2:
        f64, mx = forms[0], forms[1]
        rho64 = f64["final"][0].reshape(-1)
        rhom = mx["final"][0].reshape(-1)
        l2 = float(torch.linalg.vector_norm(rhom - rho64) / torch.linalg.vector_norm(rho64))
        out["forms"] = {
            "fp64": {"value": dofs * 5 * args.steps / (f64["ms"] * 1e-3), "ms_per_step": f64["ms"] / args.steps,
                     "rhs_ms": f64["ms_rhs"], "lift_ms": f64["ms_lift"]},
            "mixed": {"value": dofs * 5 * args.steps / (mx["ms"] * 1e-3), "ms_per_step": mx["ms"] / args.steps,
                      "rhs_ms": mx["ms_rhs"], "lift_ms": mx["ms_lift"],
                      "speedup_vs_fp64": f64["ms"] / mx["ms"],
                      "l2_rel_rho_vs_fp64": l2,
                      "l2_note": f"relative L2 of rho, mixed vs FP64 GPU run, same initial state and dt, "
                                 f"after {args.steps} steps"},
        }
    if len(forms) == 2:
        # the HLLC flux (FP64) on the same workload
        hl = run_form(nsk, m, U0, w, 0, args.steps, args.warmup, args.tile, flux=1)
        rh = f64["final"][0].reshape(-1)
        out["forms"]["hllc_fp64"] = {
            "value": dofs * 5 * args.steps / (hl["ms"] * 1e-3), "ms_per_step": hl["ms"] / args.steps,
            "rhs_ms": hl["ms_rhs"], "lift_ms": hl["ms_lift"],
            "roofline_frac": dofs * (bytes_per_node(m.dim, True, False)["rhs"]
                                     + 4 * bytes_per_node(m.dim, False, False)["rhs"]) / 5.0
                             / (hl["ms_rhs"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "l2_rel_rho_vs_rusanov": float(torch.linalg.vector_norm(hl["final"][0].reshape(-1) - rh)
                                           / torch.linalg.vector_norm(rh)),
            "tile": {"variant": hl["variant"], "order": hl["order"]},
        }
        del hl
        out["forms"]["nsk_original_fp64"] = run_nsk_form(nsk, m, U0, w, args.steps, args.warmup, args.tile, f64)
        if not args.no_implicit:
            out["forms"]["implicit_esdirk"] = run_implicit_form(nsk, m, U0, w)
        out["forms"]["subcell_fp64"] = run_subcell_form(nsk, m, U0, w, dict(f64, steps=args.steps))
    del forms
    if not args.no_forms and not args.no_batched and args.workload == "3d-collision":
        out.setdefault("forms", {})["batched"] = run_batched(nsk, 200, 2)
        out["forms"]["batched_small"] = run_batched_small(nsk)
    if not args.no_forms and not args.no_closure and args.workload == "3d-collision":
        out.setdefault("forms", {})["closure"] = run_closure_form(nsk)
    if not args.no_forms and args.workload == "3d-collision":
        out.setdefault("forms", {})["configs_small"] = run_small_configs(nsk, not args.no_cpu_baseline)
        if not args.no_long_runs:
            out["forms"]["long_runs"] = run_long_runs(nsk, U0)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, sample, sub)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
