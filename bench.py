#!/usr/bin/env python3
"""Throughput benchmark: one Hermite step of a 2^20-body Plummer sphere with
every particle active, on one MI355X.

A step is one pass of the hot path with every particle due (a shared step
of 2^-10, so the block is all N particles in order and needs no selection
pass): the O(N^2) pairwise acceleration/jerk/potential kernel, then the
float64 corrector fused with the float64 prediction of every particle to
the next step and its packing into the device layout.  The block-step form
(integer selection, plan, split) is timed in the block_steps section.
Inputs are resident in HBM before the timed region.

Prints ONE JSON line (rank 0, N = 1):
  value     whole-job interactions per second (Ginteractions/s), N^2 per step
  roofline  the pairwise kernel against the FP32 vector peak, from HIP events
            recorded around each kernel launch on its stream
  cpu_baseline  the float64 oracle on a bounded i-subset on the host's cores
  accuracy  per-particle relative errors of both precisions on that subset
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_INTERACTION = 60          # acc + jerk + potential convention (Eq. 3, k = 60)
FP32_PEAK_TFLOPS = 157.3            # MI355X FP32 vector peak (256 CU x 64 x 2 x 2 x 2.4 GHz)
PAPER_GINT_S = 1.0995116e12 / 279.4067 / 1e9   # 8800GTX, N = 2^20, Table 4 (context)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_ds_plummer1m_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "force_plummer1m_valu_clock.txt")
# the headline kernel: its tile loop, its instantiations and the rules that
# pick its launch shape and j-split
KERNEL_SRCS = [os.path.join(ROOT, "paper_0707_0438_amd", "csrc", f)
               for f in ("force_block.h", "force.hip", "launch_shape.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha256() -> str:
    """One sha256 over the pairwise kernels and the launch-shape rules they run
    under; counter summaries record it and are used only while it matches."""
    h = hashlib.sha256()
    for src in KERNEL_SRCS:
        h.update(open(src, "rb").read())
    return h.hexdigest()


def profile_keys(path):
    """The `key: value` lines of a committed counter summary, or None when the
    file is missing or was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    kv = {}
    for ln in open(path):
        if ":" in ln:
            k, v = ln.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_sha256():
        return None
    return kv


def traffic_per_launch(prec: str):
    """HBM bytes per launch of the pairwise kernel from the committed rocprofv3
    counter summary, or None when it is missing or the kernel source or the
    launch-shape rules changed since the counters were taken."""
    kv = profile_keys(TRAFFIC_FILE) if prec == "ds" else None
    try:
        return float(kv["traffic_bytes_per_launch"]) if kv else None
    except (KeyError, ValueError):
        return None


def executed_flops(prec: str, gint_s: float):
    """Executed FP32 flop rate of the pairwise kernel: the flop per interaction
    the VALU counters measured (ADD + MUL + TRANS + 2 FMA instructions x 64
    lanes, per interaction; committed summary, used only while the kernel
    sources match) times the measured interaction rate.  None otherwise."""
    kv = profile_keys(VALU_FILE)
    key = ("ds" if prec == "ds" else "fp32") + "_executed_flop_per_interaction"
    try:
        f = float(kv[key]) if kv else None
    except (KeyError, ValueError):
        f = None
    if f is None:
        return None
    tf = f * gint_s / 1e3
    return {"flop_per_interaction": f, "TFLOP_s": round(tf, 2),
            "pct_fp32_peak": round(100.0 * tf / FP32_PEAK_TFLOPS, 2),
            "source": os.path.relpath(VALU_FILE, ROOT)}


def device_clock_ghz():
    """Peak engine clock the HIP runtime reports for device 0 (GHz), or None."""
    import ctypes
    import paper_0707_0438_amd as nb
    try:
        hip = ctypes.CDLL(nb.LIB_PATH)   # resolves the runtime libnbody links
        khz = ctypes.c_int(0)
        # hipDeviceAttributeClockRate (5): peak clock in kHz
        if hip.hipDeviceGetAttribute(ctypes.byref(khz), 5, 0) != 0 or khz.value <= 0:
            return None
        return khz.value / 1e6
    except (OSError, AttributeError):
        return None


def device_info():
    """What the runtime reports about the GPU, and how the FP32 peak used for
    the roofline is derived (the published 157.3 TFLOP/s is the one used)."""
    import torch
    pr = torch.cuda.get_device_properties(0)
    cu = pr.multi_processor_count
    ghz = device_clock_ghz()
    info = {"name": pr.name, "arch": getattr(pr, "gcnArchName", ""), "compute_units": cu,
            "memory_GiB": round(pr.total_memory / 2 ** 30, 1),
            "fp32_peak": f"{cu} CU x 64 lanes x 2 (packed FP32 rate) x 2 (FMA) x 2.4 GHz "
                         f"= {cu * 64 * 2 * 2 * 2.4e9 / 1e12:.1f} TFLOP/s"}
    if ghz:
        info["reported_peak_clock_GHz"] = round(ghz, 3)
        info["fp32_peak_at_reported_clock_TFLOP_s"] = round(cu * 64 * 2 * 2 * ghz * 1e9 / 1e12, 1)
    return info


def time_steps(ctx, h, steps, warmup):
    import torch
    for _ in range(warmup):
        h.step()
    torch.cuda.synchronize()
    ctx.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_active = 0
    for _ in range(steps):
        na, _ = h.step()
        total_active += na
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, launches = ctx.kernel_time()
    ctx.kernel_timing(False)
    return t1 - t0, total_active, kms, launches


def cpu_baseline(p, eps, budget_s):
    """Time the float64 oracle on the first k particles against all n.
    Returns the baseline record and the oracle's rows (for the accuracy
    report)."""
    import numpy as np
    import oracle
    n = p.n
    # a short call first (thread start-up, page-in), then 1024 timed rows
    oracle.force(p.pos[:, :64], p.vel[:, :64], p.pos, p.vel, p.mass, eps, iself=np.arange(64))
    t0 = time.perf_counter()
    oracle.force(p.pos[:, :1024], p.vel[:, :1024], p.pos, p.vel, p.mass, eps, iself=np.arange(1024))
    t1024 = time.perf_counter() - t0
    # rows sized to fill about budget_s of host work (at least the 4096-row subset)
    k = int(max(4096, min(n, budget_s / max(t1024, 1e-6) * 1024)))
    sel = np.arange(k)
    t0 = time.perf_counter()
    ref = oracle.force(p.pos[:, sel], p.vel[:, sel], p.pos, p.vel, p.mass, eps, iself=sel)
    dt = time.perf_counter() - t0
    return {"value": round(k * n / dt / 1e9, 6), "unit": "Ginteractions/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"float64 oracle force (acc+jerk+pot) of the first {k} particles against "
                      f"all {n} (eps={eps}), {dt:.1f} s"}, ref, k


def rel_error_stats(got, ref):
    """Per-particle relative errors |g - r| / |r| of acceleration, jerk (3-vectors,
    rows [3, k]) and potential: p99 (nearest rank) and maximum."""
    import numpy as np

    def stats(e):
        e = np.sort(e)
        return {"p99": float(f"{e[int(np.ceil(0.99 * e.size)) - 1]:.3e}"), "max": float(f"{e[-1]:.3e}")}

    out = {}
    for name, g, r in zip(("acc", "jerk"), got[:2], ref[:2]):
        out[name] = stats(np.linalg.norm(g - r, axis=0) / np.linalg.norm(r, axis=0))
    out["pot"] = stats(np.abs(got[2] - ref[2]) / np.abs(ref[2]))
    return out


def accuracy(ctx, X, V, M, eps, ref, k):
    """Both precisions of the N = n evaluation on the oracle's k rows."""
    import torch
    S = torch.arange(X.shape[1], dtype=torch.int32, device="cuda")
    out = {"sample": f"the first {k} particles against the float64 oracle (the cpu_baseline rows); "
                     "per-particle |d|/|ref|, p99 by nearest rank"}
    for prec in ("ds", "fp32"):
        a, j, pt = ctx.force(X, V, X, V, M, eps, prec=prec, i_self=S)
        torch.cuda.synchronize()
        got = (a[:, :k].cpu().numpy(), j[:, :k].cpu().numpy(), pt[:k].cpu().numpy())
        out["ds_comp" if prec == "ds" else "fp32"] = rel_error_stats(got, ref)
    return out


def adjoint_timing(nb, ctx, prec, reps=10):
    """Adjoint/forward times at the differentiation workload (N = 16384,
    eps = 1e-3): one force evaluation against the fused adjoint pass, and a
    64-step shared Hermite run (dt = 1/128, checkpoints every 8) against its
    checkpointed backward."""
    import numpy as np
    import torch
    import nbody_inputs as ics
    p = ics.workload("plummer16k_adjoint")
    eps, dt, steps = 1e-3, 1.0 / 128, 64
    X = torch.from_numpy(p.pos).to("cuda")
    V = torch.from_numpy(p.vel).to("cuda")
    M = torch.from_numpy(p.mass).to("cuda")
    g = np.random.default_rng(1)
    ga = torch.from_numpy(g.normal(size=(3, p.n))).to("cuda")
    gj = torch.from_numpy(g.normal(size=(3, p.n))).to("cuda")
    gp = torch.from_numpy(g.normal(size=p.n)).to("cuda")
    S = torch.arange(p.n, dtype=torch.int32, device="cuda")

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    t_f = timed(lambda: ctx.force(X, V, X, V, M, eps, prec=prec, i_self=S), reps)
    t_b = timed(lambda: ctx.force_vjp_self(X, V, M, eps, ga, gj, gp, prec=prec), reps)
    w = torch.from_numpy(ics.rng(ics.seed_for(3), 9).normal(size=(3, p.n))).to("cuda")
    state = {}

    def fwd():
        state["ck"] = ctx.shared_run(X, V, M, eps, dt, steps, prec=prec, ckpt_every=8)[2]

    t_run = timed(fwd, 2)
    t_adj = timed(lambda: ctx.shared_adjoint(X, V, M, eps, dt, steps, state["ck"], w, prec=prec,
                                             ckpt_every=8), 2)
    return {"workload": "plummer16k_adjoint: N=16384, eps=1e-3; 64 shared Hermite steps of 1/128, "
                        "checkpoints every 8",
            "force_ms": round(t_f, 3), "vjp_ms": round(t_b, 3),
            "adjoint_over_forward": round(t_b / t_f, 3),
            "run_ms": round(t_run, 2), "run_backward_ms": round(t_adj, 2),
            "backward_over_forward": round(t_adj / t_run, 3)}


def batched_timing(ctx, prec, steps=32, graph=True):
    """512 independent Plummer clusters (N_c log-uniform in [64, 8192],
    eps_c = 1/(4 N_c^(1/3))), 32 shared Hermite steps of 1/256: one captured
    hipGraph against the same steps launched eagerly and against one
    shared-step run per cluster.  The launch shape is picked by the batched
    autotuner first."""
    import numpy as np
    import torch
    import nbody_inputs as ics
    off, eps, p = ics.clusters(512, ics.seed_for(4))
    n = p.n
    sizes = np.diff(off)
    inter_step = float((sizes.astype(np.float64) ** 2).sum())
    X = torch.from_numpy(p.pos).to("cuda")
    V = torch.from_numpy(p.vel).to("cuda")
    M = torch.from_numpy(p.mass).to("cuda")
    O = torch.from_numpy(off).to("cuda")
    E = torch.from_numpy(eps).to("cuda")
    tile, tile_ms = ctx.autotune_batched(X, V, M, O, E, prec=prec, reps=3)
    a0, j0, _ = ctx.force_batched(X, V, M, O, E, prec=prec)
    dt = 1.0 / 256

    def run(mode):
        x, v, a, j = X.clone(), V.clone(), a0.clone(), j0.clone()
        ctx.batch_hermite(x, v, a, j, M, O, E, dt, steps, prec=prec, use_graph=(mode == "graph"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.batch_hermite(x, v, a, j, M, O, E, dt, steps, prec=prec, use_graph=(mode == "graph"))
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    t_graph = run("graph") if graph else float("nan")
    t_eager = run("eager")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(len(sizes)):
        lo, hi = int(off[c]), int(off[c + 1])
        ctx.shared_run(X[:, lo:hi].contiguous(), V[:, lo:hi].contiguous(), M[lo:hi].contiguous(),
                       float(eps[c]), dt, steps, prec=prec, checkpoints=False)
    torch.cuda.synchronize()
    t_per = time.perf_counter() - t0
    tot = inter_step * steps
    return {"workload": "clusters512_batched: 512 Plummer clusters, N_c log-uniform in [64, 8192] "
                        f"(total {n} particles, sum N_c^2 = {inter_step:.4g}), eps_c = 1/(4 N_c^(1/3)); "
                        "32 shared Hermite steps of 1/256",
            "tile": tile, "autotuned_force_ms": round(tile_ms, 3),
            "graph_ms": round(t_graph * 1e3, 2) if graph else None, "eager_ms": round(t_eager * 1e3, 2),
            "per_cluster_ms": round(t_per * 1e3, 2),
            "graph_Gint_s": round(tot / t_graph / 1e9, 1) if graph else None,
            "eager_Gint_s": round(tot / t_eager / 1e9, 1),
            "per_cluster_Gint_s": round(tot / t_per / 1e9, 1)}


def batched_probe(prec, steps=2):
    """The batched workload without the autotuner, the per-cluster runs or a
    graph: one force evaluation of the 512 clusters and `steps` eagerly
    launched shared Hermite steps in the default launch shape (a short run
    for profiler counter passes)."""
    import numpy as np
    import torch
    import nbody_inputs as ics
    import paper_0707_0438_amd as nb
    off, eps, p = ics.clusters(512, ics.seed_for(4))
    X, V, M = (torch.from_numpy(a).to("cuda") for a in (p.pos, p.vel, p.mass))
    O, E = torch.from_numpy(off).to("cuda"), torch.from_numpy(eps).to("cuda")
    ctx = nb.Context(0)
    try:
        a, j, _ = ctx.force_batched(X, V, M, O, E, prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.batch_hermite(X, V, a, j, M, O, E, 1.0 / 256, steps, prec=prec, use_graph=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        ctx.close()
    inter = float((np.diff(off).astype(np.float64) ** 2).sum()) * steps
    return {"workload": "clusters512_batched (default shape, eager launches)", "prec": prec, "steps": steps,
            "wall_s": round(wall, 4), "Gint_s": round(inter / wall / 1e9, 1)}


def kinds_timing(ctx, X, V, M, eps, prec, full_kernel_ms, reps=2):
    """The force-only (acceleration + potential, 38 conventional flops per
    interaction) and nearest-neighbour evaluations on the same N = 2^20
    system, timed per launch with HIP events on the launch stream."""
    import torch
    n = X.shape[1]
    S = torch.arange(n, dtype=torch.int32, device="cuda")
    out = {}
    for name, fn in (("force_only", lambda: ctx.force_acc(X, X, M, eps, prec=prec, i_self=S)),
                     ("nearest_neighbour", lambda: ctx.force_nn(X, V, X, V, M, eps, prec=prec, i_self=S))):
        fn()
        torch.cuda.synchronize()
        ctx.kernel_timing(True)
        for _ in range(reps):
            fn()
        ms, launches = ctx.kernel_time()
        ctx.kernel_timing(False)
        ms /= max(launches, 1)
        gint = float(n) * n / (ms * 1e-3) / 1e9
        k = 38 if name == "force_only" else FLOPS_PER_INTERACTION
        out[name] = {"kernel_ms": round(ms, 3), "Gint_s": round(gint, 1),
                     "conventional_TFLOPs": round(k * gint / 1e3, 2), "flops_per_interaction": k,
                     "pct_fp32_peak": round(100.0 * k * gint / 1e3 / FP32_PEAK_TFLOPS, 2),
                     "time_vs_full_kernel": round(ms / full_kernel_ms, 3)}
    out["workload"] = f"plummer1m_force (N={n}, eps={eps}), all particles, {reps} launches each"
    return out


def shard_timing(ctx, X, V, M, eps, prec, full_kernel_ms, shards=8, reps=3):
    """One GPU's share of an i-parallel evaluation over `shards` GPUs: the
    first N/shards particles of the N = 2^20 system as i against all N as j
    (self excluded by index), the shape each GPU would run.  Timed per
    launch with HIP events on the launch stream."""
    import torch
    n = X.shape[1]
    ni = n // shards
    xi, vi = X[:, :ni].contiguous(), V[:, :ni].contiguous()
    S = torch.arange(ni, dtype=torch.int32, device="cuda")
    fn = lambda: ctx.force(xi, vi, X, V, M, eps, prec=prec, i_self=S)
    fn()
    torch.cuda.synchronize()
    ctx.kernel_timing(True)
    for _ in range(reps):
        fn()
    ms, launches = ctx.kernel_time()
    ctx.kernel_timing(False)
    ms /= max(launches, 1)
    gint = float(ni) * n / (ms * 1e-3) / 1e9
    return {"workload": f"plummer1m_force i-slice: the first {ni} of N={n} particles (eps={eps}) against all {n}, "
                        f"one GPU's share of a {shards}-GPU i-parallel evaluation, {reps} launches",
            "tile": ctx.get_tile(ni, n, prec), "kernel_ms": round(ms, 3), "Gint_s": round(gint, 1),
            "pct_fp32_peak": round(100.0 * FLOPS_PER_INTERACTION * gint / 1e3 / FP32_PEAK_TFLOPS, 2),
            "time_vs_full_kernel": round(ms / full_kernel_ms, 4)}


def shared1k_timing(ctx, reps=5):
    """The N = 1024 shared-step workload (equal-mass Plummer, eps = 1/256,
    dt = 1/256 to t = 1/8, 32 steps): wall time per step (best of reps, state
    reset each time) in both precisions, and the largest position difference
    from the float64 oracle's run at the end."""
    import numpy as np
    import torch
    import nbody_inputs as ics
    import oracle
    p = ics.workload("plummer1k_hermite")
    X, V, M = (torch.from_numpy(a).to("cuda") for a in (p.pos, p.vel, p.mass))
    ref = oracle.HermiteState(p.pos, p.vel, p.mass)
    t0 = time.perf_counter()
    oracle.hermite_run(ref, (1 << 20) // 8, eps=1.0 / 256, shared_log2=-8, init=True)
    t_oracle = time.perf_counter() - t0
    out = {"workload": "plummer1k_hermite: N=1024 equal-mass Plummer, eps=1/256, 32 shared Hermite steps of 1/256",
           "oracle_s": round(t_oracle, 4), "oracle_cores": oracle.num_threads()}
    for prec in ("ds", "fp32"):
        h = ctx.hermite(p.n, eps=1.0 / 256, shared_dt_log2=-8, prec=prec)
        best = 1e30
        for _ in range(reps):
            h.set_state(X, V, M)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = h.advance((1 << 20) // 8)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        x = h.get_state()["x"].cpu().numpy()
        out[prec] = {"us_per_step": round(best / st["steps"] * 1e6, 2), "steps": st["steps"],
                     "max_abs_dx_vs_oracle": float(np.abs(x - ref.x).max())}
        h.close()
    return out


def block_run(n, t_end, precs, report_every=0.0, ctx=None, marks_out=True):
    """Hermite block steps on the Salpeter workload (Plummer positions and
    velocities, Salpeter masses 0.1-100 normalised to 1, eps = 1e-3,
    Aarseth eta = 0.02, levels 2^-3 .. 2^-20) from t = 0 to t_end in the
    given precisions; returns the result dict."""
    import torch
    import nbody_inputs as ics
    import paper_0707_0438_amd as nb
    p = ics.plummer(n, ics.seed_for(1), "salpeter")
    X = torch.from_numpy(p.pos).to("cuda")
    V = torch.from_numpy(p.vel).to("cuda")
    M = torch.from_numpy(p.mass).to("cuda")
    own = ctx is None
    if own:
        ctx = nb.Context(0)
    T = int(round(t_end * (1 << 20)))
    out = {"workload": f"salpeter_block: N={n} Plummer, Salpeter masses [0.1, 100] (sum 1), eps=1e-3, "
                       f"eta=0.02, block levels 2^-3..2^-20, t = 0 -> {t_end}",
           "runs": {}}
    for prec in precs:
        h = ctx.hermite(n, eps=1e-3, eta=0.02, eta_start=0.01, dt_min_log2=-20, dt_max_log2=-3, prec=prec)
        h.set_state(X, V, M)
        ek0, ep0 = h.energy()
        e0 = ek0 + ep0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        chunk = max(1, int(round((report_every or t_end) * (1 << 20))))
        target = 0
        marks = []
        diag = 0.0   # wall time spent in energy diagnostics, not counted
        while target < T:
            target = min(T, target + chunk)
            st = h.advance(target)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0 - diag
            mark = {"t": st["t_ticks"] / (1 << 20), "steps": st["steps"], "sum_active": st["sum_active"],
                    "wall_s": round(el, 3)}
            if report_every and target < T:
                d0 = time.perf_counter()
                ekm, epm = h.energy()
                mark["dE_over_E"] = (ekm + epm - e0) / e0
                diag += time.perf_counter() - d0
            marks.append(mark)
            log(f"[block] {prec} t={st['t_ticks'] / (1 << 20):.5f} steps={st['steps']} "
                f"sum_active={st['sum_active']} wall={el:.1f}s")
        wall = time.perf_counter() - t0 - diag
        ek, ep = h.energy()
        e1 = ek + ep
        if marks:
            marks[-1]["dE_over_E"] = (e1 - e0) / e0
        inter = float(st["sum_active"]) * n
        out["runs"][prec] = {
            "wall_s": round(wall, 3), "block_steps": st["steps"], "sum_active": st["sum_active"],
            "mean_active": round(st["sum_active"] / max(st["steps"], 1), 2),
            "Gint_s": round(inter / wall / 1e9, 3), "t_end": st["t_ticks"] / (1 << 20),
            "E0": e0, "E1": e1, "dE_over_E": (e1 - e0) / e0,
            "drift_per_time_unit": abs((e1 - e0) / e0) / max(st["t_ticks"] / (1 << 20), 1e-30),
            "max_abs_dE_over_E": max([abs(mk["dE_over_E"]) for mk in marks if "dE_over_E" in mk] + [abs((e1 - e0) / e0)]),
            "us_per_block_step": round(wall / max(st["steps"], 1) * 1e6, 2),
        }
        if marks_out:
            out["runs"][prec]["marks"] = marks
        h.close()
    if own:
        ctx.close()
    return out


def copy_calibration(nbytes=1 << 30, reps=4):
    """A plain device-to-device copy of `nbytes` (read nbytes + write nbytes
    per launch), to scale the HBM counters of the force kernel."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read_per_launch": nbytes, "copy_bytes_written_per_launch": nbytes,
                      "launches": reps, "GBps": round(2 * nbytes / dt / 1e9, 1)}), flush=True)


def block_size_table(trace_csv, steps_jsonl, n_total=65536):
    """Per-block-size time of block steps: join a rocprofv3 kernel trace
    (CSV) of a --block-run with the NBODY_TRACE step lines of the same run.
    The i-th traced step of each integrator is the i-th front-end launch of
    its precision; its pairwise launch and reduce + corrector launch follow
    it.  Launches past the last traced step (the end-time gate's no-op
    steps) are left out.  n_total: particles of the run (for the
    interaction rate).  Returns the table as text."""
    import csv
    import re
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    lines = [json.loads(x) for x in open(steps_jsonl) if '"mode": "block"' in x]
    runs, cur = [], []
    for x in lines:                      # step numbers restart with each integrator
        if cur and x["step"] <= cur[-1]["step"]:
            runs.append(cur)
            cur = []
        cur.append(x)
    if cur:
        runs.append(cur)
    name = lambda r: re.sub(r"\(.*", "", r["Kernel_Name"])
    dur = lambda r: (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    bins = [(1, 1), (2, 15), (16, 63), (64, 255), (256, 1023), (1024, 4095), (4096, 16383), (16384, 1 << 40)]
    out = []
    for prec, run in zip((0, 1), runs):     # the block run traces fp32 first, then ds
        front = [r for r in rows if f"blk_front_kernel<{prec}>" in name(r)]
        pair = [r for r in rows if f"blk_step_kernel<{prec}," in name(r)]
        rc_all = [r for r in rows if "blk_reduce_correct" in name(r)]
        rc, j = [], 0
        for r in pair:                   # the reduce + corrector launch after each pairwise launch
            t = int(r["Start_Timestamp"])
            while j < len(rc_all) and int(rc_all[j]["Start_Timestamp"]) < t:
                j += 1
            rc.append(rc_all[j] if j < len(rc_all) else None)
        acc = {b: [0, 0.0, 0.0, 0.0, 0] for b in bins}
        for k, st in enumerate(run):
            a = acc[next(b for b in bins if b[0] <= st["n_act"] <= b[1])]
            a[0] += 1
            a[1] += dur(front[k])
            a[2] += dur(pair[k])
            a[3] += dur(rc[k])
            a[4] += st["n_act"]
        out.append(f"{'fp32' if prec == 0 else 'ds'}: {len(run)} traced block steps; us per step by block size")
        out.append(f"  {'block size':>14s} {'steps':>6s} {'front':>8s} {'pairwise':>9s} {'reduce+corr':>11s} {'pairwise Gint/s':>15s}")
        for b in bins:
            a = acc[b]
            if a[0]:
                hi = "" if b[1] >= 1 << 40 else str(b[1])
                out.append(f"  {str(b[0]) + '-' + hi:>14s} {a[0]:6d} {a[1] / a[0]:8.2f} {a[2] / a[0]:9.2f} "
                           f"{a[3] / a[0]:11.2f} {a[4] * n_total / a[2] / 1e3:15.1f}")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--prec", choices=["ds", "fp32"], default="ds")
    ap.add_argument("--compare-steps", type=int, default=3,
                    help="steps timed in the other precision for comparison (0: skip)")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (HBM counter calibration)")
    ap.add_argument("--block-run", action="store_true",
                    help="only run the Salpeter block-step workload (--n, --t-end) and print its JSON")
    ap.add_argument("--t-end", type=float, default=1.0)
    ap.add_argument("--extras", default="batched,adjoint,kinds,shard,block,shared1k",
                    help="comma list of extra measurements (batched, adjoint, kinds, shard, block, shared1k) or 'none'")
    ap.add_argument("--report-every", type=float, default=0.0)
    ap.add_argument("--batched-probe", action="store_true",
                    help="only run the batched clusters briefly, eagerly, in the default shape "
                         "(profiler counter passes) and print its JSON")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch the batched steps eagerly only (no hipGraph capture), e.g. under "
                         "profiler counter passes")
    ap.add_argument("--block-sizes", nargs=2, metavar=("TRACE_CSV", "STEPS_JSONL"),
                    help="only print the per-block-size times of a traced --block-run (rocprofv3 "
                         "kernel-trace CSV, NBODY_TRACE file of the same run; its --n)")
    args = ap.parse_args()
    if args.block_sizes:
        print(block_size_table(*args.block_sizes, n_total=args.n if args.n != (1 << 20) else 65536), flush=True)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.batched_probe:
        print(json.dumps(batched_probe(args.prec)), flush=True)
        return
    if args.block_run:
        out = block_run(args.n if args.n != (1 << 20) else 65536, args.t_end, ["fp32", "ds"], args.report_every)
        print(json.dumps(out), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described in the design notes, not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import nbody_inputs as ics
    import paper_0707_0438_amd as nb

    eps = 1e-4
    n = args.n
    log(f"[bench] generating Plummer N={n}")
    p = ics.plummer(n, ics.seed_for(2))
    X = torch.from_numpy(p.pos).to("cuda")
    V = torch.from_numpy(p.vel).to("cuda")
    M = torch.from_numpy(p.mass).to("cuda")
    ctx = nb.Context(0)
    results = {}
    for prec, steps in ((args.prec, args.steps),
                        ("fp32" if args.prec == "ds" else "ds", args.compare_steps)):
        if steps <= 0:
            continue
        h = ctx.hermite(n, eps=eps, shared_dt_log2=-10, prec=prec)
        log(f"[bench] {prec}: initial evaluation")
        h.set_state(X, V, M)
        torch.cuda.synchronize()
        log(f"[bench] {prec}: {args.warmup} warm-up + {steps} timed steps")
        wall, active, kms, launches = time_steps(ctx, h, steps, args.warmup)
        inter = float(active) * n
        results[prec] = {"wall": wall, "inter": inter, "kms": kms, "launches": launches,
                         "tile": ctx.get_tile(n, n, prec), "steps": steps}
        log(f"[bench] {prec}: {wall:.3f} s, {inter / wall / 1e9:.1f} Gint/s, "
            f"kernel {kms / max(launches, 1):.2f} ms/launch")
        h.close()
    r = results[args.prec]
    value = r["inter"] / r["wall"] / 1e9
    k_ms = r["kms"] / max(r["launches"], 1)
    achieved = FLOPS_PER_INTERACTION * float(n) * n / (k_ms * 1e-3) / 1e12
    traffic = traffic_per_launch(args.prec)
    line = {
        "metric": "Ginteractions/s (acc+jerk) at N=2^20, % FP32 peak; adjoint/forward time",
        "value": round(value, 3),
        "unit": "Ginteractions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["wall"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(value / PAPER_GINT_S, 2),
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "plummer1m_force: equal-mass Plummer sphere N=2^20 (seeded AHW sampling), "
                        "eps=1e-4, all particles active; one step = pairwise acc/jerk/pot + f64 Hermite "
                        "corrector fused with the f64 predict/pack of the next step (shared dt 2^-10)",
            "n": n, "eps": eps, "G": 1.0,
            "prec": "ds_comp" if args.prec == "ds" else "fp32",
            "tile": r["tile"],
        },
        "pct_fp32_peak": round(100.0 * FLOPS_PER_INTERACTION * value * 1e9 / (FP32_PEAK_TFLOPS * 1e12), 2),
        "device": device_info(),
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
            "traffic": traffic,
            "kernel": "force_kernel (pairwise acc+jerk+pot)",
            "kernel_ms": round(k_ms, 3),
            "launches": r["launches"],
        },
    }
    other = "fp32" if args.prec == "ds" else "ds"
    if other in results:
        o = results[other]
        ov = o["inter"] / o["wall"] / 1e9
        line[f"{other}_compare"] = {
            "value": round(ov, 3),
            "ms_per_step": round(o["wall"] / o["steps"] * 1e3, 3),
            "kernel_ms": round(o["kms"] / max(o["launches"], 1), 3),
            "pct_fp32_peak": round(100.0 * FLOPS_PER_INTERACTION * ov * 1e9 / (FP32_PEAK_TFLOPS * 1e12), 2),
        }
    line["executed"] = executed_flops(args.prec, float(n) * n / (k_ms * 1e-3) / 1e9)
    extras = [] if args.extras == "none" else args.extras.split(",")
    precs = (args.prec, other)
    pname = lambda q: "ds_comp" if q == "ds" else "fp32"
    if "batched" in extras:
        line["batched"] = {}
        for q in precs:
            log(f"[bench] batched clusters ({q})")
            line["batched"][pname(q)] = batched_timing(ctx, q, graph=not args.no_graph)
    if "adjoint" in extras:
        line["adjoint"] = {}
        for q in precs:
            log(f"[bench] adjoint/forward timing ({q})")
            line["adjoint"][pname(q)] = adjoint_timing(nb, ctx, q)
    if "kinds" in extras:
        log("[bench] force-only and nearest-neighbour evaluations")
        line["kinds"] = kinds_timing(ctx, X, V, M, eps, args.prec, k_ms)
    if "shard" in extras:
        log("[bench] one GPU's share of an 8-GPU i-parallel evaluation")
        line["shard8"] = shard_timing(ctx, X, V, M, eps, args.prec, k_ms)
    if "block" in extras:
        log("[bench] block steps, Salpeter N=65536 to t=1 (energy every 1/4)")
        line["block_steps"] = block_run(65536, 1.0, ["ds", "fp32"], report_every=0.25, ctx=ctx)
    if "shared1k" in extras:
        log("[bench] shared steps, N=1024")
        line["shared1k"] = shared1k_timing(ctx)
    if args.cpu_budget > 0:
        log("[bench] cpu baseline (oracle)")
        line["cpu_baseline"], ref, k = cpu_baseline(p, eps, args.cpu_budget)
        log("[bench] accuracy of both precisions on the oracle's rows")
        line["accuracy"] = accuracy(ctx, X, V, M, eps, ref, k)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
