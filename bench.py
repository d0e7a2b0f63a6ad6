#!/usr/bin/env python3
"""Joint MM vs alternating MU on one MI355X: iterations/s, time-to-objective,
per-kernel roofline, and the FP64 CPU oracle timed on the host cores.

A step is one outer iteration (W update, H update, normalization, objective of
the entry iterate) of the joint method on the chosen workload; the alternating
method is timed the same way and reported beside it.  Inputs are resident in
device memory before timing starts.

    python bench.py [--steps K] [--warmup W] [--workload batched]

The default workload is the largest single-GPU configuration: 512 uneven
problems (F in 128..1025, N in 200..5000, K in 8..64, beta in {0, .5, 1, 1.5, 2})
updated by one persistent launch per outer iteration, replayed from a HIP
graph.  `--workload counts_kl` (20000 x 10000, K = 50, beta = 1), `faces_euc`,
`spectro_is` and `tiny_kl` time one problem instead.

Prints one JSON line.  Only one GPU is used; --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "joint-MM vs alternating-MU iterations/s and time-to-objective per β, 1 MI355X"
PEAK_MFMA = {"fp32": 157.3e12, "bf16": 2.5e15, "fp16": 2.5e15}  # dense matrix FLOP/s
PEAK_HBM = 8.0e12           # bytes/s
# float32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz x 2
# (two-wide packed FMA) = 157.3 TFLOP/s; without packed instructions half of it
PEAK_VALU_F32 = 157.3e12


# The paper's own measurements (CPU time to its stopping rule, Matlab 2020a on an
# Intel i7-8650U at 1.90 GHz, 16 GB RAM; Sec. 4, Table 4): context, not a target.
PAPER_CPU_REFERENCE = {
    "hardware": "Intel i7-8650U @ 1.90 GHz, 16 GB RAM, Matlab 2020a (precision and threads not stated)",
    "metric": "CPU seconds to the 1e-5 relative-decrease stop, mean over 25 initializations",
    "rows": [
        {"data": "faces 4096x400", "beta": 2, "K": 10, "bmm_s": 55, "jmm_s": 36, "reduction": "35%"},
        {"data": "faces 4096x400", "beta": 1, "K": 10, "bmm_s": 40, "jmm_s": 34, "reduction": "16%"},
        {"data": "faces 4096x400", "beta": 0, "K": 10, "bmm_s": 229, "jmm_s": 63, "reduction": "72%"},
        {"data": "spectrogram 1025x2152", "beta": 0, "K": 10, "bmm_s": 291, "jmm_s": 41, "reduction": "86%"},
        {"data": "play counts 16301x12118", "beta": 1, "K": 50, "bmm_s": 6776, "jmm_s": 5909, "reduction": "13%"},
        {"data": "hyperspectral 189x2500", "beta": 2, "K": 3, "bmm_s": 39, "jmm_s": 24, "reduction": "35%"},
        {"data": "hyperspectral 189x2500", "beta": 1.5, "K": 3, "bmm_s": 107, "jmm_s": 123, "reduction": "-18%"},
    ],
}


def _flops_bytes(F, N, K, beta, mode, gram=False):
    """Algorithmic work per launch of each kernel (one outer iteration).

    sweep_w    : Lambda = W~H~ (2FNK) + P H~^T (2FNK) + Q H~^T (2FNK; omitted at
                 beta = 1, where the denominator is a row sum, and in the Gram
                 form at beta = 2, where it is W~ (H~ H~^T)); reads V once (4FN bytes).
    sweep_h    : the two H-step contractions (4FNK; 2FNK at beta = 1 and in the
                 Gram form).  Re-forming Lambda costs another 2FNK: algorithmic
                 for the alternating method (Lambda' = W_new H~; not needed in the
                 Gram form), implementation overhead for the joint one.
    fused_step : the whole iteration: joint 10FNK (6FNK at beta = 1) reading V
                 once; alternating 12FNK (8FNK) reading V twice.
    """
    b1 = (beta == 1.0)
    fnk = F * N * K
    sw = (4 if b1 or gram else 6) * fnk
    sh = (2 if b1 or gram else 4) * fnk + (2 * fnk if mode == "alternating" and not gram else 0)
    vb = 4 * F * N
    return {"sweep_w": (sw, vb), "sweep_h": (sh, vb),
            "fused_step": (sw + sh, vb if mode == "joint" else 2 * vb)}


KERNEL_NAMES = ("sweep_w", "update_w", "sweep_h", "update_h", "fused_step")


def source_digest() -> str:
    """SHA-256 over the library sources and the public header: identifies the
    kernels a committed counter summary was taken on."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2106_15214_amd", "csrc", "*")))
    files += sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, precision: str, kernel: str, beta=None, field: str = "traffic_joint"):
    """Calibrated HBM bytes per launch of `kernel` in the joint step, from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of this workload, or None
    when there is none, it was taken at another beta (another kernel
    instantiation), or the kernels changed since it was taken.  `field`
    "mfma_busy" reads the matrix-core utilization of the same summary instead."""
    name = f"kernels_{workload}" + ("" if precision == "fp32" else f"_precision_{precision}") + ".txt"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    digest, value, pbeta = None, None, None
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 2 and parts[0] == "source_sha256":
                digest = parts[1]
            elif len(parts) == 2 and parts[0] == "beta":
                pbeta = float(parts[1])
            elif len(parts) == 3 and parts[0] == field and parts[1] == kernel:
                value = float(parts[2])
    if digest != source_digest():
        return None
    if beta is not None and pbeta != float(beta):
        return None
    return value


# outer iterations of each workload's time-to-objective runs (the iteration
# counts of the configurations; independent of --steps)
TTO_ITERS = {"tiny_kl": 100, "faces_euc": 500, "spectro_is": 300, "counts_kl": 100, "counts_kl_sparse": 100,
             "batched": 200}
DEFAULT_STEPS = {"batched": 50, "counts_kl": 50, "counts_kl_sparse": 50}


def cpu_model() -> str:
    """Host CPU model name (from /proc/cpuinfo), for the CPU-baseline record."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    import platform
    return platform.processor() or "unknown"


_GRAM = {"on": False}  # --gram: the Gram-form denominators at beta = 2


def _run_steps(nb, V, W, H, beta, mode, n, ctx, obj=None, trace=None, precision="fp32", inner=1):
    gram = _GRAM["on"] and beta == 2.0
    for t in range(n):
        o = trace[t:t + 1] if trace is not None else obj
        nb.step(V, W, H, beta, mode, precision=precision, inner_iters=inner, gram=gram, objective_out=o, ctx=ctx)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed iterations (default 50 for batched and counts_kl, else 500)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed iterations (default 5 batched, else 20)")
    ap.add_argument("--workload", default="batched",
                    choices=["batched", "counts_kl", "counts_kl_sparse", "faces_euc", "spectro_is", "tiny_kl"])
    ap.add_argument("--gram", action="store_true",
                    help="beta = 2: Gram-form denominators (K x K products) instead of the Q contractions")
    ap.add_argument("--sparse", action="store_true",
                    help="count workloads: V by its nonzeros (CSR + CSC), the sparse beta = 1 path")
    ap.add_argument("--tto-iters", type=int, default=None,
                    help="iterations of the time-to-objective runs (default: the workload's own count)")
    ap.add_argument("--beta", type=float, default=None)
    ap.add_argument("--kappa", type=float, default=None,
                    help="batched workload: smoothing constant of Sec. 4.1.3 (default 1e-9: its count data with "
                         "zeros at beta < 1 drive entries of WH to zero at kappa = 0)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the oracle timing sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration under a profiler)")
    ap.add_argument("--path", default="auto", choices=["auto", "stream", "fused"])
    ap.add_argument("--target-blocks", type=int, default=0)
    ap.add_argument("--min-tiles", type=int, default=0)
    ap.add_argument("--problems", type=int, default=512, help="batched workload: number of problems")
    ap.add_argument("--tune", default=None,
                    help="batched workload: tune the per-bucket tile table, caching it in this text file")
    ap.add_argument("--tiles", type=int, default=0, help="batched workload: tiles per pass item (0: library default)")
    ap.add_argument("--lag", type=int, default=0, help="batched workload: queue order (0 phase-major, d pipelined)")
    ap.add_argument("--inner-iters", type=int, default=1,
                    help="sub-iterations L per outer iteration (both methods; L > 1: float32)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp16"],
                    help="operand type of the matrix products (element-wise terms stay float32)")
    args = ap.parse_args(argv)
    if args.steps is None:
        args.steps = DEFAULT_STEPS.get(args.workload, 500)
    if args.warmup is None:
        args.warmup = 5 if args.workload == "batched" else 20
    if args.tto_iters is None:
        args.tto_iters = TTO_ITERS[args.workload]
    _GRAM["on"] = bool(args.gram)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}), flush=True)
        return 2

    import numpy as np
    import torch
    import synth
    import paper_2106_15214_amd as nb

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        return 2
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "batched":
        return main_batched(args, nb, synth, torch, np, dev)
    if args.sparse:
        if not args.workload.startswith("counts_kl"):
            print(json.dumps({"error": "--sparse applies to the count workloads"}), flush=True)
            return 2
        return main_sparse(args, nb, synth, torch, np, dev)
    p = synth.make_problem(args.workload, beta=args.beta)
    F, N, K = p.shape
    beta = p.beta
    print(f"# workload {args.workload}: F={F} N={N} K={K} beta={beta}", file=sys.stderr, flush=True)

    ctx = nb.Context(0)
    ctx.set_launch(args.target_blocks, args.min_tiles)
    ctx.set_path(args.path)
    ctx.reserve(F, N, K)
    V = torch.from_numpy(p.V).to(dev)
    W0 = torch.from_numpy(p.W).to(dev)
    H0 = torch.from_numpy(p.H).to(dev)
    obj = torch.zeros(1, dtype=torch.float64, device=dev)
    res = {}

    for mode in ("joint", "alternating"):
        W, H = W0.clone(), H0.clone()
        _run_steps(nb, V, W, H, beta, mode, args.warmup, ctx, obj=obj, precision=args.precision,
                   inner=args.inner_iters)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        _run_steps(nb, V, W, H, beta, mode, args.steps, ctx, obj=obj, precision=args.precision,
                   inner=args.inner_iters)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1) / args.steps
        res[mode] = {"ms_per_step": ms, "iters_per_s": 1e3 / ms, "wall_s": wall}
        print(f"# {mode}: {ms * 1e3:.2f} us/iteration ({1e3 / ms:.1f} it/s)", file=sys.stderr, flush=True)
    if nb.get_flags(clear=True, ctx=ctx):
        print("# warning: numeric flags raised", file=sys.stderr)

    # per-kernel durations with HIP events on the launch stream (same K steps)
    kern, phases = {}, {}
    for mode in ("joint", "alternating"):
        W, H = W0.clone(), H0.clone()
        _run_steps(nb, V, W, H, beta, mode, 2, ctx, obj=obj, precision=args.precision)
        torch.cuda.synchronize()
        ctx.profile(KERNEL_NAMES)
        _run_steps(nb, V, W, H, beta, mode, args.steps, ctx, obj=obj, precision=args.precision)
        torch.cuda.synchronize()
        kern[mode] = {}
        for k in KERNEL_NAMES:
            tot, n = ctx.profile_read(k)
            if n:
                kern[mode][k] = {"avg_us": 1e3 * tot / n, "launches": n}
        if "fused_step" in kern[mode]:
            phases[mode] = dict(zip(["w_pass", "barrier1", "w_update", "barrier2", "h_pass", "barrier3", "h_update"],
                                    [round(x, 2) for x in ctx.profile_phases()]))
        ctx.profile([])
    fb = _flops_bytes(F, N, K, beta, "joint", gram=args.gram)
    dom = max((k for k in kern["joint"] if k in fb), key=lambda k: kern["joint"][k]["avg_us"])
    flops, vbytes = fb[dom]
    t_dom = kern["joint"][dom]["avg_us"] * 1e-6
    intensity = flops / vbytes
    peak_mfma = PEAK_MFMA[args.precision]
    if intensity >= peak_mfma / PEAK_HBM:
        roof = {"bound": "mfma", "achieved": flops / t_dom / 1e12, "peak": peak_mfma / 1e12,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": vbytes / t_dom / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(args.workload, args.precision, dom, beta)
    roof["mfma_busy_profiled"] = measured_traffic(args.workload, args.precision, dom, beta, field="mfma_busy")
    roof["kernel"] = dom
    roof["algorithmic_flops_per_launch"] = flops
    roof["algorithmic_bytes_per_launch"] = vbytes
    roof["avg_launch_us"] = kern["joint"][dom]["avg_us"]

    # backward: gradient of D_beta w.r.t. W and H (plus the objective) in one call,
    # as the autograd function's backward runs it
    W, H = W0.clone(), H0.clone()
    dW, dH = torch.empty_like(W), torch.empty_like(H)
    og = torch.zeros(1, dtype=torch.float64, device=dev)
    nb.grad(V, W, H, beta, dW=dW, dH=dH, objective_out=og, ctx=ctx)
    torch.cuda.synchronize()
    ng = max(1, min(args.steps, 50))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(ng):
        nb.grad(V, W, H, beta, dW=dW, dH=dH, objective_out=og, ctx=ctx)
    e1.record()
    torch.cuda.synchronize()
    grad_ms = e0.elapsed_time(e1) / ng

    # time-to-objective: same init, objective of every iterate, T = the
    # workload's iteration count
    T = args.tto_iters
    tto_main = time_to_objective(nb, torch, np, ctx, V, W0, H0, beta, T, args.precision, dev, args.inner_iters)
    tto_main.pop("_traces")
    # the same for every beta of the paper's experiments on this data (at most
    # 500 iterations; beta <= 0 only when V has no zero, where d_beta is finite)
    per_beta = {}
    has_zero = bool((V == 0).any().item())
    for b in (0.0, 0.5, 1.0, 1.5, 2.0):
        if b <= 0.0 and has_zero:
            continue
        r = time_to_objective(nb, torch, np, ctx, V, W0, H0, b, min(T, 500), args.precision, dev, args.inner_iters)
        r.pop("_traces")
        per_beta[str(b)] = r

    out = {
        "metric": METRIC,
        "value": res["joint"]["iters_per_s"],
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["joint"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp16": "f16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "F": F, "N": N, "K": K, "beta": beta, "mode": "joint",
                   "inner_iters": args.inner_iters,
                   "precision": args.precision, "objective_every_step": True, "normalize": True,
                   "gram_denominators": bool(args.gram and beta == 2.0),
                   "path": "fused" if "fused_step" in kern["joint"] else "stream"},
        "alternating": {"value": res["alternating"]["iters_per_s"], "ms_per_step": res["alternating"]["ms_per_step"]},
        "joint_speedup_per_iteration": res["alternating"]["ms_per_step"] / res["joint"]["ms_per_step"],
        "backward_ms": grad_ms,
        "time_to_objective": tto_main,
        "time_to_objective_per_beta": per_beta,
        "roofline": roof,
        "paper_cpu_reference": PAPER_CPU_REFERENCE,
        "kernels_us": kern,
        "fused_phases_us": phases,
    }

    if args.calib_copy:
        out["calib_copy_bytes"] = calib_copy(torch, dev)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds, res["joint"]["iters_per_s"])
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def main_sparse(args, nb, synth, torch, np, dev):
    """The beta = 1 step on a count workload held by its nonzeros (CSR and CSC):
    iterations/s of both methods with the objective of every iterate, the
    row/column pass kernel against its roofline, time-to-objective."""
    p = synth.make_problem(args.workload)
    F, N, K = p.shape
    rp, ci, rv = synth.to_csr(p.V)
    cp, ri, cv = synth.to_csc(p.V)
    nnz = int(ci.size)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    Vs = nb.SparseV(F, N, t(rp), t(ci), t(rv), t(cp), t(ri), t(cv))
    print(f"# sparse {args.workload}: F={F} N={N} K={K} nnz={nnz} ({nnz / (F * N) * 100:.2f}%)", file=sys.stderr,
          flush=True)
    ctx = nb.Context(0)
    W0, H0 = t(p.W), t(p.H)
    obj = torch.zeros(1, dtype=torch.float64, device=dev)
    res, kern = {}, {}
    for mode in ("joint", "alternating"):
        W, H = W0.clone(), H0.clone()
        for _ in range(args.warmup):
            nb.kl_step_sparse(Vs, W, H, mode, objective_out=obj, ctx=ctx)
        torch.cuda.synchronize()
        # the step's short launches are replayed from a HIP graph (one step per
        # replay), so the host's launch rate does not set the iteration time
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            nb.kl_step_sparse(Vs, W, H, mode, objective_out=obj, ctx=ctx)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        del graph
        # eager launches, for comparison
        e0.record()
        for _ in range(args.steps):
            nb.kl_step_sparse(Vs, W, H, mode, objective_out=obj, ctx=ctx)
        e1.record()
        torch.cuda.synchronize()
        eager = e0.elapsed_time(e1) / args.steps
        res[mode] = {"ms_per_step": ms, "iters_per_s": 1e3 / ms, "eager_ms_per_step": eager}
        print(f"# sparse {mode}: {ms * 1e3:.1f} us/iteration (graph), {eager * 1e3:.1f} eager", file=sys.stderr,
              flush=True)
        ctx.profile(["sparse_pass", "sparse_cols"])
        for _ in range(args.steps):
            nb.kl_step_sparse(Vs, W, H, mode, objective_out=obj, ctx=ctx)
        torch.cuda.synchronize()
        kern[mode] = {}
        for k in ("sparse_pass", "sparse_cols"):
            tot, n = ctx.profile_read(k)
            if n:
                kern[mode][k] = {"avg_us": 1e3 * tot / n, "launches": n}
        ctx.profile([])
    if nb.get_flags(clear=True, ctx=ctx):
        print("# warning: numeric flags raised", file=sys.stderr)
    # dominant kernel: the joint pass (row pass + column pass in one launch).
    # Per stored entry and traversal: lambda (2K flops), the numerator term (2K),
    # and 8 bytes of index and value; both traversals per launch.
    t_dom = kern["joint"]["sparse_pass"]["avg_us"] * 1e-6
    flops = 2 * nnz * 4 * K
    nbytes = 2 * nnz * 8
    roof = {"bound": "alu", "achieved": flops / t_dom / 1e12, "peak": PEAK_VALU_F32 / 1e12, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(args.workload + "_csr", "fp32", "sparse_pass")
    roof["kernel"] = "sparse_pass"
    roof["algorithmic_flops_per_launch"] = flops
    roof["algorithmic_bytes_per_launch"] = nbytes
    roof["avg_launch_us"] = kern["joint"]["sparse_pass"]["avg_us"]
    roof["hbm_GBps_algorithmic"] = nbytes / t_dom / 1e9
    # time-to-objective from the common init
    T = args.tto_iters
    traces = {}
    for mode in ("joint", "alternating"):
        W, H = W0.clone(), H0.clone()
        tr = torch.zeros(T + 1, dtype=torch.float64, device=dev)
        for i in range(T):
            nb.kl_step_sparse(Vs, W, H, mode, objective_out=tr[i:i + 1], ctx=ctx)
        nb.kl_objective_sparse(Vs, W, H, out=tr[T:T + 1], ctx=ctx)
        torch.cuda.synchronize()
        traces[mode] = tr.cpu().numpy()
    tto = targets_from_traces(np, traces, {m: res[m]["ms_per_step"] for m in res})
    out = {
        "metric": METRIC, "value": res["joint"]["iters_per_s"], "unit": "iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["joint"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload + " (sparse V)", "F": F, "N": N, "K": K, "beta": 1.0, "nnz": nnz,
                   "density": nnz / (F * N), "mode": "joint", "objective_every_step": True, "normalize": True,
                   "graph_replay": True},
        "alternating": {"value": res["alternating"]["iters_per_s"], "ms_per_step": res["alternating"]["ms_per_step"]},
        "joint_speedup_per_iteration": res["alternating"]["ms_per_step"] / res["joint"]["ms_per_step"],
        "eager_ms_per_step": {m: res[m]["eager_ms_per_step"] for m in res},
        "time_to_objective": dict(T=T, **tto), "roofline": roof, "kernels_us": kern,
        "paper_cpu_reference": PAPER_CPU_REFERENCE,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_sparse(p, (rp, ci, rv), args.cpu_seconds, res["joint"]["iters_per_s"])
    if args.calib_copy:
        out["calib_copy_bytes"] = calib_copy(torch, dev)
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def targets_from_traces(np, traces, tper):
    """Iterations and milliseconds for both methods to reach 90 / 99 / 99.9 / 100 %
    of the larger final decrease, from objective traces of the same init."""
    D0 = traces["joint"][0]
    Dend = max(traces["joint"][-1], traces["alternating"][-1])
    rows = {}
    for q in (0.9, 0.99, 0.999, 1.0):
        target = D0 - q * (D0 - Dend)
        row = {"target": float(target)}
        for mode in traces:
            hit = np.nonzero(traces[mode] <= target * (1 + 1e-12))[0]
            it = int(hit[0]) if hit.size else None
            row[mode] = {"iterations": it, "ms": (it * tper[mode]) if it is not None else None}
        rows[str(q)] = row
    return {"D0": float(D0), "D_T": {m: float(traces[m][-1]) for m in traces}, "ms_per_iteration": tper,
            "targets": rows, "objective_increases": {m: int(np.sum(np.diff(traces[m]) > 0)) for m in traces}}


def cpu_baseline_sparse(p, csr, budget_s, gpu_value):
    """The FP64 oracle's sparse joint iteration (objective + update +
    normalization) on the whole count workload, all threads and one thread."""
    import numpy as np
    import oracle
    rp, ci, rv = csr
    state = {"W": p.W.astype(np.float64), "H": p.H.astype(np.float64)}

    def one():
        oracle.kl_sparse_objective(rp, ci, rv, state["W"], state["H"])
        state["W"], state["H"] = oracle.kl_sparse_iteration(rp, ci, rv, state["W"], state["H"], "joint")

    n_all, el_all, th_all = _timed_oracle(one, budget_s / 2)
    state.update(W=p.W.astype(np.float64), H=p.H.astype(np.float64))
    n_one, el_one, _ = _timed_oracle(one, budget_s / 2, threads=1)
    return {"value": n_all / el_all, "unit": "iterations/s", "cores": th_all, "kind": "oracle",
            "sample": f"{n_all} sparse joint iterations (objective + update + normalization, float64 NumPy, "
                      f"row loops) of the {p.name} workload in {el_all:.1f} s on {th_all} threads; {n_one} in "
                      f"{el_one:.1f} s on 1 thread",
            "one_thread": {"value": n_one / el_one, "cores": 1}, "cpu_model": cpu_model(),
            "host_cores_available": len(os.sched_getaffinity(0)), "gpu_over_cpu": gpu_value / (n_all / el_all)}


def time_to_objective(nb, torch, np, ctx, V, W0, H0, beta, T, precision, dev, inner=1):
    """Both methods from the same init for T iterations with the objective of
    every iterate: iterations and milliseconds to reach 90 / 99 / 99.9 / 100 % of
    the larger final decrease, the iteration where the 1e-5 relative-decrease
    stop fires, and the count of objective increases."""
    traces, tper = {}, {}
    for mode in ("joint", "alternating"):
        W, H = W0.clone(), H0.clone()
        tr = torch.zeros(T + 1, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _run_steps(nb, V, W, H, beta, mode, T, ctx, trace=tr, precision=precision, inner=inner)
        e1.record()
        nb.objective(V, W, H, beta, out=tr[T:T + 1], ctx=ctx)
        torch.cuda.synchronize()
        traces[mode] = tr.cpu().numpy()
        tper[mode] = e0.elapsed_time(e1) / T
    D0 = traces["joint"][0]
    Dend = max(traces["joint"][-1], traces["alternating"][-1])
    tto = {}
    for q in (0.9, 0.99, 0.999, 1.0):
        target = D0 - q * (D0 - Dend)
        row = {"target": target}
        for mode in ("joint", "alternating"):
            hit = np.nonzero(traces[mode] <= target * (1 + 1e-12))[0]
            it = int(hit[0]) if hit.size else None
            row[mode] = {"iterations": it, "ms": (it * tper[mode]) if it is not None else None}
        tto[str(q)] = row
    # the stopping rule of Sec. 4.1.2 (eps = 1e-5) evaluated on the device by
    # the library's run call, from the same init, within the same T iterations
    stop = {}
    for mode in ("joint", "alternating"):
        W, H = W0.clone(), H0.clone()
        _, st = nb.run(V, W, H, beta, mode, max_iters=T, eps=1e-5, precision=precision, inner_iters=inner,
                       gram=_GRAM["on"] and beta == 2.0, ctx=ctx)
        t_stop = int(st.item())
        stop[mode] = t_stop if t_stop >= 0 else None
    mono = {m: int(np.sum(np.diff(traces[m]) > 0)) for m in traces}
    return {"T": T, "D0": float(D0), "D_T": {m: float(traces[m][-1]) for m in traces}, "ms_per_iteration": tper,
            "targets": tto, "stop_rule_1e-5_iteration": stop, "objective_increases": mono, "_traces": traces}


def calib_copy(torch, dev):
    """A plain 256 MiB device-to-device copy (three times): the known-size
    reference that scales FETCH_SIZE / WRITE_SIZE counter readings."""
    x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    return {"read": x.numel() * 4, "write": y.numel() * 4}


def main_batched(args, nb, synth, torch, np, dev):
    """Many uneven problems (each with its own beta and rank) updated by one
    persistent launch per outer iteration, replayed from a HIP graph.  A step is
    one outer iteration of every problem; `value` is steps per second."""
    specs = synth.batched_specs(args.problems)
    # Sec. 4.1.3's smoothing: at kappa = 0 the count-data problems with zeros at
    # beta < 1 drive entries of WH to zero within ~130 iterations (in float64 as
    # well) until an update ratio is undefined
    kappa = 1e-9 if args.kappa is None else float(args.kappa)
    args.kappa_batched = kappa
    t0 = time.perf_counter()
    probs, host = [], []
    for sp in specs:
        q = synth.make_batched_problem(sp)
        host.append(q)
        probs.append((torch.from_numpy(q.V).to(dev), torch.from_numpy(q.W).to(dev), torch.from_numpy(q.H).to(dev),
                      q.beta))
    fnk = sum(q.V.shape[0] * q.V.shape[1] * q.W.shape[1] for q in host)
    fn = sum(q.V.shape[0] * q.V.shape[1] for q in host)
    # algorithmic work of one outer iteration (Sec. 3.3.2, Table 3 counts of the
    # products): joint 10 FNK (6 FNK at beta = 1: the W-step denominator is a row
    # sum and Q = 1), alternating 12 FNK (8 FNK) with Lambda' formed again; V is
    # read by both passes (8 FN bytes)
    def alg_flops(mode):
        c1, c = (6, 10) if mode == "joint" else (8, 12)
        return sum((c1 if q.beta == 1.0 else c) * q.V.shape[0] * q.V.shape[1] * q.W.shape[1] for q in host)
    vbytes = 8 * fn
    print(f"# batched: {len(probs)} problems, sum FN = {fn:.3e}, sum FNK = {fnk:.3e} "
          f"(generated in {time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    ctx = nb.Context(0)
    cfg = {"tiles_per_item": args.tiles, "workers": 0, "lag": args.lag}
    tuned_ms = None
    if args.tune:
        tiles, tuned_ms, hit = nb.tune(probs, "joint", precision=args.precision, kappa=kappa, iters=3, cache=args.tune,
                                      ctx=ctx)
        print(f"# tuned bucket tiles {tiles} ({tuned_ms:.3f} ms/step, {'cached' if hit else 'measured'})",
              file=sys.stderr, flush=True)
    bucket_tiles = nb.get_batch_tiles(ctx)
    res, traces = {}, {}
    W0 = [(W.clone(), H.clone()) for _, W, H, _ in probs]

    def reset():
        for (_, W, H, _), (Ws, Hs) in zip(probs, W0):
            W.copy_(Ws)
            H.copy_(Hs)

    T = args.tto_iters
    for mode in ("joint", "alternating"):
        reset()
        b = nb.Batch(probs, mode, precision=args.precision, kappa=kappa, ctx=ctx, **cfg)
        obj = torch.zeros(len(probs), dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            b.step(objectives=obj)
        torch.cuda.synchronize()
        # one iteration of all problems = one persistent launch, captured in a graph
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            b.step(objectives=obj)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        fl = b.flags(clear=True)
        res[mode] = {"ms_per_step": ms, "steps_per_s": 1e3 / ms, "flags": fl, "graph_replay": True, **b.info()}
        print(f"# {mode}: {ms:.3f} ms/step (graph replays), flags {fl}, {b.info()}", file=sys.stderr, flush=True)
        del graph
        # time-to-objective: T iterations from the common init, the objective of
        # every problem's iterate 0..T recorded on the device
        reset()
        tr = torch.zeros((T + 1, len(probs)), dtype=torch.float64, device=dev)
        for t in range(T + 1):
            b.step(objectives=tr[t])
        torch.cuda.synchronize()
        traces[mode] = tr.cpu().numpy()
        if b.flags(clear=True):
            print(f"# warning: flags raised in the {mode} trajectory", file=sys.stderr, flush=True)
        b.close()
        if args.tiles == 0 and args.lag == 0:
            res[mode]["device_planned_ms_per_step"] = device_planned_ms(nb, torch, probs, mode, args, ctx, reset)
    tto = batched_time_to_objective(np, host, traces, {m: res[m]["ms_per_step"] for m in res}, T)

    t = res["joint"]["ms_per_step"] * 1e-3
    flops = alg_flops("joint")
    peak_mfma = PEAK_MFMA[args.precision]
    if flops / vbytes >= peak_mfma / PEAK_HBM:
        roof = {"bound": "mfma", "achieved": flops / t / 1e12, "peak": peak_mfma / 1e12, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": vbytes / t / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic("batched", args.precision, "batched_step")
    roof["mfma_busy_profiled"] = measured_traffic("batched", args.precision, "batched_step", field="mfma_busy")
    roof["kernel"] = "batched_step"
    roof["algorithmic_flops_per_launch"] = flops
    roof["algorithmic_bytes_per_launch"] = vbytes
    roof["avg_launch_us"] = res["joint"]["ms_per_step"] * 1e3
    ta = res["alternating"]["ms_per_step"] * 1e-3
    alt_frac = (alg_flops("alternating") / ta / peak_mfma) if roof["bound"] == "mfma" else (vbytes / ta / PEAK_HBM)
    out = {
        "metric": METRIC,
        "value": res["joint"]["steps_per_s"],
        "unit": "iterations/s (all problems per iteration)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["joint"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp16": "f16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "batched", "problems": len(probs), "sum_FN": fn, "sum_FNK": fnk, "mode": "joint",
                   "precision": args.precision, "kappa": kappa, "objective_every_step": True, "launches_per_step": 1,
                   "graph_replay": True, **cfg, "bucket_tiles": bucket_tiles},
        "problem_iterations_per_s": len(probs) * res["joint"]["steps_per_s"],
        "alternating": {"value": res["alternating"]["steps_per_s"], "ms_per_step": res["alternating"]["ms_per_step"],
                        "roofline_frac": alt_frac},
        "joint_speedup_per_iteration": res["alternating"]["ms_per_step"] / res["joint"]["ms_per_step"],
        "time_to_objective_per_beta": tto,
        "tuned_ms": tuned_ms,
        "roofline": roof,
        "paper_cpu_reference": PAPER_CPU_REFERENCE,
        "batch": res,
    }
    if args.calib_copy:
        out["calib_copy_bytes"] = calib_copy(torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(host, args.cpu_seconds, res["joint"]["steps_per_s"], kappa)
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def device_planned_ms(nb, torch, probs, mode, args, ctx, reset):
    """Time per step of the same batch through nmf_beta_step_batched (the
    descriptors in device memory, planned on the device each step: a planning
    launch plus the persistent launch), replayed from a graph."""
    reset()
    shapes = [(V.shape[0], V.shape[1], W.shape[1], beta) for V, W, H, beta in probs]
    tiles = nb.get_batch_tiles(ctx)
    ctx = nb.Context(0)  # its own region: a captured region is never re-reserved
    nb.set_batch_tiles(tiles, ctx=ctx)
    items, nbytes = nb.batch_requirements(shapes, mode, tiles, args.precision)
    nb.reserve_batched(len(probs), items, nbytes, ctx=ctx)
    dp = nb.DeviceProblems(len(probs))
    dp.set(probs)
    obj = torch.zeros(len(probs), dtype=torch.float64, device=probs[0][0].device)
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        nb.step_batched(dp, mode, precision=args.precision, kappa=args.kappa_batched, objectives=obj, stream=s, ctx=ctx)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    fl = nb.get_flags(clear=True, ctx=ctx)
    print(f"# {mode}: {ms:.3f} ms/step device-planned (graph replays), flags {fl}", file=sys.stderr, flush=True)
    del graph
    ctx.close()
    return ms


def batched_time_to_objective(np, host, traces, ms_per_iter, T):
    """Per beta group (and for the whole batch): the summed objective of the
    group's problems at iterates 0..T of both methods from the same init, and
    the iterations and milliseconds (whole-batch iteration time) to reach
    90 / 99 / 99.9 / 100 % of the larger final decrease.  Also the number of
    per-problem objective increases."""
    betas = np.array([q.beta for q in host])
    # a problem whose trajectory reached an undefined update (a factor entry
    # underflowed to zero in float32: flagged, non-finite objective) in either
    # method is left out of the sums and counted
    finite = np.all(np.isfinite(traces["joint"]), axis=0) & np.all(np.isfinite(traces["alternating"]), axis=0)
    groups = {str(b): betas == b for b in sorted(set(betas.tolist()))}
    groups["all"] = np.ones_like(betas, dtype=bool)
    out = {"T": T, "ms_per_iteration": ms_per_iter, "groups": {},
           "nonfinite_problems": {m: int(np.sum(~np.all(np.isfinite(traces[m]), axis=0))) for m in traces}}
    for name, sel0 in groups.items():
        sel = sel0 & finite
        d = {m: traces[m][:, sel].sum(axis=1) for m in traces}
        D0 = d["joint"][0]
        Dend = max(d["joint"][-1], d["alternating"][-1])
        rows = {}
        for q in (0.9, 0.99, 0.999, 1.0):
            target = D0 - q * (D0 - Dend)
            row = {"target": float(target)}
            for m in d:
                hit = np.nonzero(d[m] <= target * (1 + 1e-12))[0]
                it = int(hit[0]) if hit.size else None
                row[m] = {"iterations": it, "ms": (it * ms_per_iter[m]) if it is not None else None}
            rows[str(q)] = row
        out["groups"][name] = {"problems": int(sel.sum()), "excluded_nonfinite": int((sel0 & ~finite).sum()),
                               "D0": float(D0),
                               "D_T": {m: float(d[m][-1]) for m in d}, "targets": rows}
    out["objective_increases"] = {m: int(np.sum(traces[m][1:, finite] > traces[m][:-1, finite] * (1 + 1e-12)))
                                  for m in traces}
    return out


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        return len(os.sched_getaffinity(0))


def _timed_oracle(fn, budget_s, threads=None):
    """Runs fn() repeatedly for about budget_s seconds (at least once), with the
    BLAS pool limited to `threads` when given; returns (calls, seconds, threads used)."""
    from contextlib import nullcontext
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(limits=threads) if threads else nullcontext()
    except Exception:  # pragma: no cover
        lim = nullcontext()
    with lim:
        used = _blas_threads()
        n = 0
        t0 = time.perf_counter()
        while True:
            fn()
            n += 1
            el = time.perf_counter() - t0
            if el >= budget_s:
                break
    return n, el, used


def cpu_baseline_batched(host, budget_s, gpu_value, kappa=0.0):
    """The FP64 oracle's joint iteration (objective + update + normalization) on a
    fixed random sample of 16 of the problems, timed with all host cores and with
    one thread (about budget_s / 2 seconds each), scaled to one iteration of the
    whole batch by the sample's share of sum(FNK)."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(0)
    idx = sorted(rng.choice(len(host), size=min(16, len(host)), replace=False).tolist())
    sample = [(host[i].V.astype(np.float64), host[i].W.astype(np.float64), host[i].H.astype(np.float64),
               host[i].beta) for i in idx]
    total = sum(q.V.shape[0] * q.V.shape[1] * q.W.shape[1] for q in host)
    share = sum(V.shape[0] * V.shape[1] * W.shape[1] for V, W, _, _ in sample) / total

    def sweep():
        for V, W, H, beta in sample:
            oracle.objective(V, W, H, beta, kappa=kappa)
            oracle.jmm_iteration(V, W, H, beta, kappa=kappa)

    n_all, el_all, th_all = _timed_oracle(sweep, budget_s / 2)
    n_one, el_one, _ = _timed_oracle(sweep, budget_s / 2, threads=1)
    v_all = share * n_all / el_all
    v_one = share * n_one / el_one
    desc = (f"problems {idx} of {len(host)} ({share * 100:.2f}% of sum FNK), one joint iteration each "
            f"(objective + update + normalization, float64 NumPy); {n_all} sweeps in {el_all:.1f} s on "
            f"{th_all} threads and {n_one} in {el_one:.1f} s on 1 thread; iterations/s of the whole batch "
            f"EXTRAPOLATED from the sample by its share of sum FNK")
    return {"value": v_all, "unit": "iterations/s (all problems per iteration, extrapolated)", "cores": th_all,
            "kind": "oracle", "sample": desc, "one_thread": {"value": v_one, "cores": 1},
            "cpu_model": cpu_model(), "host_cores_available": len(os.sched_getaffinity(0)),
            "gpu_over_cpu": gpu_value / v_all}


def cpu_baseline(p, budget_s, gpu_value):
    """The FP64 oracle's joint iteration (with the objective, as on the GPU) timed
    on the host cores from the benchmark's init, for about budget_s / 2 seconds
    with all threads and as long with one thread."""
    import numpy as np
    import oracle
    V = p.V.astype(np.float64)
    state = {"W": p.W.astype(np.float64), "H": p.H.astype(np.float64)}

    def one():
        oracle.objective(V, state["W"], state["H"], p.beta)
        state["W"], state["H"] = oracle.jmm_iteration(V, state["W"], state["H"], p.beta)

    n_all, el_all, th_all = _timed_oracle(one, budget_s / 2)
    state.update(W=p.W.astype(np.float64), H=p.H.astype(np.float64))
    n_one, el_one, _ = _timed_oracle(one, budget_s / 2, threads=1)
    return {"value": n_all / el_all, "unit": "iterations/s", "cores": th_all, "kind": "oracle",
            "sample": f"{n_all} joint iterations (objective + update + normalization, float64 NumPy) of the "
                      f"{p.name} workload from the benchmark's init in {el_all:.1f} s on {th_all} threads; "
                      f"{n_one} in {el_one:.1f} s on 1 thread",
            "one_thread": {"value": n_one / el_one, "cores": 1}, "cpu_model": cpu_model(),
            "host_cores_available": len(os.sched_getaffinity(0)), "gpu_over_cpu": gpu_value / (n_all / el_all)}


if __name__ == "__main__":
    sys.exit(main())
