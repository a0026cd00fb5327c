#!/usr/bin/env python3
"""Benchmark: Newton-Raphson power flows per second on one MI355X.

Default workload: the 1,350-bus synthetic meshed grid with 10,000 Monte Carlo scenarios,
plain FP64 Newton-Raphson from flat start, tolerance 1e-8 pu, at most 10 iterations.
One step = one pf_solve_batch over the whole batch (layout transform in, every Newton
iteration of every instance, layout transform out) with inputs resident in device memory.

Prints one JSON line with the throughput of converged flows, the roofline position of the
solver kernel (algorithmic bytes per launch / launch time, timed with events on the
launch stream) and the CPU oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c1": dict(key="c1", desc="1350-bus synthetic meshed grid (avg degree 2.8, 15% PV), 10,000 Monte "
                             "Carlo scenarios, NR from flat start, tol 1e-8 pu, max 10 iterations"),
    "c2": dict(key="c2", desc="9000-bus synthetic meshed grid (avg degree 2.6, 20% PV), 2,000 Monte "
                             "Carlo scenarios, NR from flat start, tol 1e-8 pu, max 10 iterations"),
    "c0": dict(key="c0", desc="14-bus synthetic meshed grid, 64 scenarios, NR from flat start, "
                             "tol 1e-8 pu, max 10 iterations"),
}


def algorithmic_bytes(info, iters: np.ndarray, precision_fp32: bool) -> float:
    """Compulsory HBM bytes of one launch: per Newton iteration of an instance
    4 b nnz_lu + 80 n + 32 N (mismatch, Jacobian, refactor, substitutions, update), plus
    the final mismatch 32 n + 8 N of every instance and the layout transform 48 n."""
    n, N = info["n_bus"], info["n_unknowns"]
    per_iter = info["bytes_iter_fp32"] if precision_fp32 else info["bytes_iter_fp64"]
    return float(iters.astype(np.int64).sum()) * per_iter + iters.shape[0] * (32 * n + 8 * N + 48 * n)


def cpu_baseline(g, yb, sc, tol, max_iter, target_s=15.0):
    import oracle
    osys = oracle.System.from_ybus(yb, g.bus_type)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    probe = min(64, sc.batch)
    t0 = time.perf_counter()
    osys.solve(sc.sbus[:probe], sc.v0[:probe], tol=tol, max_iter=max_iter, threads=cores)
    dt = max(time.perf_counter() - t0, 1e-4)
    count = int(min(sc.batch, max(probe, probe * target_s / dt)))
    t0 = time.perf_counter()
    r = osys.solve(sc.sbus[:count], sc.v0[:count], tol=tol, max_iter=max_iter, threads=cores)
    dt = time.perf_counter() - t0
    return {"value": float(r.converged.sum() / dt), "unit": "flows/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"first {count} of the {sc.batch} scenarios, FP64 oracle (own minimum-degree "
                      f"order, pivoting left-looking LU), {cores} threads, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c1", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32lu"])
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--count", type=int, default=0, help="cap the scenario count (testing only)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver shards over instances with no "
              "communication, so a multi-GPU figure is not part of this benchmark", file=sys.stderr)
        sys.exit(2)

    import torch
    import gridgen as gg
    import paper_2101_02270_amd as pf

    wl = WORKLOADS[args.workload]
    (g, yb, sc), = gg.workload(wl["key"], count=args.count or None)
    tol, max_iter = 1e-8, 10
    fp32 = args.precision == "fp32lu"
    prec = pf.PF_FP32_LU if fp32 else pf.PF_FP64
    print(f"[bench] workload {args.workload}: n={g.n} batch={sc.batch} precision={args.precision}",
          file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    plan = pf.Plan.from_ybus(yb, g.bus_type)
    analyze_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info

    dev = torch.device("cuda", 0)
    y = torch.from_numpy(yb.val).to(dev)
    s = torch.from_numpy(np.ascontiguousarray(sc.sbus)).to(dev)
    v0 = torch.from_numpy(np.ascontiguousarray(sc.v0)).to(dev)
    B = sc.batch
    out = pf.Result(v=torch.empty((B, g.n, 2), dtype=torch.float64, device=dev),
                    iters=torch.empty(B, dtype=torch.int32, device=dev),
                    converged=torch.empty(B, dtype=torch.uint8, device=dev),
                    status=torch.empty(B, dtype=torch.int8, device=dev))
    ws = torch.empty(plan.workspace_bytes(B, prec, args.tile, args.waves) + 256, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        pf.solve_batch(plan, y, s, v0, tol=tol, max_iter=max_iter, precision=prec, tile=args.tile,
                       waves=args.waves, workspace=ws, stream=stream, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        step()
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(starts, ends)]))
    print(f"[bench] timed {args.steps} steps in {wall:.3f} s", file=sys.stderr, flush=True)

    iters = out.iters.cpu().numpy()
    conv = out.converged.cpu().numpy().astype(bool)
    n_conv = int(conv.sum())
    ms_per_step = wall * 1e3 / args.steps
    value = n_conv * args.steps / wall

    abytes = algorithmic_bytes(info, iters, fp32)
    achieved = abytes / (kernel_ms * 1e-3) / 1e9
    res = {
        "metric": "NR power flows/sec to 1e-8 pu (FP64 vs FP32-LU+warm start), 1 GPU",
        "value": round(value, 1),
        "unit": "flows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "batch": B, "n_bus": g.n, "precision": args.precision,
                   "start": "flat", "tol": tol, "max_iter": max_iter},
        "converged_fraction": round(n_conv / B, 5),
        "iterations_mean": round(float(iters[conv].mean()) if n_conv else 0.0, 4),
        "analyze_ms": round(analyze_ms, 2),
        "plan": {k: info[k] for k in ("n_unknowns", "nnz_lu", "n_levels", "flops_refactor", "max_col")},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "nr_tile_kernel", "kernel_ms": round(kernel_ms, 4),
                     "algorithmic_bytes_per_launch": abytes},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(g, yb, sc, tol, max_iter)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
