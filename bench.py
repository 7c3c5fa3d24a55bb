#!/usr/bin/env python3
"""Benchmark of the sLLG Heun step on one MI355X.

Workload: the 200x200x33 simple-cubic granular slab (1.32M sites, Voronoi
8 nm grains with 1 nm non-magnetic boundaries, 800 K Gaussian laser spot
moving at 10 m/s over 300 K, -0.8 T write field), seeded synthetic input.
A step is one full Heun step of every site (spot temperature, Philox noise,
Box-Muller, exchange, anisotropy, Zeeman, predictor, corrector).

Prints one JSON line: spin-updates/s (magnetic sites x steps / s) with the
roofline of the dominant kernel (algorithmic bytes per launch / its average
duration from HIP events on the handle's stream) and the FP64 CPU oracle
timed on a bounded sample.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--kernel", choices=["auto", "plain", "fused"], default="auto")
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=0, help="oracle steps (0: auto ~15 s)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device copy of known size (HBM counter calibration)")
    return ap.parse_args()


def bytes_per_site(precision: str, kernel: str) -> int:
    """Algorithmic HBM bytes per lattice site and step: read S once, write S once."""
    e = 8 if precision == "fp64" else 4
    return 2 * 3 * e


def time_steps(torch, h, k):
    """Whole-job time of k steps on the handle's stream (events + synchronize)."""
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(h.stream)
    h.step(k)
    stop.record(h.stream)
    stop.synchronize()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3


def kernel_duration(torch, h, k):
    """Average duration of one step launch: events recorded on the handle's
    stream around each eager step launch."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(k)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record(h.stream)
        h.step(1)
        b.record(h.stream)
    torch.cuda.synchronize()
    d = np.array([a.elapsed_time(b) for a, b in evs]) / 1e3
    return float(np.median(d)), float(np.mean(d))


def gpu_run(args, precision_name, kernel_name, steps, warmup, graph_steps):
    import torch
    import workloads as W
    from paper_2502_02236_amd import asd as A
    from paper_2502_02236_amd import bridge

    prec = A.ASD_FP32 if precision_name == "fp32" else A.ASD_FP64
    kern = {"auto": A.ASD_KERNEL_AUTO, "plain": A.ASD_KERNEL_PLAIN,
            "fused": A.ASD_KERNEL_FUSED}[kernel_name]
    w = W.c2_granular_slab()
    h = bridge.make_handle(w, prec, kernel=A.ASD_KERNEL_PLAIN, graph_steps=graph_steps)
    lab = h.labels()
    S0 = W.initial_spins(len(lab), w.seed + 100)
    S0[:, lab < 0] = 0
    h.set_spins(S0)
    if kern == A.ASD_KERNEL_AUTO:
        os.makedirs(os.path.join(ROOT, "_build"), exist_ok=True)
        h.autotune(os.path.join(ROOT, "_build", "asd_tune.json"))
        h.set_spins(S0)
        h.set_step(0)
    elif kern == A.ASD_KERNEL_FUSED:
        h.set_variant(A.ASD_KERNEL_FUSED, max(args.tile, 0))
    elif args.tile >= 0:
        h.set_variant(A.ASD_KERNEL_PLAIN, args.tile)
    kernel_used, tile_used = h.variant()
    n_mag = int((lab >= 0).sum())
    n_sites = len(lab)
    h.step(warmup)
    torch.cuda.synchronize()
    t = time_steps(torch, h, steps)
    med, mean = kernel_duration(torch, h, min(200, steps))
    S = h.get_spins().astype(np.float64)
    norm_err = float(np.max(np.abs(np.sqrt((S[:, lab >= 0] ** 2).sum(0)) - 1)))
    h.close()
    return dict(w=w, t=t, n_mag=n_mag, n_sites=n_sites, steps=steps, kernel=kernel_used,
                tile=tile_used, step_med=med, step_mean=mean, norm_err=norm_err)


def cpu_baseline(target_s=15.0, steps=0):
    """The FP64 oracle, single-threaded plain C, on the full lattice for a few steps."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import workloads as W
    from oracle_build import oracle_labels, oracle_system

    w = W.c2_granular_slab()
    lab = oracle_labels(w)
    sysm = oracle_system(w, labels=lab)
    S = W.initial_spins(len(lab), w.seed + 100)
    S[:, lab < 0] = 0
    t0 = time.perf_counter()
    S = sysm.heun(S, 0, 1)
    one = time.perf_counter() - t0
    k = steps if steps > 0 else max(2, int(target_s / max(one, 1e-3)))
    t0 = time.perf_counter()
    sysm.heun(S, 1, k)
    dt = time.perf_counter() - t0
    n_mag = int((lab >= 0).sum())
    return dict(value=n_mag * k / dt, unit="spin-updates/s", cores=1, kind="oracle",
                sample=f"full 200x200x33 slab, {k} Heun steps (steps 1..{k}), FP64, "
                       f"single-threaded plain C, {dt:.1f} s")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are "
                                   "not part of this build (see DESIGN.md: sharding)"}))
        sys.exit(2)
    r = gpu_run(args, args.precision, args.kernel, args.steps, args.warmup, args.graph_steps)
    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    value = r["n_mag"] * r["steps"] / r["t"]
    bps = bytes_per_site(args.precision, "fused" if r["kernel"] == 2 else "plain")
    alg_bytes = bps * r["n_sites"]
    achieved = alg_bytes / r["step_mean"] / 1e9
    out = {
        "metric": "atomistic spin-updates/s (spins x Heun steps)",
        "value": value,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["t"] / r["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": r["w"].name, "lattice": "sc", "sites": r["n_sites"],
                   "magnetic_sites": r["n_mag"], "dt_fs": 1.0, "precision": args.precision,
                   "kernel": {1: "plain", 2: "fused"}.get(r["kernel"], "?"), "tile": r["tile"],
                   "graph_steps": args.graph_steps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "heun step (predictor + corrector kernels)" if r["kernel"] != 2
                     else "k_fused_sc", "bytes_per_site": bps,
                     "step_ms_mean": 1e3 * r["step_mean"], "step_ms_median": 1e3 * r["step_med"]},
        "max_norm_error": r["norm_err"],
    }
    if not args.no_fp64_compare and args.precision == "fp32":
        r64 = gpu_run(args, "fp64", "plain", max(200, args.steps // 10), 20, 0)
        v64 = r64["n_mag"] * r64["steps"] / r64["t"]
        out["fp64_plain_value"] = v64
        out["speedup_vs_fp64_plain"] = value / v64
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(steps=args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
