#!/usr/bin/env python3
"""Benchmark of the sLLG Heun step on one MI355X.

Default workload (--workload track): the moving-window recording batch, 16
seeds of a 400x200x33 simple-cubic window (120x60x10 nm at a = 0.3 nm) in
800-column tracks, each seed with its own Voronoi grain map (8 nm grains, 1 nm
non-magnetic boundaries) and a 5 % per-grain anisotropy spread, an 800 K
Gaussian laser spot locked to the window, a +-0.8 T write field carrying
20 nm bits at 20 m/s, FP32, 42.2M lattice sites in one launch per step;
seeded synthetic input.  A step is one full Heun step of every window site
(spot temperature, Philox noise, Box-Muller, exchange, anisotropy, Zeeman,
predictor, corrector); the window shifts by one column every 15 000 steps.
The timed steps run as HIP-graph segments (the largest even divisor of
--steps up to 1000 steps, so exactly --steps steps are timed).

Other workloads: slab (the 200x200x33 granular slab, cache-resident), l10
(L1_0 Fe sublattice window, four shells, 2.19M sites), cylinders (512 isolated
grains of uneven size, each at its own temperature, moment statistics every 10
steps), and the rows beyond the step (transfer, demag, mc, mm, multiscale).

Prints one JSON line: spin-updates/s (magnetic sites x steps / s) with the
roofline of the dominant kernel (algorithmic bytes or VALU work per launch / its
average duration from HIP events on the handle's stream; the bound is whichever
of the two takes longer at its peak, and the other is reported beside it),
the same step on other lattices and precisions, and the FP64 CPU oracle timed
on a cropped window of the same workload.
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
# VALU issue rate: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz non-packed FP32 FMAs
# per second (the published 157.3 TFLOP/s FP32 vector peak, two flops per FMA).
# An FP32 add, multiply or 32-bit integer operation costs one such slot; the
# other classes the step uses are weighed by their issue cost relative to the
# FMA, as measured by `bench.py --issue-rates` on the MI355X:
VALU_PEAK_T = 256 * 4 * 32 * 2.4e9 / 1e12
W_PRODUCT = 1.56  # v_mad_u64_u32: the 32 x 32 -> 64 product of a Philox round
W_TRANS = 2.75    # v_log_f32, v_rsq_f32 (and the other transcendentals)


TUNE_CACHE = os.path.join(ROOT, "paper_2502_02236_amd", "tune_mi355x.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--workload", choices=["slab", "l10", "cylinders", "track", "transfer",
                                           "demag", "track_demag", "mc", "mm", "multiscale"],
                    default="track")
    ap.add_argument("--demag-cell", type=int, nargs=3, default=[4, 4, 3],
                    help="coarse cell of the demag and track_demag workloads, in lattice cells")
    ap.add_argument("--demag-once", action="store_true",
                    help="demag and track_demag workloads: the field evaluated once per step and "
                         "held through both Heun stages (default: at both stages)")
    ap.add_argument("--window-demag", action="store_true",
                    help="multiscale workload: add the demagnetising field of the whole window "
                         "(regions and atoms as one mesh)")
    ap.add_argument("--kernel", choices=["auto", "plain", "fused"], default="auto")
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--graph-steps", type=int, default=-1,
                    help="steps per HIP-graph segment (-1: the largest even divisor of "
                         "--steps up to 1000; 0: eager launches)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotuner cache (the tile picks measured on MI355X)")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other lattices and precisions beside the headline")
    ap.add_argument("--cpu-steps", type=int, default=1000, help="oracle steps per CPU process")
    ap.add_argument("--cpu-worker", type=int, default=-1, help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device copy of known size (HBM counter calibration)")
    ap.add_argument("--issue-rates", action="store_true",
                    help="only measure the VALU issue cost of the instruction classes the "
                         "cost model weighs, and print them")
    return ap.parse_args()


def segment_steps(steps: int, cap: int = 1000) -> int:
    """Steps per graph segment: the largest even divisor of `steps` (of steps - 1
    when odd) not above `cap`; 0 when there is none (eager launches)."""
    n = steps if steps % 2 == 0 else steps - 1
    best = 0
    for g in range(2, min(cap, n) + 1, 2):
        if n % g == 0:
            best = g
    return best


def issue_rates():
    """SIMD cycles per wave64 instruction of each calibrated class (independent
    chains, 32 waves per SIMD, nominal 2.4 GHz clock), and its weight relative
    to a non-packed FP32 FMA."""
    import ctypes

    import torch
    from paper_2502_02236_amd import build as B
    # a measurement-only probe, not part of libasd: built here on demand
    src = os.path.join(ROOT, "tests", "helpers", "issue_rate.hip")
    lib = ctypes.CDLL(B.build_probe(src, os.path.join(ROOT, "_build", "libissue_rate.so")))
    lib.issue_rate_name.restype = ctypes.c_char_p
    lib.issue_rate_time.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_float)]
    blocks, iters, simds = 256 * 32, 4096, 256 * 4
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    waves = blocks * 256 / 64
    res = {}
    for k in range(lib.issue_rate_classes()):
        ms = ctypes.c_float()
        rc = lib.issue_rate_time(k, ctypes.c_void_p(out.data_ptr()), blocks, iters, ctypes.byref(ms))
        if rc:
            raise RuntimeError(f"issue_rate_time({k}) returned {rc}")
        instr = waves * iters * lib.issue_rate_chains()
        res[lib.issue_rate_name(k).decode()] = ms.value * 1e-3 * 2.4e9 * simds / instr
    base = res["v_fma_f32"]
    return {name: {"cycles_per_wave64_instruction": c, "fma_f32_equivalents": c / base}
            for name, c in res.items()}


def bytes_per_site(precision: str, workload: str, kernel_name: str) -> int:
    """Algorithmic HBM bytes per lattice site and step: read S once, write S once
    (+2 B grain label where k_u varies per grain; +72 B of neighbour indices when
    the L1_0 two-pass kernels read the neighbour table)."""
    e = 8 if precision == "fp64" else 4
    b = 2 * 3 * e
    if workload in ("track", "track_demag"):
        b += 2
    if workload == "l10" and not kernel_name.startswith("k_fused"):
        b += 4 * 18
    return b


def alu_ops_per_site(precision: str, workload: str):
    """Algorithmic VALU work per magnetic site and Heun step of the FP32 path
    (nothing recomputed, no halo), in FP32-FMA issue slots.  Operations:
    Philox4x32-10 40 (20 32 x 32 -> 64 products, 20 three-way xors), uniforms
    8, Box-Muller radii 6 and angles 3, scaling 3; per stage exchange 18 (SC) or
    54 (L1_0, four shells), field assembly 4 (+3 once), LL right-hand side 18;
    predictor update 10, corrector update 13: 166 operations for SC (238 for
    L1_0), of which 20 products (weight W_PRODUCT) and 9 transcendentals
    (weight W_TRANS): 192.95 slots for SC, 264.95 for L1_0.  None for FP64
    (software transcendentals; reported against HBM)."""
    if precision != "fp32":
        return None
    ops = 166 + (2 * (54 - 18) if workload == "l10" else 0)
    return round(ops - 20 - 9 + 20 * W_PRODUCT + 9 * W_TRANS, 6)


def kernel_sources_hash():
    """Hash of the step kernels' source code: the files the step kernels are
    compiled from, with comments and blank space removed (a comment edit does
    not change the kernels, so it does not retire the committed counters)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("asd_device.h", "asd_step.inc", "asd_fused.inc", "asd_fused_l10.inc", "asd_variants.h",
              "asd_internal.h"):
        with open(os.path.join(ROOT, "paper_2502_02236_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name, workload, precision, tile):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE summary, if it was
    taken on this kernel variant, workload and precision with the current kernel sources."""
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", "*traffic*.json")):
        with open(path) as f:
            t = json.load(f)
        if (t.get("kernel", "").split("(")[0].replace("void asd::", "") == kernel_name
                and t.get("workload") == workload and t.get("precision") == precision
                and t.get("tile") == tile and t.get("source_hash") == kernel_sources_hash()):
            return t["traffic_bytes"], os.path.basename(path)
    return None, None


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


def build_workload(name, prec, graph_steps, demag_cell=(0, 0, 0)):
    """Handle + per-system initial spins + window-magnetic count for a workload."""
    import workloads as W
    from paper_2502_02236_amd import asd as A
    from paper_2502_02236_amd import bridge

    extra = {}
    if name in ("slab", "l10", "demag"):
        w = W.c3_l10_window() if name == "l10" else W.c2_granular_slab()
        h = bridge.make_handle(w, prec, kernel=A.ASD_KERNEL_PLAIN, graph_steps=graph_steps,
                               demag_cell=tuple(demag_cell) if name == "demag" else (0, 0, 0))
        labs = [h.labels()]
        window = [np.ones(len(labs[0]), bool)]
    elif name == "cylinders":
        cyl = W.cylinder_batch(n=512)
        w = W.Workload("cylinders512_d5-12nm_h8-12nm_T300-900K", bc=(0, 0, 0),
                       B=(0.0, 0.0, 0.0), seed=4)
        ins = [bridge.SystemInputs(w.scaled(nx=c.nx, ny=c.ny, nz=c.nz), labels=c.labels,
                                   T_system=c.T) for c in cyl]
        h = A.Handle(bridge.params_for(w, prec, graph_steps=graph_steps), [i.desc for i in ins])
        dr, _ = bridge.drive_for(w, T_amb=0.0)
        h.set_drive(dr)
        h._inputs = ins
        labs = [c.labels for c in cyl]
        window = [np.ones(len(l), bool) for l in labs]
        extra["moments_every"] = 10
    else:  # track (track_demag: with the window's demagnetising field and the track's stray field)
        n_seeds = 16
        w = W.c5_track_window()
        ins = []
        for k in range(n_seeds):
            wk = w.scaled(seed=w.seed + k)
            seeds = W.voronoi_seeds(wk)
            ku = W.grain_ku(len(seeds), w.ku, w.ku_spread, wk.seed)
            ins.append(bridge.SystemInputs(wk, seeds=seeds, ku_grain=ku))
        cell = tuple(demag_cell) if name == "track_demag" else (0, 0, 0)
        h = A.Handle(bridge.params_for(w, prec, graph_steps=graph_steps, demag_cell=cell),
                     [i.desc for i in ins])
        dr, bits = bridge.drive_for(w)
        h.set_drive(dr)
        h._inputs = (ins, bits)
        labs = [h.labels(k) for k in range(n_seeds)]
        xs = np.arange(len(labs[0])) % w.track_nx
        window = [(xs < w.nx)] * n_seeds
        extra["shift_every"] = W.steps_per_column(w)
    S0s = []
    for k, lab in enumerate(labs):
        S0 = W.initial_spins(len(lab), w.seed + 100 + k)
        S0[:, lab < 0] = 0
        S0s.append(S0)
        h.set_spins(S0, k)
    n_mag = int(sum(((l >= 0) & m).sum() for l, m in zip(labs, window)))
    n_sites = int(sum(m.sum() for m in window))
    return w, h, S0s, n_mag, n_sites, extra


def run_steps(h, k, extra, done):
    """k steps of the workload (moment samples / window shifts where it has them)."""
    me = extra.get("moments_every", 0)
    se = extra.get("shift_every", 0)
    every = me or se
    if not every:
        h.step(k)
        return
    t = 0
    while t < k:
        nxt = min(k - t, every - (done + t) % every)
        h.step(nxt)
        t += nxt
        if (done + t) % every == 0:
            if me:
                h.accumulate_moments(reset=(done + t) == me)
            else:
                h.shift_window(1)


RAMP_S = 0.3


def clock_ramp(torch, h, S0s, graph_steps, seconds=RAMP_S):
    """Untimed set-up: step the handle for about `seconds` so that the GPU
    reaches its sustained clocks (a cold GPU runs the first milliseconds of
    steps ~5-15 % slower), then put back the initial spins (device copies) and
    step 0.  The warm-up and timed steps that follow start from the same state
    as without it.  Returns the seconds spent."""
    dev = [torch.from_numpy(np.ascontiguousarray(S0, dtype=h.dtype)).to(h.device) for S0 in S0s]
    seg = graph_steps if graph_steps > 0 else 100
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        h.step(seg)
        h.stream.synchronize()
    for k, S in enumerate(dev):
        h.set_spins(S, k)
    h.set_step(0)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def gpu_run(args, precision_name, kernel_name, steps, warmup, graph_steps, workload=None,
            tile=None, demag_once=None):
    import torch
    from paper_2502_02236_amd import asd as A

    prec = A.ASD_FP32 if precision_name == "fp32" else A.ASD_FP64
    kern = {"auto": A.ASD_KERNEL_AUTO, "plain": A.ASD_KERNEL_PLAIN,
            "fused": A.ASD_KERNEL_FUSED}[kernel_name]
    workload = workload or args.workload
    tile = args.tile if tile is None else tile
    w, h, S0s, n_mag, n_sites, extra = build_workload(workload, prec, graph_steps,
                                                      args.demag_cell)
    once = args.demag_once if demag_once is None else demag_once
    if workload in ("demag", "track_demag") and once:
        h.set_demag_reading(A.ASD_DEMAG_ONCE)
    if kern == A.ASD_KERNEL_AUTO:
        os.makedirs(os.path.join(ROOT, "_build"), exist_ok=True)
        cache = (os.path.join(ROOT, "_build", "asd_tune_fresh.json") if args.retune
                 else args.tune_cache)
        h.autotune(cache)
        for k, S0 in enumerate(S0s):
            h.set_spins(S0, k)
        h.set_step(0)
    elif kern == A.ASD_KERNEL_FUSED:
        h.set_variant(A.ASD_KERNEL_FUSED, max(tile, 0))
    elif tile >= 0:
        h.set_variant(A.ASD_KERNEL_PLAIN, tile)
    kernel_used, tile_used = h.variant()
    kname = h.variant_name()
    h.prepare()  # capture the step graphs before the warm-up (untimed)
    ramp_s = clock_ramp(torch, h, S0s, graph_steps)
    run_steps(h, warmup, extra, 0)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(h.stream)
    run_steps(h, steps, extra, warmup)
    stop.record(h.stream)
    stop.synchronize()
    torch.cuda.synchronize()
    t = start.elapsed_time(stop) / 1e3
    med, mean = kernel_duration(torch, h, min(200, steps))
    S = h.get_spins(0).astype(np.float64)
    mag = np.abs(S).sum(0) > 0
    norm_err = float(np.max(np.abs(np.sqrt((S[:, mag] ** 2).sum(0)) - 1)))
    h.close()
    return dict(w=w, t=t, n_mag=n_mag, n_sites=n_sites, steps=steps, kernel=kernel_used, ramp_s=ramp_s,
                tile=tile_used, step_med=med, step_mean=mean, norm_err=norm_err, kname=kname,
                graph_steps=graph_steps, workload=workload, precision=precision_name,
                eager_steps=steps - (steps // graph_steps) * graph_steps if graph_steps else steps)


def step_roofline(r):
    """Roofline of the step kernel of a gpu_run result: algorithmic bytes and (FP32)
    VALU work per launch over the average launch duration in the timed region."""
    precision, workload = r["precision"], r["workload"]
    bps = bytes_per_site(precision, workload, r["kname"])
    alg_bytes = bps * r["n_sites"]
    # average launch duration of the step kernel over the timed region (kernels
    # back to back on the handle's stream; includes the gaps between them)
    launch_s = r["t"] / r["steps"]
    achieved = alg_bytes / launch_s / 1e9
    traffic, traffic_src = measured_traffic(r["kname"], workload, precision, r["tile"])
    hbm = {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "bytes_per_site": bps,
           "algorithmic_bytes_per_launch": alg_bytes}
    roof = dict(bound="hbm", **hbm)
    cyc = alu_ops_per_site(precision, workload)
    if cyc is not None:
        # the bound is whichever of the algorithmic HBM bytes and VALU work takes
        # longer at its peak; the other roofline is reported beside it
        alu_ops = cyc * r["n_mag"]
        alu_ach = alu_ops / launch_s / 1e12
        alu = {"achieved": alu_ach, "peak": VALU_PEAK_T, "unit": "T FP32-FMA slots/s",
               "frac": alu_ach / VALU_PEAK_T, "alu_ops_per_magnetic_site": cyc,
               "alu_ops_per_launch": alu_ops}
        if alu_ops / (VALU_PEAK_T * 1e12) > alg_bytes / (HBM_PEAK_GBS * 1e9):
            roof = dict(bound="alu", **alu)
            roof["hbm"] = hbm
        else:
            roof["alu"] = alu
    roof.update({"traffic": traffic, "traffic_source": traffic_src, "kernel": r["kname"],
                 "launch_us_mean": 1e6 * launch_s,
                 "launch_us_eager_events_median": 1e6 * r["step_med"]})
    return roof


def step_summary(r, **extra):
    """One workload beside the headline: rate, step time and roofline fractions."""
    roof = step_roofline(r)
    out = {"workload": r["w"].name, "precision": r["precision"],
           "kernel": {1: "plain", 2: "fused"}.get(r["kernel"], "?"), "tile": r["tile"],
           "kernel_name": r["kname"], "steps": r["steps"], "graph_steps": r["graph_steps"],
           "value": r["n_mag"] * r["steps"] / r["t"], "unit": "spin-updates/s",
           "ms_per_step": 1e3 * r["t"] / r["steps"], "sites": r["n_sites"],
           "magnetic_sites": r["n_mag"], "bound": roof["bound"], "frac": roof["frac"],
           "hbm_frac": roof["hbm"]["frac"] if "hbm" in roof else roof["frac"]}
    if "alu" in roof:
        out["alu_frac"] = roof["alu"]["frac"]
    elif roof["bound"] == "alu":
        out["alu_frac"] = roof["frac"]
    out.update(extra)
    return out


def transfer_run(args, cell=7, reps=20):
    """Window-end transfer (Eq. 6 both ways) over the 16-seed track: every
    stored column of every system coarse-grained into cells of cell^3
    lattice cells, then every window column thermalised from a coarse field.
    Times `reps` rounds with HIP events on the handle's stream."""
    import ctypes as C
    import torch
    from paper_2502_02236_amd import asd as A

    prec = A.ASD_FP32 if args.precision == "fp32" else A.ASD_FP64
    w, h, S0s, n_mag, n_sites, extra = build_workload("track", prec, 0)
    L = A.lib()
    n_sys = len(S0s)
    sx = w.track_nx
    ncell = h.coarse_cells(0, sx, cell, cell, cell)
    out = torch.empty((n_sys, ncell, 4), dtype=torch.float64, device=h.device)
    nwc = h.coarse_cells(0, w.nx, cell, cell, cell)
    mc = torch.zeros((nwc, 3), dtype=torch.float64, device=h.device)
    mc[:, 2] = 0.8
    torch.cuda.synchronize()

    def coarse():
        for s in range(n_sys):
            A._check(L.asd_coarse_grain(h.h, s, 0, sx, cell, cell, cell, out[s].data_ptr()), h.h)

    def cone():
        for s in range(n_sys):
            A._check(L.asd_thermalise_columns(h.h, s, 0, w.nx, cell, cell, cell, mc.data_ptr(),
                                              C.c_uint32(7)), h.h)

    res = {}
    for name, fn in (("coarse_grain", coarse), ("thermalise", cone)):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(h.stream)
        for _ in range(reps):
            fn()
        e1.record(h.stream)
        e1.synchronize()
        res[name] = e0.elapsed_time(e1) / 1e3 / reps  # s per round (n_sys launches)
    sites_cg = n_sys * sx * w.ny * w.nz
    sites_th = n_sys * w.nx * w.ny * w.nz
    e = 4 if prec == A.ASD_FP32 else 8
    cg_bytes = sites_cg * (3 * e + 2)       # spins + label read once
    th_bytes = sites_th * (2 * 3 * e + 2)   # label read, both buffers written
    h.close()
    return dict(w=w, res=res, sites_cg=sites_cg, sites_th=sites_th, cg_bytes=cg_bytes,
                th_bytes=th_bytes, e=e, cell=cell, reps=reps)


MM_ALU_PER_STAGE = 66


def mm_run(args):
    """Micromagnetic window of the paper's multiscale runs (Sec. III): 300 x 60 x 16 nm
    in 1 x 1 x 2 nm cells (300 x 60 x 8), SC parameters (Ms0 5.2e5 A/m, K0 2.2e6 J/m^3,
    A0 = J / 2a with J = 6.8e-21 J, a = 0.5 nm, lambda 0.1, T_C 710 K), RK4 at
    dt = 20 fs, 800 K spot locked to the window, write field 0.8 T with 20 nm bits.
    Algorithmic VALU operations per cell and RK4 stage: Laplacian 36, field 7,
    Landau-Lifshitz right-hand side 15, stage update 8: 66."""
    import torch
    from paper_2502_02236_amd import asd as A

    prec = A.ASD_FP32 if args.precision == "fp32" else A.ASD_FP64
    a, J = 0.5e-9, 6.8e-21
    p = A.asd_mm_params()
    p.precision = prec
    p.nx, p.ny, p.nz = 300, 60, 8
    p.bc_x = p.bc_y = p.bc_z = A.ASD_BC_OPEN
    p.h[0], p.h[1], p.h[2] = 1e-9, 1e-9, 2e-9
    p.Ms0, p.A0, p.K0, p.lambda_, p.gamma = 5.2e5, J / (2 * a), 2.2e6, 0.1, 1.76e11
    p.Tc, p.mu_s, p.dt, p.graph_steps = 710.0, 5.2e5 * a ** 3, 20e-15, 100
    g = A.MMHandle(p)
    d = A.asd_drive()
    d.B[2] = 0.8
    bits = np.ascontiguousarray([int(b) for b in "0010111100101101100100001"], dtype=np.uint8)
    d.n_bits = len(bits)
    d.bits = bits.ctypes.data_as(A.C.POINTER(A.C.c_uint8))
    d.steps_per_bit = int(round(20e-9 / (20.0 * p.dt)))
    d.spot_mode = A.ASD_SPOT_LOCKED
    d.T_amb, d.T_peak, d.fwhm, d.x0, d.y0 = 300.0, 800.0, 40e-9, 150e-9, 30e-9
    g.set_drive(d)
    g.step(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(g.stream)
    g.step(args.steps)
    e1.record(g.stream)
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3
    m = g.get_m().astype(np.float64)
    g.close()
    return dict(t=t, n=300 * 60 * 8, mz=float(m[2].mean()))


def multiscale_run(args):
    """The paper's multiscale window (Sec. III): 100 nm of SC atoms (334 x 200 x 33 at
    a = 0.3 nm, 60 x 10 nm cross-section, Voronoi grains) between two 100 nm
    micromagnetic regions of 4 x 4 x 3 lattice cells (84 x 50 x 11 cells each),
    exchange-coupled through their faces, 800 K spot locked to the atomistic window,
    dt = 1 fs for both (one RK4 step per Heun step)."""
    import torch
    import workloads as W
    from paper_2502_02236_amd import asd as A
    from paper_2502_02236_amd import bridge

    prec = A.ASD_FP32 if args.precision == "fp32" else A.ASD_FP64
    cell = (4, 4, 3)
    # with the window's demagnetising field the atoms fill whole coarse cells
    nxa = 336 if args.window_demag else 334
    w = W.c5_track_window().scaled(nx=nxa, track_nx=nxa + 2 * cell[0], ku_spread=0.0,
                                   x0=50e-9, y0=30e-9)
    h = bridge.make_handle(w, prec, kernel=A.ASD_KERNEL_AUTO,
                           demag_cell=cell if args.window_demag else (0, 0, 0))
    h.shift_window(cell[0])
    a = w.a
    regions = []
    for _ in range(2):
        p = A.asd_mm_params()
        p.precision = prec
        p.nx, p.ny, p.nz = 84, -(-w.ny // cell[1]), -(-w.nz // cell[2])
        p.bc_x = p.bc_y = p.bc_z = A.ASD_BC_OPEN
        for k in range(3):
            p.h[k] = cell[k] * a
        p.Ms0, p.A0, p.K0 = w.mu_s / a ** 3, w.J[0] / (2 * a), w.ku / a ** 3
        p.lambda_, p.gamma, p.Tc, p.mu_s, p.dt = w.alpha, w.gamma, 710.0, w.mu_s, w.dt
        g = A.MMHandle(p, stream=h.stream)
        d = A.asd_drive()
        d.B[2] = 0.8
        d.T_amb = 300.0
        g.set_drive(d)
        regions.append(g)
    n_atoms = int((h.labels() >= 0).sum() * nxa / w.track_nx)
    msd = A.MultiscaleDemag(h, 0, regions[0], regions[1], cell) if args.window_demag else None

    def steps(n):
        if msd is not None:
            msd.step(n)
        else:
            A.multiscale_step(h, 0, regions[0], regions[1], cell, n)

    steps(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(h.stream)
    steps(args.steps)
    e1.record(h.stream)
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3
    kname = h.variant_name()
    if msd is not None:
        msd.close()
    for g in regions:
        g.close()
    h.close()
    return dict(t=t, n_atoms=n_atoms, n_cells=2 * 84 * 50 * 11, kernel=kname, name=w.name)


# 89 operations: 20 products, 4 transcendentals, 65 others
MC_ALU_OPS = round(65 + 20 * W_PRODUCT + 4 * W_TRANS, 6)


def mc_run(args):
    """Metropolis sweeps of the 200x200x33 granular slab at its 300 K ambient
    temperature (the exchange calibration of Sec. III with Eq. 8), timed with HIP
    events on the handle's stream.  Algorithmic VALU operations per visited
    magnetic site: Philox4x32-10 40 (20 products), uniforms 6, trial S_z and
    radius 2 + a square root, azimuth sine and cosine 2 + 2 transcendentals,
    exchange sum and scale 18, local field 3, energy change 11, Boltzmann factor
    and test 3 + an exponential: 89, weighed as in alu_ops_per_site: 107.2
    FP32-FMA slots."""
    import torch
    from paper_2502_02236_amd import asd as A

    prec = A.ASD_FP32 if args.precision == "fp32" else A.ASD_FP64
    w, h, S0s, n_mag, n_sites, extra = build_workload("slab", prec, 0)
    h.mc_sweep(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(h.stream)
    h.mc_sweep(args.steps)
    e1.record(h.stream)
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3
    S = h.get_spins(0).astype(np.float64)
    mz = float(S[2].sum() / n_mag)
    h.close()
    return dict(w=w, t=t, n_mag=n_mag, n_sites=n_sites, mz=mz)


def cpu_crop(k: int = 0):
    """The track workload cropped for the CPU oracle: a 64x64x33 window at the
    start of a 128-column track (the same lattice, grains of the same size law,
    per-grain anisotropy spread, window-locked 800 K spot centred in the crop,
    20 nm bits); seed k of the batch."""
    import workloads as W
    w = W.c5_track_window()
    c = w.scaled(nx=64, ny=64, nz=33, track_nx=128, x0=32 * w.a, y0=32 * w.a, seed=w.seed + k)
    return c


def cpu_worker(k: int, steps: int) -> dict:
    """One oracle run of the cropped track window (seed k, system id k):
    `steps` Heun steps from the seeded initial spins; returns the magnetic
    spin-updates and the seconds the steps took."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import workloads as W
    from oracle_build import oracle_labels, oracle_system, window_mask

    w = cpu_crop(k)
    seeds = W.voronoi_seeds(w)
    lab = oracle_labels(w, seeds=seeds)
    ku = W.grain_ku(len(seeds), w.ku, w.ku_spread, w.seed)
    win = window_mask(w, 0)
    sysm = oracle_system(w, labels=lab, ku_grain=ku, sys_id=k, active=win, origin=0)
    S = W.initial_spins(len(lab), w.seed + 100)
    S[:, lab < 0] = 0
    t0 = time.perf_counter()
    sysm.heun(S, 0, steps)
    dt = time.perf_counter() - t0
    n_mag = int(((lab >= 0) & (win > 0)).sum())
    return {"updates": n_mag * steps, "seconds": dt, "magnetic_sites": n_mag}


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline(steps: int = 1000):
    """The FP64 oracle (single-threaded plain C, as it stands) on the GPU machine's
    host: the cropped track window for `steps` Heun steps, once alone (per-core
    rate) and then as one independent seed per core in separate processes
    (aggregate rate), at most 16 processes (the host share of one GPU)."""
    import subprocess
    model, nproc, usable = cpu_info()
    P = max(1, min(usable, 16))

    def launch(k):
        return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(k),
                                 "--cpu-steps", str(steps)], stdout=subprocess.PIPE, text=True)

    def collect(procs):
        res = []
        for p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                raise RuntimeError(f"oracle worker failed with {p.returncode}")
            res.append(json.loads(out.strip().splitlines()[-1]))
        return res

    one = collect([launch(0)])[0]
    many = collect([launch(k) for k in range(P)])
    per_core = one["updates"] / one["seconds"]
    aggregate = sum(r["updates"] / r["seconds"] for r in many)
    w = cpu_crop(0)
    return dict(value=aggregate, unit="spin-updates/s", cores=P, kind="oracle",
                sample=f"track window cropped to {w.nx}x{w.ny}x{w.nz} in a {w.track_nx}-column "
                       f"track ({one['magnetic_sites']} magnetic sites), {steps} Heun steps per "
                       f"process, FP64 single-threaded plain C; per core: one process alone "
                       f"({one['seconds']:.1f} s); all cores: {P} seeds in {P} concurrent "
                       f"processes (sum of their rates)",
                per_core_value=per_core, all_core_value=aggregate, processes=P,
                cpu_model=model, nproc=nproc, usable_cpus=usable)


def main():
    args = parse()
    if args.cpu_worker >= 0:
        print(json.dumps(cpu_worker(args.cpu_worker, args.cpu_steps)), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the step "
                                   "library drives a single device, and runs over several "
                                   "GPUs are not provided"}))
        sys.exit(2)
    if args.issue_rates:
        r = issue_rates()
        print(json.dumps({"metric": "VALU issue cost per wave64 instruction", "unit": "SIMD cycles",
                          "clock_ghz": 2.4, "classes": r}), flush=True)
        return
    if args.workload == "transfer":
        t = transfer_run(args)
        cg, th = t["res"]["coarse_grain"], t["res"]["thermalise"]
        ach = t["cg_bytes"] / cg / 1e9
        print(json.dumps({
            "metric": "window-end transfer: atomistic sites coarse-grained per s (Eq. 6)",
            "value": t["sites_cg"] / cg, "unit": "sites/s", "n_gpus": 1, "steps": t["reps"],
            "warmup": 1, "ms_per_step": 1e3 * cg, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else "f64",
            "data": "synthetic",
            "config": {"workload": "transfer_track16x800x200x33", "cell": t["cell"],
                       "precision": args.precision},
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k_coarse_grain", "bytes_per_site": 3 * t["e"] + 2},
            "thermalise_sites_per_s": t["sites_th"] / th,
            "thermalise_roofline": {"bound": "hbm", "achieved": t["th_bytes"] / th / 1e9,
                                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": t["th_bytes"] / th / 1e9 / HBM_PEAK_GBS,
                                    "kernel": "k_cone_columns",
                                    "bytes_per_site": 2 * 3 * t["e"] + 2},
        }), flush=True)
        return
    if args.workload == "multiscale":
        r = multiscale_run(args)
        per_step = r["t"] / args.steps
        print(json.dumps({
            "metric": "multiscale window steps/s (atomistic Heun + two micromagnetic RK4 regions)",
            "value": args.steps / r["t"], "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * per_step, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if args.precision == "fp32" else "f64", "data": "synthetic",
            "config": {"workload": "multiscale_window_mm100nm_atoms100nm_mm100nm_60x10nm" +
                                   ("_window_demag" if args.window_demag else ""),
                       "atomistic_magnetic_sites": r["n_atoms"], "micromagnetic_cells": r["n_cells"],
                       "atomistic_kernel": r["kernel"], "precision": args.precision},
            "atomistic_spin_updates_per_s": r["n_atoms"] / per_step,
            "roofline": None}), flush=True)
        return
    if args.workload == "mm":
        r = mm_run(args)
        per_step = r["t"] / args.steps
        e = 4 if args.precision == "fp32" else 8
        hbm = 2 * 3 * e * r["n"] / per_step / 1e9
        alu = 4 * MM_ALU_PER_STAGE * r["n"] / per_step / 1e12
        peak = VALU_PEAK_T if args.precision == "fp32" else VALU_PEAK_T / 2
        print(json.dumps({
            "metric": "micromagnetic cell-updates/s (cells x RK4 steps)",
            "value": r["n"] * args.steps / r["t"], "unit": "cell-updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * per_step,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if args.precision == "fp32" else "f64", "data": "synthetic",
            "config": {"workload": "mm_window300x60x8_cells1x1x2nm_spot800K_locked",
                       "cells": r["n"], "dt_fs": 20.0, "precision": args.precision},
            "roofline": {"bound": "alu", "achieved": alu, "peak": peak,
                         "unit": "T FP32-FMA slots/s" if args.precision == "fp32"
                         else "T FP64-FMA slots/s", "frac": alu / peak,
                         "alu_ops_per_cell_step": 4 * MM_ALU_PER_STAGE,
                         "hbm": {"achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": hbm / HBM_PEAK_GBS, "bytes_per_cell": 6 * e},
                         "traffic": None, "kernel": "k_mm_stage (four launches per step)"},
            "final_mz": r["mz"]}), flush=True)
        return
    if args.workload == "mc":
        r = mc_run(args)
        per_sweep = r["t"] / args.steps
        e = 4 if args.precision == "fp32" else 8
        hbm = 2 * 3 * e * r["n_sites"] / per_sweep / 1e9
        roof = {"bound": "hbm", "achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": hbm / HBM_PEAK_GBS, "bytes_per_site": 6 * e}
        if args.precision == "fp32":
            ach = MC_ALU_OPS * r["n_mag"] / per_sweep / 1e12
            alu = {"achieved": ach, "peak": VALU_PEAK_T, "unit": "T FP32-FMA slots/s",
                   "frac": ach / VALU_PEAK_T, "alu_ops_per_magnetic_site": MC_ALU_OPS}
            if ach / VALU_PEAK_T > hbm / HBM_PEAK_GBS:  # the longer of the two at peak
                roof = dict(bound="alu", **alu)
                roof["hbm"] = {"achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": hbm / HBM_PEAK_GBS, "bytes_per_site": 6 * e}
            else:
                roof["alu"] = alu
        roof.update({"traffic": None, "kernel": "k_mc_colour (two launches per sweep)"})
        print(json.dumps({
            "metric": "Metropolis spin-updates/s (magnetic sites x sweeps)",
            "value": r["n_mag"] * args.steps / r["t"], "unit": "spin-updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * per_sweep,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if args.precision == "fp32" else "f64", "data": "synthetic",
            "config": {"workload": r["w"].name + "+metropolis300K", "sites": r["n_sites"],
                       "magnetic_sites": r["n_mag"], "precision": args.precision},
            "roofline": roof, "final_mz": r["mz"]}), flush=True)
        return
    g = segment_steps(args.steps) if args.graph_steps < 0 else args.graph_steps
    r = gpu_run(args, args.precision, args.kernel, args.steps, args.warmup, g)
    demag = None
    if args.workload in ("demag", "track_demag"):
        # the same workload without the field, on the fastest kernel (the
        # fused step): the cost of the field is the ratio of the two steps
        base = "slab" if args.workload == "demag" else "track"
        r0 = gpu_run(args, args.precision, "auto", args.steps, args.warmup, g, workload=base)
        cx, cy, cz = args.demag_cell
        w = r["w"]
        mesh = (-(-w.nx // cx), -(-w.ny // cy), -(-w.nz // cz))
        t1, t0 = r["t"] / r["steps"], r0["t"] / r0["steps"]
        demag = {"cell": [cx, cy, cz], "mesh": list(mesh),
                 "padded_fft": [1 << (2 * n - 1 - 1).bit_length() if n > 1 else 1 for n in mesh],
                 "reading": "once per step, held through both stages" if args.demag_once
                 else "at both Heun stages",
                 "evaluations_per_step": 1 if args.demag_once else 2, "kernel": r["kname"],
                 "step_ms": 1e3 * t1,
                 "step_without_demag_ms": 1e3 * t0, "kernel_without_demag": r0["kname"],
                 "ratio_to_step_without_demag": t1 / t0}
        if not args.demag_once and not args.no_extras:
            # beside it, the other reading: the field held through the step
            r2 = gpu_run(args, args.precision, args.kernel, args.steps, args.warmup, g,
                         demag_once=True)
            t2 = r2["t"] / r2["steps"]
            demag["held_field"] = {"reading": "once per step, held through both stages",
                                   "kernel": r2["kname"], "step_ms": 1e3 * t2,
                                   "ratio_to_step_without_demag": t2 / t0}
    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    value = r["n_mag"] * r["steps"] / r["t"]
    roof = step_roofline(r)
    if args.workload == "track" and args.precision == "fp32":
        # the goal for this path: 60 % of the HBM peak
        hf = roof["frac"] if roof["bound"] == "hbm" else roof["hbm"]["frac"]
        roof["hbm_target_frac"] = 0.60
        roof["hbm_frac_of_target"] = hf / 0.60
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
        "config": {"workload": r["w"].name + ("_x16seeds" if args.workload in ("track", "track_demag")
                                              else ""),
                   "lattice": "l10" if args.workload == "l10" else "sc",
                   "sites": r["n_sites"],
                   "magnetic_sites": r["n_mag"], "dt_fs": 1.0, "precision": args.precision,
                   "kernel": {1: "plain", 2: "fused"}.get(r["kernel"], "?"), "tile": r["tile"],
                   "graph_steps": r["graph_steps"],
                   "timed_graph_segments": r["steps"] // r["graph_steps"] if r["graph_steps"] else 0,
                   "timed_eager_steps": r["eager_steps"],
                   "untimed_clock_ramp_s": round(r["ramp_s"], 3),
                   "cache_resident": args.workload in ("slab", "l10")},
        "roofline": roof,
        "lattice_site_updates_per_s": r["n_sites"] * r["steps"] / r["t"],
        "max_norm_error": r["norm_err"],
    }
    if demag is not None:
        out["metric"] = "atomistic spin-updates/s (spins x Heun steps) with the demagnetising field"
        out["config"]["workload"] += f"+demag{cx}x{cy}x{cz}"
        out["demag"] = demag
    if not args.no_extras and args.workload == "track" and args.precision == "fp32":
        # the same step beside the headline: the plain FP64 two-pass kernels and the
        # FP64 fused kernel on the same lattice, and the cache-resident lattices
        n64 = 200
        r64 = gpu_run(args, "fp64", "plain", n64, 20, segment_steps(n64), workload="track")
        r64f = gpu_run(args, "fp64", "auto", n64, 20, segment_steps(n64), workload="track")
        out["fp64_plain"] = step_summary(r64)
        out["fp64_fused"] = step_summary(r64f)
        out["speedup_vs_fp64_plain"] = value / out["fp64_plain"]["value"]
        rs = gpu_run(args, "fp32", "auto", 2000, 200, segment_steps(2000), workload="slab")
        rl = gpu_run(args, "fp32", "auto", 1000, 100, segment_steps(1000), workload="l10")
        out["slab_fp32"] = step_summary(rs, cache_resident=True)
        out["l10_fp32"] = step_summary(rl, cache_resident=True)
    if not args.no_cpu_baseline and args.workload == "track":
        out["cpu_baseline"] = cpu_baseline(steps=args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
