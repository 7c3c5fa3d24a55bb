"""Parity at the benchmark's full sizes, in the configuration bench.py times
(its workload builder, the autotuner's pick among all variants, step graphs of
100 steps): the L1_0 window (260x156x27 cells, four shells, 2.19M Fe sites),
512 isolated cylinders of uneven size each at its own temperature (11.4M
sites in one launch) and 16 seeds of the 400x200x33 moving window in
800-column tracks with per-grain anisotropy and a window shift.

Three steps (two, a shift of one column on the track, one more) are compared
with the oracle at every site of the L1_0 window, of a sample of cylinders (the
first, last, smallest, largest and two in between) and of the first and last
track seeds; then 100 more steps are checked by invariants on every system:
unit length of magnetic spins, zero at non-magnetic sites, per-system magnetic
site counts.  The track is also run for 100 steps as one graph segment, a
shift and two more steps, with a seed compared against the oracle at every
site.  Bars: FP64 within 1e-12 per component, FP32 within 1e-4 (the FP32 path
at every stage against the FP64 oracle).
"""
import sys

import numpy as np
import pytest

import bench
import workloads as W
from oracle_build import oracle_geometry, oracle_labels, oracle_system, window_mask
from paper_2502_02236_amd import asd as A

pytestmark = pytest.mark.gpu

TOL = {A.ASD_FP64: 1e-12, A.ASD_FP32: 1e-4}
NORM_TOL = {A.ASD_FP64: 1e-12, A.ASD_FP32: 1e-6}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    A.lib()
    return torch


def bench_handle(name, prec, tmp_path):
    """The benchmark's handle for a workload, autotuned as bench.py does."""
    w, h, S0s, n_mag, n_sites, extra = bench.build_workload(name, prec, 100)
    h.autotune(bench.TUNE_CACHE)  # the tile picks bench.py times
    for k, S0 in enumerate(S0s):
        h.set_spins(S0, k)
    h.set_step(0)
    h.prepare()
    say(f"[{name}] prec={prec} variant {h.variant()} {h.variant_name()}")
    return w, h, S0s


# the oracle's results, shared by both precisions (the initial spins are the
# same FP64 arrays; the FP32 handle rounds them on upload), and its lattice
# geometry, shared by every system of one lattice
_RESULTS = {}
_GEOMETRY = {}


def oracle_run(key, w, labels_of, S0, ku=None, sys_id=0, T_amb=None, track=False):
    """(labels, spins) of the oracle after two steps, (on a track) a shift of one
    column, one step; labels_of() gives the oracle's own grain labels."""
    if key in _RESULTS:
        return _RESULTS[key]
    labels = labels_of()
    gkey = (w.kind, w.track_nx or w.nx, w.ny, w.nz, tuple(w.bc), w.a, w.c)
    if gkey not in _GEOMETRY:
        say(f"  oracle neighbour shells of {gkey[:4]} ...")
        _GEOMETRY.clear()
        _GEOMETRY[gkey] = oracle_geometry(w)
    sysm = oracle_system(w, labels=labels, ku_grain=ku, sys_id=sys_id, T_amb=T_amb,
                         active=window_mask(w, 0) if track else None, origin=0,
                         geometry=_GEOMETRY[gkey])
    S = sysm.heun(np.array(S0, np.float64), 0, 2)
    if track:
        sysm.set_active(window_mask(w, 1), 1)
    _RESULTS[key] = labels, sysm.heun(S, 2, 1)
    return _RESULTS[key]


def gpu_three_steps(h, track=False):
    h.step(2)
    if track:
        h.shift_window(1)
    h.step(1)


def check_invariants(h, labels, prec, window=None):
    """100 more steps; `window`: the sites the magnetisation sums cover (all
    stored sites when None)."""
    h.step(100)
    _, per_sys = h.magnetization()
    for k, lab in enumerate(labels):
        S = h.get_spins(k).astype(np.float64)
        mag = lab >= 0
        assert np.all(S[:, ~mag] == 0), k
        assert np.max(np.abs(np.sqrt((S[:, mag] ** 2).sum(0)) - 1)) < NORM_TOL[prec], k
        counted = mag if window is None else mag & window
        assert per_sys[k, 3] == counted.sum(), k


@pytest.mark.parametrize("prec", [A.ASD_FP64, A.ASD_FP32], ids=["fp64", "fp32"])
def test_full_size_l10_window(prec, tmp_path):
    w, h, S0s = bench_handle("l10", prec, tmp_path)
    lab = h.labels()
    gpu_three_steps(h)
    olab, So = oracle_run("l10", w, lambda: oracle_labels(w), S0s[0])
    assert np.array_equal(lab, olab)
    err = float(np.max(np.abs(h.get_spins().astype(np.float64) - So)))
    say(f"  L1_0 {lab.size} sites: max |dS| {err:.3e}")
    assert err <= TOL[prec]
    check_invariants(h, [lab], prec)
    h.close()


@pytest.mark.parametrize("prec", [A.ASD_FP64, A.ASD_FP32], ids=["fp64", "fp32"])
def test_full_size_cylinder_batch(prec, tmp_path):
    w, h, S0s = bench_handle("cylinders", prec, tmp_path)
    cyl = W.cylinder_batch(n=512)
    assert len(h.systems) == len(cyl) == 512
    gpu_three_steps(h)
    sizes = np.array([c.labels.size for c in cyl])
    sample = sorted({0, 1, 255, 511, int(np.argmin(sizes)), int(np.argmax(sizes))})
    say(f"  {sizes.sum()} sites in {len(cyl)} systems ({sizes.min()}..{sizes.max()}); sample {sample}")
    for k in sample:
        c = cyl[k]
        wc = w.scaled(nx=c.nx, ny=c.ny, nz=c.nz)
        _, So = oracle_run(("cylinder", k), wc, lambda: c.labels, S0s[k], sys_id=k, T_amb=c.T)
        err = float(np.max(np.abs(h.get_spins(k).astype(np.float64) - So)))
        say(f"  cylinder {k} ({c.labels.size} sites, {c.T:.0f} K): max |dS| {err:.3e}")
        assert err <= TOL[prec], (k, err)
    check_invariants(h, [c.labels for c in cyl], prec)
    h.close()


@pytest.mark.parametrize("prec", [A.ASD_FP64, A.ASD_FP32], ids=["fp64", "fp32"])
def test_full_size_track_seeds(prec, tmp_path):
    w, h, S0s = bench_handle("track", prec, tmp_path)
    ins, _ = h._inputs
    n_seeds = len(ins)
    assert n_seeds == 16
    labs = [h.labels(k) for k in range(n_seeds)]
    gpu_three_steps(h, track=True)
    for k in (0, n_seeds - 1):
        # one Philox key for the handle (w.seed); the seeds differ in grains,
        # anisotropy and system id
        olab, So = oracle_run(("track", k), w, lambda: oracle_labels(w, seeds=ins[k].seeds),
                              S0s[k], ku=ins[k].ku, sys_id=k, track=True)
        assert np.array_equal(labs[k], olab), k
        err = float(np.max(np.abs(h.get_spins(k).astype(np.float64) - So)))
        say(f"  track seed {k} ({labs[k].size} stored sites): max |dS| {err:.3e}")
        assert err <= TOL[prec], (k, err)
    check_invariants(h, labs, prec, window=window_mask(w, 1).astype(bool))
    h.close()


_LONG = {}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [A.ASD_FP64, A.ASD_FP32], ids=["fp64", "fp32"])
def test_full_size_track_seed_100_steps(prec, tmp_path):
    """The 16-seed track in the benchmark's autotuned variant: 100 steps as one
    graph segment, a shift of one column, two more steps; the last seed (all
    2.64M window sites of an 800-column track) against the oracle."""
    w, h, S0s = bench_handle("track", prec, tmp_path)
    ins, _ = h._inputs
    k = len(ins) - 1
    h.step(100)
    h.shift_window(1)
    h.step(2)
    Sg = h.get_spins(k).astype(np.float64)
    lab = h.labels(k)
    h.close()
    if "S" not in _LONG:
        olab = oracle_labels(w, seeds=ins[k].seeds)
        assert np.array_equal(lab, olab)
        say("  oracle: neighbour shells of the 800-column track ...")
        sysm = oracle_system(w, labels=olab, ku_grain=ins[k].ku, sys_id=k,
                             active=window_mask(w, 0), origin=0)
        S = np.array(S0s[k], np.float64)
        for n0 in range(0, 100, 10):
            S = sysm.heun(S, n0, 10)
            say(f"  oracle step {n0 + 10}/100")
        sysm.set_active(window_mask(w, 1), 1)
        _LONG["S"] = sysm.heun(S, 100, 2)
    err = float(np.max(np.abs(Sg - _LONG["S"])))
    say(f"  track seed {k}, 102 steps with a shift: max |dS| {err:.3e}")
    assert err <= TOL[prec], err
