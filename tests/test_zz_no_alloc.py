"""asd_reduce_magnetization_static (the sums kept in the library's static
device array, nothing allocated) against asd_reduce_magnetization (the sums
in the handle's workspace) through the C ABI: the same kernels in the same
order, so the FP64 sums must be bit-identical.  Two calls in a row on two
handles, the second with fewer grains and systems than the first (the array
keeps the first call's contents), in both precisions; and the size limit.
"""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W
from paper_2502_02236_amd import asd as A
from paper_2502_02236_amd import bridge

pytestmark = pytest.mark.gpu

SCRATCH_SUMS = 32768  # grains + systems the 1 MiB static array holds


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


def sums(h, fn):
    ng = sum(h.grain_count(s) for s in range(len(h.systems)))
    pg = np.full((max(ng, 1), 4), np.nan)
    ps = np.full((len(h.systems), 4), np.nan)
    rc = fn(h.h, pg, ps)
    assert rc == A.ASD_OK, (rc, A.lib().asd_last_error(h.h))
    return pg[:ng], ps


def big_handle(prec):
    """Three seeds of a track crop, stepped with a window shift."""
    w = W.c5_track_window().scaled(nx=40, ny=30, nz=6, track_nx=64, steps_per_bit=25,
                                   x0=6e-9, y0=4.5e-9, grain_pitch=3.0e-9)
    ins = []
    for k in range(3):
        wk = w.scaled(seed=w.seed + k)
        seeds = W.voronoi_seeds(wk)
        ku = W.grain_ku(len(seeds), w.ku, w.ku_spread, wk.seed)
        ins.append(bridge.SystemInputs(wk, seeds=seeds, ku_grain=ku))
    h = A.Handle(bridge.params_for(w, prec), [i.desc for i in ins])
    dr, _ = bridge.drive_for(w)
    h.set_drive(dr)
    h._inputs = ins
    for k in range(3):
        lab = h.labels(k)
        S0 = W.initial_spins(len(lab), w.seed + 100 + k)
        S0[:, lab < 0] = 0
        h.set_spins(S0, k)
    h.step(12)
    h.shift_window(2)
    h.step(8)
    return h


def small_handle(prec):
    """One small granular slab: fewer grains and systems than big_handle."""
    w = W.c2_granular_slab().scaled(nx=21, ny=17, nz=5, x0=3e-9, y0=2.5e-9, grain_pitch=3.0e-9)
    h = bridge.make_handle(w, prec)
    lab = h.labels()
    S0 = W.initial_spins(len(lab), w.seed + 7)
    S0[:, lab < 0] = 0
    h.set_spins(S0)
    h.step(10)
    return h


@pytest.mark.parametrize("prec", [A.ASD_FP64, A.ASD_FP32], ids=["fp64", "fp32"])
def test_static_scratch_sums_match_workspace_sums(prec):
    hb = big_handle(prec)
    hs = small_handle(prec)
    nb = sum(hb.grain_count(s) for s in range(3))
    ns = hs.grain_count(0)
    say(f"grains: first handle {nb} over 3 systems, second {ns} over 1")
    assert ns + 1 < nb + 3
    for h in (hb, hs):  # the second call has the smaller input
        g_ws, s_ws = sums(h, A.asd_reduce_magnetization)
        g_st, s_st = sums(h, A.asd_reduce_magnetization_static)
        say("per-system sums", s_st.tolist())
        assert np.all(np.isfinite(s_st)) and np.all(s_st[:, 3] > 0)
        np.testing.assert_array_equal(g_st, g_ws)
        np.testing.assert_array_equal(s_st, s_ws)
    # the first handle again after the smaller call, then after more steps
    for k in range(2):
        g_ws, s_ws = sums(hb, A.asd_reduce_magnetization)
        g_st, s_st = sums(hb, A.asd_reduce_magnetization_static)
        np.testing.assert_array_equal(g_st, g_ws)
        np.testing.assert_array_equal(s_st, s_ws)
        hb.step(5)
    # one output pointer only
    ps = np.full((3, 4), np.nan)
    assert A.lib().asd_reduce_magnetization_static(hb.h, None, A._np_ptr(ps)) == A.ASD_OK
    np.testing.assert_array_equal(ps, sums(hb, A.asd_reduce_magnetization)[1])
    hb.close()
    hs.close()


def test_static_scratch_rejects_too_many_sums():
    """A checkerboard lattice whose every magnetic site is its own grain:
    more grains than the static array holds."""
    nx, ny, nz = 48, 48, 32
    x, y, z = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    mag = ((x + y + z) % 2 == 0).transpose(2, 1, 0).ravel()  # site index x + nx (y + ny z)
    labels = np.full(nx * ny * nz, -1, np.int32)
    labels[mag] = np.arange(int(mag.sum()), dtype=np.int32)
    assert mag.sum() + 1 > SCRATCH_SUMS
    w = W.c1_plain_sc().scaled(nx=nx, ny=ny, nz=nz, bc=(0, 0, 0))
    h = bridge.make_handle(w, A.ASD_FP64, labels=labels)
    assert h.grain_count(0) == mag.sum()
    pg = np.zeros((int(mag.sum()), 4))
    ps = np.zeros((1, 4))
    rc = A.asd_reduce_magnetization_static(h.h, pg, ps)
    assert rc == A.ASD_EINVAL
    msg = A.lib().asd_last_error(h.h).decode()
    say("rejected:", msg)
    assert "static scratch" in msg
    # the workspace entry point serves the same handle
    g, s = sums(h, A.asd_reduce_magnetization)
    assert s[0, 3] == mag.sum()
    h.close()
