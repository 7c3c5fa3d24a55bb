"""The batched M(T) sweep of 512 isolated grains of uneven size (diameters
5-12 nm, heights 8-12 nm, simple cubic, open boundaries, each grain at its own
temperature T_g = 300 + 5 (g mod 121) K, no field): 20 000 steps to equilibrate
and 20 000 sampling steps in one launch per step, FP32, with the FP64 moment
sums of |m| every 10 steps.  From them each grain's susceptibility
chi_g = N_g (<m^2> - <|m|>^2) mu_s / kB T, and per 1 nm diameter bin the Curie
temperature at the peak of chi(T) (the finite-size ordering temperature of the
grains that write the bits, Sec. III).  A subset of the grains is checked
against an FP64 oracle ensemble: <|m|> within 3 combined standard errors.
"""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle_build import oracle_system
from paper_2502_02236_amd import asd as A
from paper_2502_02236_amd import bridge

pytestmark = pytest.mark.gpu


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


def batch_handle(cyl, seed, graph_steps=0):
    w0 = W.Workload("cylinders", bc=(0, 0, 0), B=(0.0, 0.0, 0.0), seed=seed)
    ins = [bridge.SystemInputs(w0.scaled(nx=c.nx, ny=c.ny, nz=c.nz), labels=c.labels, T_system=c.T)
           for c in cyl]
    h = A.Handle(bridge.params_for(w0, A.ASD_FP32, graph_steps=graph_steps), [i.desc for i in ins])
    dr, _ = bridge.drive_for(w0, T_amb=0.0)
    h.set_drive(dr)
    h._inputs = ins
    for k, c in enumerate(cyl):
        S0 = W.initial_spins(len(c.labels), seed + 100 + k)
        S0[:, c.labels < 0] = 0
        h.set_spins(S0, k)
    return w0, h


def diameter_of(c, a=0.3e-9):
    """Area-equivalent diameter of the grain's magnetic cross-section (m)."""
    n_xy = int((c.labels.reshape(c.nz, c.ny, c.nx)[0] >= 0).sum())
    return 2.0 * math.sqrt(n_xy / math.pi) * a


@pytest.mark.timeout(900)
def test_config4_curie_temperature_per_diameter_bin():
    cyl = W.cylinder_batch(n=512)
    equil, sample, every = 20000, 20000, 10
    w0, h = batch_handle(cyl, 4, graph_steps=every)
    h.set_variant(A.ASD_KERNEL_FUSED, 9)
    say(f"[config 4] 512 grains, {sum(int((c.labels >= 0).sum()) for c in cyl)} magnetic sites, "
        f"kernel {h.variant_name()}")
    h.step(equil)
    for s in range(sample // every):
        h.step(every)
        h.accumulate_moments(reset=(s == 0))
    st = h.moment_stats()
    assert np.all(st[:, 0] == sample // every)
    m1, m2 = st[:, 1] / st[:, 0], st[:, 2] / st[:, 0]
    N = np.array([int((c.labels >= 0).sum()) for c in cyl], dtype=np.float64)
    T = np.array([c.T for c in cyl])
    chi = N * (m2 - m1 * m1) * w0.mu_s / (W.KB * T)  # in 1/T: mu_s-weighted, per tesla
    d = np.array([diameter_of(c) for c in cyl]) * 1e9
    say("  T (K)  <|m|> of the grains nearest 300, 500, 650, 750, 900 K:",
        [round(float(m1[np.argmin(np.abs(T - t))]), 3) for t in (300, 500, 650, 750, 900)])
    assert m1[T <= 350].min() > 0.7 and m1[T >= 850].max() < 0.35
    # Curie temperature per 1 nm diameter bin: peak of chi(T) smoothed over 50 K
    tc = {}
    for lo in range(5, 12):
        sel = (d >= lo) & (d < lo + 1)
        if sel.sum() < 30:
            continue
        grid = np.arange(450.0, 851.0, 5.0)
        ts, cs = T[sel], chi[sel] / N[sel]  # per spin, so grains of one bin compare
        sm = np.array([cs[np.abs(ts - g) <= 25.0].mean() if np.any(np.abs(ts - g) <= 25.0) else 0.0
                       for g in grid])
        tc[lo] = float(grid[int(np.argmax(sm))])
        say(f"  d in [{lo}, {lo + 1}) nm: {int(sel.sum())} grains, T_C (chi peak) = {tc[lo]:.0f} K")
    assert len(tc) >= 4
    # finite-size ordering temperatures below and near the bulk 700 K of the
    # simple-cubic Heisenberg model with J = 6.7e-21 J (1.443 J / kB)
    for lo, t in tc.items():
        assert 500.0 <= t <= 760.0, (lo, t)
    bins = sorted(tc)
    assert tc[bins[-1]] >= tc[bins[0]] - 25.0
    h.close()


@pytest.mark.timeout(900)
def test_config4_grains_against_oracle_ensemble():
    """Three grains of the batch (the smallest ones, at their own temperatures):
    <|m|> of 8 FP32 replicas in one launch against 4 FP64 oracle replicas
    (independent noise streams), 3000 + 3000 steps, samples every 10 steps."""
    cyl = W.cylinder_batch(n=512)
    small = sorted(range(512), key=lambda g: int((cyl[g].labels >= 0).sum()))[:3]
    pick = [cyl[g] for g in small]
    reps_g, reps_o = 8, 4
    equil, sample, every = 3000, 3000, 10
    batch = [c for c in pick for _ in range(reps_g)]
    w0, h = batch_handle(batch, 40)
    h.step(equil)
    for s in range(sample // every):
        h.step(every)
        h.accumulate_moments(reset=(s == 0))
    st = h.moment_stats()
    m_gpu = (st[:, 1] / st[:, 0]).reshape(len(pick), reps_g)
    for i, c in enumerate(pick):
        wc = w0.scaled(nx=c.nx, ny=c.ny, nz=c.nz)
        acc_o = []
        for r in range(reps_o):
            sysm = oracle_system(wc, labels=c.labels, sys_id=5000 + 10 * i + r, T_amb=c.T)
            S = W.initial_spins(len(c.labels), 40 + 100 + i * reps_g)
            S[:, c.labels < 0] = 0
            S = sysm.heun(S, 0, equil)
            ms = []
            for s in range(sample // every):
                S = sysm.heun(S, equil + s * every, every)
                _, tot = sysm.magnetisation(S, 1)
                ms.append(np.sqrt((tot[:3] ** 2).sum()) / tot[3])
            acc_o.append(np.mean(ms))
        a, b = m_gpu[i], np.array(acc_o)
        se = math.sqrt(a.var(ddof=1) / len(a) + b.var(ddof=1) / len(b))
        say(f"  grain of {int((c.labels >= 0).sum())} sites at {c.T:.0f} K: gpu {a.mean():.4f} "
            f"oracle {b.mean():.4f} se {se:.4f}")
        assert abs(a.mean() - b.mean()) <= 3 * se + 1e-12
    h.close()
