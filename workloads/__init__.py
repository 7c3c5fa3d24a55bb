"""Seeded synthetic inputs and workload definitions.

This module holds no arithmetic of the sLLG method: it only states the
workload parameters (sizes, material constants, drive) and draws the seeded
random inputs the method takes from outside -- initial spin directions,
Voronoi seed points, per-grain anisotropy spread and the geometry of
isolated cylindrical grains.  Both the GPU library's tests/benchmark and the
oracle receive the same arrays from here; each side then builds its own
lattice, neighbour shells, grain labels and dynamics.

Paper parameters cited: simple-cubic atomistic lattice, Voronoi granular
track with 8 nm grains and 1 nm boundaries, 20 m/s head velocity, 20 nm
bits, Gaussian laser spot, write field polarity (Sec. III); L1_0 Fe
sublattice and mu_s, K_1 mapping (Appendix A).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

MU_B = 9.2740100783e-24  # J/T (CODATA 2018)
KB = 1.380649e-23  # J/K (exact SI)

SC, L10 = 0, 1
BC_OPEN, BC_PERIODIC, BC_TRACK = 0, 1, 2
SPOT_NONE, SPOT_MOVING, SPOT_LOCKED = 0, 1, 2

Q_UNITS = 16  # Voronoi integer geometry: units of (lattice x unit)/16


@dataclass
class Workload:
    name: str
    kind: int = SC
    nx: int = 16
    ny: int = 16
    nz: int = 8
    bc: tuple = (BC_PERIODIC, BC_PERIODIC, BC_OPEN)
    track_nx: int = 0  # >0: x is a frozen track of this many columns (BC_TRACK)
    a: float = 0.3e-9
    c: float = 0.3e-9
    J: tuple = (6.7e-21,)
    mu_s: float = 3.23 * MU_B
    alpha: float = 0.1
    gamma: float = 1.76e11
    dt: float = 1e-15
    ku: float = 2.6e-22
    B: tuple = (0.0, 0.0, -0.8)
    bits: Optional[tuple] = None
    steps_per_bit: int = 0
    spot_mode: int = SPOT_NONE
    T_amb: float = 300.0
    T_peak: float = 300.0
    fwhm: float = 0.0
    x0: float = 0.0
    y0: float = 0.0
    v: float = 0.0
    seed: int = 1
    steps: int = 1000
    grains: bool = False  # Voronoi grains
    grain_pitch: float = 8.618e-9  # hex pitch for 8 nm mean interior diameter
    grain_jitter: float = 0.5  # jitter amplitude (fraction of the pitch): log-sd of D ~ 0.15
    boundary_w: float = 1e-9
    ku_spread: float = 0.0

    @property
    def hx(self):
        return self.a if self.kind == SC else 0.5 * self.a

    @property
    def n_sites(self):
        return (1 if self.kind == SC else 2) * self.nx * self.ny * self.nz

    @property
    def shell_radii(self):
        if self.kind == SC:
            return (self.a,)
        a, c = self.a, self.c
        return (a / math.sqrt(2.0), c, a, math.sqrt(0.5 * a * a + c * c))[: len(self.J)]

    @property
    def w_units(self):
        return int(round(self.boundary_w / self.hx * Q_UNITS))

    def scaled(self, **kw):
        return replace(self, **kw)


# --------------------------------------------------------------------------
# The five workloads (sizes and physics), plus small parity crops.
# --------------------------------------------------------------------------
def c1_plain_sc() -> Workload:
    """SC 16x16x8 (2048 spins), periodic x,y, open z, T=300 K, B=-0.8 T z, 1000 steps."""
    return Workload(name="sc16x16x8_fp64_T300", seed=1, steps=1000)


def c2_granular_slab(field_sign: float = -1.0) -> Workload:
    """SC 200x200x33 granular slab (60x60x10 nm at a=0.3 nm), Voronoi 8 nm grains with
    1 nm boundaries, 800 K Gaussian spot (FWHM 40 nm) moving at 10 m/s over 300 K."""
    return Workload(
        name="sc200x200x33_voronoi8nm_spot800K", nx=200, ny=200, nz=33, a=0.3e-9,
        B=(0.0, 0.0, 0.8 * field_sign), spot_mode=SPOT_MOVING, T_amb=300.0, T_peak=800.0,
        fwhm=40e-9, x0=30e-9, y0=30e-9, v=10.0, seed=2, steps=10000, grains=True)


def c3_l10_window() -> Workload:
    """L1_0 Fe sublattice, 260x156x27 cells (100x60x10 nm), four shells, Voronoi grains."""
    return Workload(
        name="l10_260x156x27_4shell_voronoi", kind=L10, nx=260, ny=156, nz=27, a=0.385e-9,
        c=0.371e-9, J=(6.0e-21, 1.2e-21, 0.5e-21, 0.2e-21), B=(0.0, 0.0, -0.8),
        spot_mode=SPOT_MOVING, T_amb=300.0, T_peak=800.0, fwhm=40e-9, x0=50e-9, y0=30e-9,
        v=10.0, seed=3, steps=10000, grains=True)


def c5_track_window(track_nx: int = 800) -> Workload:
    """Moving window 400x200x33 (120x60x10 nm) in a frozen SC track; window-locked
    800 K spot, 20 m/s, 20 nm bits of +-0.8 T, 5 % per-grain k_u spread."""
    a, v, dt = 0.3e-9, 20.0, 1e-15
    return Workload(
        name="sc_track_window400x200x33", nx=400, ny=200, nz=33, a=a,
        bc=(BC_TRACK, BC_OPEN, BC_OPEN), track_nx=track_nx, B=(0.0, 0.0, 0.8),
        bits=tuple(int(b) for b in "0010111100101101100100001"),
        steps_per_bit=int(round(20e-9 / (v * dt))), spot_mode=SPOT_LOCKED, T_amb=300.0,
        T_peak=800.0, fwhm=40e-9, x0=60e-9, y0=30e-9, v=v, dt=dt, seed=5, steps=2_000_000,
        grains=True, ku_spread=0.05)


def steps_per_column(w: Workload) -> int:
    """Head advance of one lattice column, in integer steps (a / (v dt) rounded)."""
    return int(round(w.hx / (w.v * w.dt)))


# --------------------------------------------------------------------------
# Seeded random inputs
# --------------------------------------------------------------------------
def initial_spins(n: int, seed: int, jitter: float = 0.1, dtype=np.float64) -> np.ndarray:
    """+z spins with uniform +-jitter in the x and y components, normalised: float[3, n]."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5151]))
    ex = rng.uniform(-jitter, jitter, n)
    ey = rng.uniform(-jitter, jitter, n)
    S = np.stack([ex, ey, np.ones(n)])
    S /= np.sqrt((S * S).sum(0))
    return S.astype(dtype)


def random_spins(n: int, seed: int) -> np.ndarray:
    """Isotropically random unit spins: float64[3, n]."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x7777]))
    v = rng.normal(size=(3, n))
    return v / np.sqrt((v * v).sum(0))


def voronoi_seeds(w: Workload, nx_extent: Optional[int] = None) -> np.ndarray:
    """Jittered hexagonal seed points, int32[n, 2], in units of hx/Q_UNITS.

    The hex pitch is adjusted per axis so that rows and columns are
    commensurate with the (periodic) box; each seed is displaced uniformly by
    up to +-grain_jitter*pitch along x and y."""
    nx = nx_extent if nx_extent is not None else (w.track_nx if w.track_nx else w.nx)
    lx_units = (nx if w.kind == SC else 2 * nx) * Q_UNITS
    ly_units = (w.ny if w.kind == SC else 2 * w.ny) * Q_UNITS
    unit = w.hx / Q_UNITS
    Lx, Ly = lx_units * unit, ly_units * unit
    ncol = max(1, int(round(Lx / w.grain_pitch)))
    nrow = max(2, int(round(Ly / (w.grain_pitch * math.sqrt(3.0) / 2.0))))
    nrow += nrow % 2
    px, py = Lx / ncol, Ly / nrow
    rng = np.random.default_rng(np.random.SeedSequence([w.seed, 0x6121]))
    pts = []
    for j in range(nrow):
        for i in range(ncol):
            x = (i + 0.5 * (j % 2) + 0.25) * px
            y = (j + 0.5) * py
            x += rng.uniform(-1, 1) * w.grain_jitter * w.grain_pitch
            y += rng.uniform(-1, 1) * w.grain_jitter * w.grain_pitch
            pts.append((int(round(x / unit)) % lx_units, int(round(y / unit)) % ly_units))
    return np.asarray(pts, dtype=np.int32)


def grain_ku(n_grains: int, ku: float, spread: float, seed: int) -> np.ndarray:
    """Per-grain k_u = ku (1 + spread xi), xi standard normal truncated at +-3."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x4B55]))
    xi = rng.normal(size=n_grains)
    while np.any(np.abs(xi) > 3.0):
        bad = np.abs(xi) > 3.0
        xi[bad] = rng.normal(size=int(bad.sum()))
    return ku * (1.0 + spread * xi)


@dataclass
class Cylinder:
    nx: int
    ny: int
    nz: int
    labels: np.ndarray  # int32[nx*ny*nz], 0 inside, -1 outside
    T: float


def cylinder_batch(n: int = 512, a: float = 0.3e-9, seed: int = 4, d_range=(5e-9, 12e-9),
                   h_range=(8e-9, 12e-9), T0: float = 300.0, dT: float = 5.0,
                   n_T: int = 121) -> list:
    """Isolated cylindrical grains of uneven size (open boundaries), each at its own T:
    T_g = T0 + dT (g mod n_T)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xC411]))
    out = []
    for g in range(n):
        d = rng.uniform(*d_range)
        h = rng.uniform(*h_range)
        r = 0.5 * d / a
        nxy = int(math.ceil(d / a))
        nz = max(1, int(round(h / a)))
        c = 0.5 * (nxy - 1)
        y, x = np.mgrid[0:nxy, 0:nxy]
        inside = ((x - c) ** 2 + (y - c) ** 2) <= r * r
        lab2d = np.where(inside, 0, -1).astype(np.int32)
        lab = np.broadcast_to(lab2d, (nz, nxy, nxy)).reshape(-1).copy()
        out.append(Cylinder(nxy, nxy, nz, lab, T0 + dT * (g % n_T)))
    return out
