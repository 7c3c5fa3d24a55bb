"""Build oracle systems from workload definitions (oracle side only).

Everything here goes through ``oracle`` (lattice, neighbour shells, Voronoi
labels, positions); the GPU library is never consulted.
"""
from __future__ import annotations

import numpy as np

import oracle
import workloads as W


def oracle_labels(w: W.Workload, seeds=None, nx_extent=None) -> np.ndarray:
    nx = nx_extent if nx_extent is not None else (w.track_nx or w.nx)
    if not w.grains:
        return np.zeros(oracle.lattice_sites(w.kind, nx, w.ny, w.nz), dtype=np.int32)
    if seeds is None:
        seeds = W.voronoi_seeds(w, nx)
    per = (int(w.bc[0] == W.BC_PERIODIC), int(w.bc[1] == W.BC_PERIODIC))
    return oracle.voronoi_labels(w.kind, nx, w.ny, w.nz, per, W.Q_UNITS, seeds, w.w_units)


def oracle_geometry(w: W.Workload):
    """The oracle's neighbour shells and site positions of the stored lattice:
    ((row_ptr, col, shell), (px, py)); they depend on the geometry only, so
    callers may reuse them for every system of one lattice."""
    nx = w.track_nx or w.nx
    per = [int(b == W.BC_PERIODIC) for b in w.bc]
    return (oracle.neighbours(w.kind, nx, w.ny, w.nz, per, w.a, w.c, w.shell_radii),
            oracle.site_positions(w.kind, nx, w.ny, w.nz, w.a))


def oracle_system(w: W.Workload, labels=None, ku_grain=None, sys_id=0, active=None, origin=0,
                  T_amb=None, geometry=None) -> oracle.System:
    """Oracle system over the full stored lattice (track length when x is a track);
    `geometry`: oracle_geometry(w), when already built."""
    (row, col, sh), (px, py) = geometry if geometry is not None else oracle_geometry(w)
    if labels is None:
        labels = oracle_labels(w)
    n = len(labels)
    return oracle.System(
        row_ptr=row, col=col, shell=sh, label=labels, px=px, py=py,
        ctr0=np.arange(n, dtype=np.uint32), n_shells=len(w.J), J=w.J, mu_s=w.mu_s,
        alpha=w.alpha, gamma=w.gamma, dt=w.dt, ku=w.ku, ku_grain=ku_grain, B=w.B,
        bits=w.bits, steps_per_bit=w.steps_per_bit, spot_mode=w.spot_mode,
        T_amb=w.T_amb if T_amb is None else T_amb, T_peak=w.T_peak, fwhm=w.fwhm, x0=w.x0,
        y0=w.y0, v=w.v, seed=w.seed, rounds=10, sys_id=sys_id, active=active, hx=w.hx,
        origin=origin)


def window_mask(w: W.Workload, origin: int) -> np.ndarray:
    """1 for sites whose x column lies inside the window [origin, origin + nx)."""
    nx = w.track_nx or w.nx
    n = oracle.lattice_sites(w.kind, nx, w.ny, w.nz)
    idx = np.arange(n)
    cell = idx if w.kind == W.SC else idx // 2
    x = cell % nx
    return ((x >= origin) & (x < origin + w.nx)).astype(np.uint8)


def free_spins_system(n: int, *, mu_s, alpha, gamma, dt, ku, B, T, seed=7, sys_id=0):
    """n uncoupled spins (no neighbours), uniform temperature T."""
    return oracle.System(
        row_ptr=np.zeros(n + 1, dtype=np.int64), col=np.zeros(1, np.int32),
        shell=np.zeros(1, np.int8), label=np.zeros(n, np.int32), px=np.zeros(n), py=np.zeros(n),
        ctr0=np.arange(n, dtype=np.uint32), n_shells=0, J=(), mu_s=mu_s, alpha=alpha,
        gamma=gamma, dt=dt, ku=ku, B=B, spot_mode=oracle.SPOT_NONE, T_amb=T, seed=seed,
        sys_id=sys_id)


def demag_cells(w: W.Workload, cell, origin: int = 0):
    """(dn, dd, dcell) of the demagnetising mesh of the window: coarse cells of
    cell[0] x cell[1] x cell[2] lattice cells in the window frame, numbered x
    fastest; dcell = -1 for stored sites outside the window."""
    nx = w.track_nx or w.nx
    n = oracle.lattice_sites(w.kind, nx, w.ny, w.nz)
    idx = np.arange(n)
    lc = idx if w.kind == W.SC else idx // 2
    x, y, z = lc % nx - origin, (lc // nx) % w.ny, lc // (nx * w.ny)
    cx, cy, cz = cell
    dn = (-(-w.nx // cx), -(-w.ny // cy), -(-w.nz // cz))
    zc = w.a if w.kind == W.SC else w.c
    dd = (cx * w.a, cy * w.a, cz * zc)
    inwin = (x >= 0) & (x < w.nx)
    dcell = np.where(inwin, x // cx + dn[0] * (y // cy + dn[1] * (z // cz)), -1).astype(np.int32)
    return dn, dd, dcell


def track_stray(w: W.Workload, cell, origin: int, S) -> np.ndarray:
    """Field (T) of the frozen track at the window's coarse cells, float[3, ncell]:
    the window's cells continued along the whole stored track (window cell i is
    track cell i + ceil(origin / cx)), Eq. 6 over the stored sites outside the
    window, Eq. 7 summed directly, read at the window's cells."""
    nx = w.track_nx or w.nx
    n = oracle.lattice_sites(w.kind, nx, w.ny, w.nz)
    idx = np.arange(n)
    lc = idx if w.kind == W.SC else idx // 2
    xw, y, z = lc % nx - origin, (lc // nx) % w.ny, lc // (nx * w.ny)
    cx, cy, cz = cell
    dn, dd, _ = demag_cells(w, cell, origin)
    i0 = -(-origin // cx)
    it = xw // cx + i0
    nt = int(it.max()) + 1
    frozen = (xw < 0) | (xw >= w.nx)
    dcell = np.where(frozen, it + nt * (y // cy + dn[1] * (z // cz)), -1).astype(np.int32)
    B = oracle.demag_field(S, dcell, (nt, dn[1], dn[2]), dd, w.mu_s)
    i, j, k = np.meshgrid(np.arange(dn[0]), np.arange(dn[1]), np.arange(dn[2]), indexing="ij")
    win = (i + i0 + nt * (j + dn[1] * k)).transpose(2, 1, 0).reshape(-1)  # window cell order
    return B[:, win]


def checkerboard(w: W.Workload) -> np.ndarray:
    """Monte Carlo colours of every stored site (stored-lattice coordinates):
    SC (x + y + z) mod 2; L1_0 s + 2 ((x + y) mod 2) + 4 (z mod 2) with s the
    sublattice, so that no two sites of any of the four shells share a colour
    (shells 1 and 4 change s, shell 2 changes z, shell 3 changes x + y)."""
    nx = w.track_nx or w.nx
    n = oracle.lattice_sites(w.kind, nx, w.ny, w.nz)
    idx = np.arange(n)
    cell = idx if w.kind == W.SC else idx // 2
    x, y, z = cell % nx, (cell // nx) % w.ny, cell // (nx * w.ny)
    if w.kind == W.SC:
        return ((x + y + z) % 2).astype(np.int8)
    s = idx % 2
    return (s + 2 * ((x + y) % 2) + 4 * (z % 2)).astype(np.int8)
