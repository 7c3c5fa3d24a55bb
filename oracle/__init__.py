"""FP64 CPU oracle for the sLLG Heun step (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  It shares no code with the GPU
library ``paper_2502_02236_amd``; it loads its own C file ``asd_oracle.c``
(plain loops, FP64, ``-ffp-contract=off``) through ctypes.

Paper: Gija et al., arXiv 2502.02236 -- Eq. 1 (sLLG), Sec. II thermal field,
Eq. 2 (exchange), Eq. 3 (anisotropy), Sec. III (spot, write field, Voronoi
track), Appendix A (L1_0 Fe sublattice), Eq. 6 (moment sums; the window-end
transfer to and from a coarse grid with cone thermalisation, Sec. II).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "asd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SC, L10 = 0, 1
SPOT_NONE, SPOT_MOVING, SPOT_LOCKED = 0, 1, 2
KB = 1.380649e-23


def build(force: bool = True) -> str:
    """Compile asd_oracle.c with gcc (-O2 -ffp-contract=off) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


P = C.POINTER
i32p, i64p, u32p, u8p, i8p, f64p = (P(C.c_int32), P(C.c_int64), P(C.c_uint32), P(C.c_uint8),
                                    P(C.c_int8), P(C.c_double))


class OrcSystem(C.Structure):
    _fields_ = [
        ("n_sites", C.c_int64), ("row_ptr", i64p), ("col", i32p), ("shell", i8p),
        ("label", i32p), ("active", u8p), ("px", f64p), ("py", f64p), ("ctr0", u32p),
        ("sys_id", C.c_uint32), ("hx", C.c_double), ("origin", C.c_int64),
        ("n_shells", C.c_int), ("J", C.c_double * 4), ("mu_s", C.c_double),
        ("alpha", C.c_double), ("gamma", C.c_double), ("dt", C.c_double), ("ku", C.c_double),
        ("ku_grain", f64p), ("B", C.c_double * 3), ("n_bits", C.c_int), ("bits", u8p),
        ("steps_per_bit", C.c_int64), ("spot_mode", C.c_int), ("T_amb", C.c_double),
        ("T_peak", C.c_double), ("fwhm", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
        ("v", C.c_double), ("seed", C.c_uint64), ("rounds", C.c_int),
        ("dn", C.c_int * 3), ("dd", C.c_double * 3), ("dcell", i32p), ("bstray", f64p),
        ("demag_once", C.c_int),
    ]


class OrcMM(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("periodic", C.c_int * 3),
        ("h", C.c_double * 3), ("Ms0", C.c_double), ("A0", C.c_double), ("K0", C.c_double),
        ("lambda_", C.c_double), ("gamma", C.c_double), ("Tc", C.c_double), ("mu_s", C.c_double),
        ("dt", C.c_double), ("B", C.c_double * 3), ("n_bits", C.c_int), ("bits", u8p),
        ("steps_per_bit", C.c_int64), ("spot_mode", C.c_int), ("T_amb", C.c_double),
        ("T_peak", C.c_double), ("fwhm", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
        ("v", C.c_double), ("ghost", f64p * 2), ("bd", f64p),
    ]


def _declare(L):
    L.orc_philox_batch.argtypes = [C.c_int, C.c_uint64, u32p, u32p, C.c_int64]
    L.orc_ln_batch.argtypes = [f64p, f64p, C.c_int64]
    L.orc_exp_batch.argtypes = [f64p, f64p, C.c_int64]
    L.orc_sincos2pi_batch.argtypes = [f64p, f64p, f64p, C.c_int64]
    L.orc_gauss3_batch.argtypes = [C.c_int, C.c_uint64, u32p, u32p, C.c_uint32, C.c_uint32,
                                   f64p, C.c_int64]
    L.orc_lattice_sites.argtypes = [C.c_int] * 4
    L.orc_lattice_sites.restype = C.c_int64
    L.orc_build_neighbours.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, i32p, C.c_double,
                                       C.c_double, C.c_int, f64p, i64p, i32p, i8p]
    L.orc_build_neighbours.restype = C.c_int64
    L.orc_site_positions.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, f64p, f64p]
    L.orc_voronoi_labels.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, i32p, C.c_int, i32p,
                                     C.c_int, C.c_int64, i32p]
    L.orc_heun_steps.argtypes = [P(OrcSystem), f64p, f64p, f64p, C.c_int64, C.c_int64]
    L.orc_heun_steps.restype = C.c_int
    L.orc_magnetisation.argtypes = [P(OrcSystem), f64p, f64p, f64p, C.c_int, f64p, f64p]
    L.orc_energy.argtypes = [P(OrcSystem), f64p, f64p, f64p, C.c_int64, f64p]
    L.orc_site_temperature.argtypes = [P(OrcSystem), C.c_int64, C.c_int64]
    L.orc_site_temperature.restype = C.c_double
    L.orc_polarity.argtypes = [P(OrcSystem), C.c_int64]
    L.orc_polarity.restype = C.c_double
    L.orc_field.argtypes = [P(OrcSystem), f64p, f64p, f64p, C.c_int64, C.c_int64, f64p]
    L.orc_coarse_grain.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, i32p, f64p, f64p, f64p,
                                   C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, f64p]
    L.orc_newell_tensor.argtypes = [C.c_double] * 6 + [f64p]
    L.orc_demag_direct.argtypes = [C.c_int] * 3 + [C.c_double] * 3 + [f64p, f64p]
    L.orc_mc_sweeps.argtypes = [P(OrcSystem), i8p, C.c_int, f64p, f64p, f64p, C.c_int64,
                                C.c_int64]
    L.orc_mc_sweeps.restype = C.c_int
    L.orc_langevin.argtypes = [C.c_double]
    L.orc_langevin.restype = C.c_double
    L.orc_mm_me.argtypes = [C.c_double, C.c_double, C.c_double]
    L.orc_mm_me.restype = C.c_double
    L.orc_mm_rk4.argtypes = [P(OrcMM), f64p, C.c_int64, C.c_int64]
    L.orc_mm_rk4.restype = C.c_int
    L.orc_mm_temperature.argtypes = [P(OrcMM), C.c_int, C.c_int, C.c_double]
    L.orc_mm_temperature.restype = C.c_double
    L.orc_mm_polarity.argtypes = [P(OrcMM), C.c_int64]
    L.orc_mm_polarity.restype = C.c_double
    L.orc_set_columns.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, i32p, f64p, f64p, f64p,
                                  C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, f64p]
    L.orc_cone_theta_max.argtypes = [C.c_double]
    L.orc_cone_theta_max.restype = C.c_double
    L.orc_cone_spin.argtypes = [f64p, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                f64p]
    L.orc_cone_columns.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, i32p, f64p, f64p, f64p,
                                   C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, f64p, C.c_int,
                                   C.c_uint64, C.c_uint32, C.c_uint32]
    L.orc_cone_spin_mode.argtypes = [C.c_int, f64p, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32,
                                     C.c_uint32, f64p]
    L.orc_cone_columns_mode.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, i32p, f64p,
                                        f64p, f64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                        f64p, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32]
    L.orc_mm_shift.argtypes = [P(OrcMM), f64p, f64p, C.c_int, f64p]
    L.orc_mm_face_moment.argtypes = [P(OrcMM), f64p, C.c_int, C.c_double, f64p]


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


# ---------------------------------------------------------------- noise
def philox(ctr, seed: int, rounds: int = 10) -> np.ndarray:
    """Philox4x32-R of each counter row (uint32[n,4]); key = (lo32 seed, hi32 seed)."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().orc_philox_batch(rounds, seed, _ptr(ctr, u32p), _ptr(out, u32p), len(ctr))
    return out


def ln(u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    lib().orc_ln_batch(_ptr(u, f64p), _ptr(out, f64p), u.size)
    return out


def exp(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().orc_exp_batch(_ptr(x, f64p), _ptr(out, f64p), x.size)
    return out


def sincos2pi(u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    s, c = np.empty_like(u), np.empty_like(u)
    lib().orc_sincos2pi_batch(_ptr(u, f64p), _ptr(s, f64p), _ptr(c, f64p), u.size)
    return s, c


def gauss3(sites, steps, sys_id: int, seed: int, stage: int = 0, rounds: int = 10) -> np.ndarray:
    sites = np.ascontiguousarray(sites, dtype=np.uint32).ravel()
    steps = np.ascontiguousarray(np.broadcast_to(np.asarray(steps, dtype=np.uint32), sites.shape))
    g = np.empty((sites.size, 3), dtype=np.float64)
    lib().orc_gauss3_batch(rounds, seed, _ptr(sites, u32p), _ptr(steps, u32p), sys_id, stage,
                           _ptr(g, f64p), sites.size)
    return g


# ---------------------------------------------------------------- lattice
def lattice_sites(kind: int, nx: int, ny: int, nz: int) -> int:
    return int(lib().orc_lattice_sites(kind, nx, ny, nz))


def neighbours(kind, nx, ny, nz, periodic, a, c, radii):
    """Brute-force neighbour shells: (row_ptr int64[n+1], col int32, shell int8)."""
    per = np.ascontiguousarray(periodic, dtype=np.int32)
    rad = np.ascontiguousarray(radii, dtype=np.float64)
    n = lattice_sites(kind, nx, ny, nz)
    row = np.empty(n + 1, dtype=np.int64)
    tot = lib().orc_build_neighbours(kind, nx, ny, nz, _ptr(per, i32p), a, c, len(rad),
                                     _ptr(rad, f64p), _ptr(row, i64p), None, None)
    col = np.empty(max(tot, 1), dtype=np.int32)
    sh = np.empty(max(tot, 1), dtype=np.int8)
    lib().orc_build_neighbours(kind, nx, ny, nz, _ptr(per, i32p), a, c, len(rad),
                               _ptr(rad, f64p), _ptr(row, i64p), _ptr(col, i32p), _ptr(sh, i8p))
    return row, col[:tot], sh[:tot]


def site_positions(kind, nx, ny, nz, a):
    n = lattice_sites(kind, nx, ny, nz)
    px, py = np.empty(n), np.empty(n)
    lib().orc_site_positions(kind, nx, ny, nz, a, _ptr(px, f64p), _ptr(py, f64p))
    return px, py


def voronoi_labels(kind, nx, ny, nz, periodic_xy, Q, seeds_xy, w_units) -> np.ndarray:
    seeds = np.ascontiguousarray(seeds_xy, dtype=np.int32).reshape(-1, 2)
    per = np.ascontiguousarray(periodic_xy, dtype=np.int32)
    lab = np.empty(lattice_sites(kind, nx, ny, nz), dtype=np.int32)
    lib().orc_voronoi_labels(kind, nx, ny, nz, _ptr(per, i32p), Q, _ptr(seeds, i32p), len(seeds),
                             int(w_units), _ptr(lab, i32p))
    return lab


# ---------------------------------------------------------------- dynamics
class System:
    """One lattice evolved by the oracle's Heun sLLG.

    Arrays are kept alive on the instance; ``S`` is float64[3, n_sites].
    """

    def __init__(self, *, row_ptr, col, shell, label, px, py, ctr0, n_shells, J, mu_s, alpha,
                 gamma, dt, ku, ku_grain=None, B=(0.0, 0.0, 0.0), bits=None, steps_per_bit=0,
                 spot_mode=SPOT_NONE, T_amb=0.0, T_peak=0.0, fwhm=0.0, x0=0.0, y0=0.0, v=0.0,
                 seed=1, rounds=10, sys_id=0, active=None, hx=0.0, origin=0, demag=None):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.shell = np.ascontiguousarray(shell, dtype=np.int8)
        self.label = np.ascontiguousarray(label, dtype=np.int32)
        self.px = np.ascontiguousarray(px, dtype=np.float64)
        self.py = np.ascontiguousarray(py, dtype=np.float64)
        self.ctr0 = np.ascontiguousarray(ctr0, dtype=np.uint32)
        self.ku_grain = None if ku_grain is None else np.ascontiguousarray(ku_grain, np.float64)
        self.bits = None if bits is None else np.ascontiguousarray(bits, dtype=np.uint8)
        self.active = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
        n = len(self.label)
        s = OrcSystem()
        s.n_sites = n
        s.row_ptr, s.col, s.shell = _ptr(self.row_ptr, i64p), _ptr(self.col, i32p), _ptr(self.shell, i8p)
        s.label = _ptr(self.label, i32p)
        s.active = _ptr(self.active, u8p)
        s.px, s.py = _ptr(self.px, f64p), _ptr(self.py, f64p)
        s.ctr0 = _ptr(self.ctr0, u32p)
        s.sys_id = sys_id
        s.hx, s.origin = hx, origin
        s.n_shells = n_shells
        for k in range(4):
            s.J[k] = J[k] if k < len(J) else 0.0
        s.mu_s, s.alpha, s.gamma, s.dt, s.ku = mu_s, alpha, gamma, dt, ku
        s.ku_grain = _ptr(self.ku_grain, f64p)
        for k in range(3):
            s.B[k] = B[k]
        s.n_bits = 0 if self.bits is None else len(self.bits)
        s.bits = _ptr(self.bits, u8p)
        s.steps_per_bit = steps_per_bit
        s.spot_mode = spot_mode
        s.T_amb, s.T_peak, s.fwhm, s.x0, s.y0, s.v = T_amb, T_peak, fwhm, x0, y0, v
        s.seed, s.rounds = seed, rounds
        self._s = s
        self.set_demag(demag)

    def set_demag(self, demag, stray=None, once=False):
        """demag = (dn, dd, dcell): coarse mesh (cells along x, y, z), cell
        edges (m) and the coarse cell of every site (-1 = none); None = off.
        stray: float[3, ncell] field (T) of sources outside the evolving sites,
        added to every cell's demagnetising field (None = none).  once: the
        field evaluated once per step from the step's starting spins and held
        through both Heun stages (else at both stages)."""
        s = self._s
        s.demag_once = 1 if once else 0
        self.bstray = None if stray is None else np.ascontiguousarray(stray, np.float64).reshape(-1)
        s.bstray = _ptr(self.bstray, f64p)
        if demag is None:
            self.dcell = None
            s.dn[0] = s.dn[1] = s.dn[2] = 0
            s.dcell = _ptr(None, i32p)
            return
        dn, dd, dcell = demag
        self.dcell = np.ascontiguousarray(dcell, dtype=np.int32)
        assert len(self.dcell) == len(self.label)
        for k in range(3):
            s.dn[k], s.dd[k] = int(dn[k]), float(dd[k])
        s.dcell = _ptr(self.dcell, i32p)

    def set_active(self, active, origin=None):
        self.active = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
        self._s.active = _ptr(self.active, u8p)
        if origin is not None:
            self._s.origin = origin

    def heun(self, S, step0: int, nsteps: int) -> np.ndarray:
        S = np.array(S, dtype=np.float64, copy=True).reshape(3, -1)
        Sx, Sy, Sz = (np.ascontiguousarray(S[k]) for k in range(3))
        rc = lib().orc_heun_steps(C.byref(self._s), _ptr(Sx, f64p), _ptr(Sy, f64p),
                                  _ptr(Sz, f64p), step0, nsteps)
        if rc != 0:
            raise MemoryError("oracle step allocation failed")
        return np.stack([Sx, Sy, Sz])

    def mc(self, S, colour, sweep0: int, nsweeps: int) -> np.ndarray:
        """Metropolis sweeps of the same Hamiltonian at T_amb (colour: int8 per
        site, 0 .. n-1 with no two neighbours alike, -1 = never visited)."""
        S = np.array(S, dtype=np.float64, copy=True).reshape(3, -1)
        Sx, Sy, Sz = (np.ascontiguousarray(S[k]) for k in range(3))
        col = np.ascontiguousarray(colour, dtype=np.int8)
        lib().orc_mc_sweeps(C.byref(self._s), _ptr(col, i8p), int(col.max()) + 1, _ptr(Sx, f64p),
                            _ptr(Sy, f64p), _ptr(Sz, f64p), sweep0, nsweeps)
        return np.stack([Sx, Sy, Sz])

    def magnetisation(self, S, n_grains: int):
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(3, -1)
        Sx, Sy, Sz = (np.ascontiguousarray(S[k]) for k in range(3))
        pg = np.zeros((max(n_grains, 1), 4))
        tot = np.zeros(4)
        lib().orc_magnetisation(C.byref(self._s), _ptr(Sx, f64p), _ptr(Sy, f64p), _ptr(Sz, f64p),
                                n_grains, _ptr(pg, f64p), _ptr(tot, f64p))
        return pg[:n_grains], tot

    def temperature(self, step: int, sites=None) -> np.ndarray:
        """Spot temperature (K) of the given sites (default: all) at `step`."""
        idx = range(len(self.label)) if sites is None else sites
        return np.array([lib().orc_site_temperature(C.byref(self._s), int(i), step) for i in idx])

    def polarity(self, step: int) -> float:
        return lib().orc_polarity(C.byref(self._s), step)

    def field(self, S, step: int, sites=None) -> np.ndarray:
        """Deterministic field (T) at the given sites, float[len, 3]: exchange,
        anisotropy and the polarised write field as a Heun stage assembles them
        (no thermal or demagnetising term)."""
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(3, -1)
        Sx, Sy, Sz = (np.ascontiguousarray(S[k]) for k in range(3))
        idx = range(len(self.label)) if sites is None else sites
        out = []
        for i in idx:
            b = np.zeros(3)
            lib().orc_field(C.byref(self._s), _ptr(Sx, f64p), _ptr(Sy, f64p), _ptr(Sz, f64p),
                            int(i), step, _ptr(b, f64p))
            out.append(b)
        return np.array(out).reshape(-1, 3)

    def energy(self, S, step: int) -> np.ndarray:
        S = np.ascontiguousarray(S, dtype=np.float64).reshape(3, -1)
        Sx, Sy, Sz = (np.ascontiguousarray(S[k]) for k in range(3))
        out = np.zeros(4)
        lib().orc_energy(C.byref(self._s), _ptr(Sx, f64p), _ptr(Sy, f64p), _ptr(Sz, f64p), step,
                         _ptr(out, f64p))
        return out


# ---------------------------------------------------------------- demagnetising field (Eq. 7)
MU0 = 1.25663706212e-6  # N/A^2 (CODATA 2018)


def newell_tensor(X, Y, Z, dx, dy, dz) -> np.ndarray:
    """Newell's cell-averaged demagnetising tensor (xx, yy, zz, xy, xz, yz)."""
    out = np.zeros(6)
    lib().orc_newell_tensor(X, Y, Z, dx, dy, dz, _ptr(out, f64p))
    return out


def demag_direct(M, nx, ny, nz, dx, dy, dz) -> np.ndarray:
    """Eq. 7 by direct summation: M float[3, nx*ny*nz] (A/m) -> H (A/m)."""
    M = np.ascontiguousarray(M, dtype=np.float64).reshape(3, -1)
    assert M.shape[1] == nx * ny * nz
    H = np.zeros_like(M)
    lib().orc_demag_direct(nx, ny, nz, dx, dy, dz, _ptr(M, f64p), _ptr(H, f64p))
    return H


def demag_field(S, dcell, dn, dd, mu_s) -> np.ndarray:
    """mu0 H_d (T) per coarse cell, float[3, ncell]: Eq. 6 (M = mu_s sum m / V over
    the sites with dcell = c) then Eq. 7 by direct summation."""
    S = np.asarray(S, dtype=np.float64).reshape(3, -1)
    dcell = np.asarray(dcell)
    nc = int(dn[0] * dn[1] * dn[2])
    M = np.zeros((3, nc))
    sel = dcell >= 0
    for k in range(3):
        np.add.at(M[k], dcell[sel], S[k, sel])
    M *= mu_s / (dd[0] * dd[1] * dd[2])
    return MU0 * demag_direct(M, int(dn[0]), int(dn[1]), int(dn[2]), *dd)


# ---------------------------------------------------------------- window-end transfer (Eq. 6)
def coarse_cells(ncols: int, ny: int, nz: int, cx: int, cy: int, cz: int) -> int:
    return -(-ncols // cx) * -(-ny // cy) * -(-nz // cz)


def coarse_grain(kind, sx, ny, nz, label, S, x0, ncols, cx, cy, cz) -> np.ndarray:
    """Per coarse cell (sum mx, sum my, sum mz, N magnetic sites) over stored
    columns [x0, x0 + ncols); cells of cx x cy x cz lattice cells."""
    S = np.ascontiguousarray(S, dtype=np.float64).reshape(3, -1)
    Sx, Sy, Sz = (np.ascontiguousarray(S[k]) for k in range(3))
    lab = np.ascontiguousarray(label, dtype=np.int32)
    out = np.zeros((coarse_cells(ncols, ny, nz, cx, cy, cz), 4))
    lib().orc_coarse_grain(kind, sx, ny, nz, _ptr(lab, i32p), _ptr(Sx, f64p), _ptr(Sy, f64p),
                           _ptr(Sz, f64p), x0, ncols, cx, cy, cz, _ptr(out, f64p))
    return out


def cone_theta_max(m: float) -> float:
    return lib().orc_cone_theta_max(float(m))


CONE_PRINTED, CONE_CAP = 0, 1  # cone readings of the inverse transfer (Sec. II)


def cone_spin(mvec, rounds, seed, site, step, sys, mode: int = CONE_PRINTED) -> np.ndarray:
    mv = np.ascontiguousarray(mvec, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_cone_spin_mode(mode, _ptr(mv, f64p), rounds, seed, site, step, sys, _ptr(out, f64p))
    return out


def cone_columns(kind, sx, ny, nz, label, S, x0, ncols, cx, cy, cz, mcell, rounds, seed, step,
                 sys, mode: int = CONE_PRINTED) -> np.ndarray:
    """S with the magnetic sites of columns [x0, x0 + ncols) replaced by cone
    spins around the reduced magnetisation of their coarse cell."""
    S = np.array(S, dtype=np.float64).reshape(3, -1)
    Sx, Sy, Sz = (np.ascontiguousarray(S[k]) for k in range(3))
    lab = np.ascontiguousarray(label, dtype=np.int32)
    mc = np.ascontiguousarray(mcell, dtype=np.float64).reshape(-1, 3)
    lib().orc_cone_columns_mode(mode, kind, sx, ny, nz, _ptr(lab, i32p), _ptr(Sx, f64p),
                                _ptr(Sy, f64p), _ptr(Sz, f64p), x0, ncols, cx, cy, cz,
                                _ptr(mc, f64p), rounds, seed, step, sys)
    return np.stack([Sx, Sy, Sz])


# ---------------------------------------------------------------- micromagnetic region
def langevin(x: float) -> float:
    return lib().orc_langevin(x)


def mm_me(T: float, Tc: float, b: float = 0.0) -> float:
    """Equilibrium reduced magnetisation m_e(T) (b = mu_s |B| / kB in kelvin)."""
    return lib().orc_mm_me(T, Tc, b)


class MM:
    """Micromagnetic LLG region integrated by RK4 (m float64[3, nx*ny*nz])."""

    def __init__(self, *, n, h, Ms0, A0, K0, lam, gamma, Tc, mu_s, dt, B=(0.0, 0.0, 0.0),
                 periodic=(0, 0, 0), bits=None, steps_per_bit=0, spot_mode=SPOT_NONE,
                 T_amb=0.0, T_peak=0.0, fwhm=0.0, x0=0.0, y0=0.0, v=0.0):
        p = OrcMM()
        p.nx, p.ny, p.nz = n
        for k in range(3):
            p.periodic[k] = int(periodic[k])
            p.h[k] = h[k]
            p.B[k] = B[k]
        p.Ms0, p.A0, p.K0, p.lambda_, p.gamma, p.Tc, p.mu_s, p.dt = (Ms0, A0, K0, lam, gamma, Tc,
                                                                      mu_s, dt)
        self.bits = None if bits is None else np.ascontiguousarray(bits, dtype=np.uint8)
        p.n_bits = 0 if self.bits is None else len(self.bits)
        p.bits = _ptr(self.bits, u8p)
        p.steps_per_bit = steps_per_bit
        p.spot_mode = spot_mode
        p.T_amb, p.T_peak, p.fwhm, p.x0, p.y0, p.v = T_amb, T_peak, fwhm, x0, y0, v
        self._p = p
        self.n = n[0] * n[1] * n[2]
        self.ghosts = [None, None]
        self.bd = None

    def set_ghost(self, face: int, dirs):
        """Direction [ny*nz, 3] of the region across x face `face` (0: -x, 1: +x)
        seen by the boundary cells' exchange stencil; None removes it."""
        self.ghosts[face] = None if dirs is None else np.ascontiguousarray(dirs, np.float64)
        self._p.ghost[face] = _ptr(self.ghosts[face], f64p)

    def set_field(self, bd):
        """A field (T) per cell [3, n] added at every RK4 stage and held through
        the step; None removes it."""
        self.bd = None if bd is None else np.ascontiguousarray(bd, np.float64).reshape(-1)
        assert self.bd is None or len(self.bd) == 3 * self.n
        self._p.bd = _ptr(self.bd, f64p)

    def equilibrium(self, t: float) -> np.ndarray:
        """m_e(T) of every cell (x fastest) at time t (s), T from the spot."""
        p = self._p
        bmag = math.sqrt((p.B[0] * p.B[0] + p.B[1] * p.B[1]) + p.B[2] * p.B[2])
        b = p.mu_s * bmag / KB
        me = np.empty(self.n)
        for c in range(self.n):
            i, j = c % p.nx, (c // p.nx) % p.ny
            me[c] = lib().orc_mm_me(self.temperature(i, j, t), p.Tc, b)
        return me

    def temperature(self, i: int, j: int, t: float) -> float:
        """Temperature (K) of cell (i, j) at time t (s)."""
        return lib().orc_mm_temperature(C.byref(self._p), i, j, t)

    def polarity(self, step: int) -> float:
        return lib().orc_mm_polarity(C.byref(self._p), step)

    def face(self, face: int, m) -> np.ndarray:
        """Directions [ny*nz, 3] of the boundary cells on x face `face`."""
        nx, ny, nz = self._p.nx, self._p.ny, self._p.nz
        M = np.asarray(m).reshape(3, nz, ny, nx)
        return np.ascontiguousarray(M[:, :, :, 0 if face == 0 else nx - 1].reshape(3, -1).T)

    def shift(self, m, enter, stride: int = 3):
        """The mesh moved one cell along +x with the window (Sec. II, Fig. 1):
        returns (m after the move, the leaving column [ny*nz, 3]); `enter`
        [ny*nz, stride] gives the new last column's directions."""
        flat = np.array(m, dtype=np.float64, copy=True).reshape(-1)
        ent = np.ascontiguousarray(enter, dtype=np.float64).reshape(-1)
        leave = np.zeros((self._p.ny * self._p.nz, 3))
        lib().orc_mm_shift(C.byref(self._p), _ptr(flat, f64p), _ptr(ent, f64p), stride,
                           _ptr(leave, f64p))
        return flat.reshape(3, -1), leave

    def face_moment(self, m, face: int, t: float) -> np.ndarray:
        """m_e(T) m of the cells on x face `face` at time t: [ny*nz, 3]."""
        flat = np.ascontiguousarray(m, dtype=np.float64).reshape(-1)
        out = np.zeros((self._p.ny * self._p.nz, 3))
        lib().orc_mm_face_moment(C.byref(self._p), _ptr(flat, f64p), face, t, _ptr(out, f64p))
        return out

    def rk4(self, m, step0: int, nsteps: int) -> np.ndarray:
        m = np.array(m, dtype=np.float64, copy=True).reshape(3, -1)
        assert m.shape[1] == self.n
        flat = np.ascontiguousarray(m.reshape(-1))
        if lib().orc_mm_rk4(C.byref(self._p), _ptr(flat, f64p), step0, nsteps) != 0:
            raise MemoryError("oracle allocation failed")
        return flat.reshape(3, -1)


def set_columns(kind, sx, ny, nz, label, S, x0, ncols, cx, cy, cz, mcell) -> np.ndarray:
    """Magnetic sites of columns [x0, x0 + ncols) take their coarse cell's direction."""
    S = np.array(S, dtype=np.float64, copy=True).reshape(3, -1)
    Sx, Sy, Sz = (np.ascontiguousarray(S[k]) for k in range(3))
    lab = np.ascontiguousarray(label, dtype=np.int32)
    mc = np.ascontiguousarray(mcell, dtype=np.float64)
    lib().orc_set_columns(kind, sx, ny, nz, _ptr(lab, i32p), _ptr(Sx, f64p), _ptr(Sy, f64p),
                          _ptr(Sz, f64p), x0, ncols, cx, cy, cz, _ptr(mc, f64p))
    return np.stack([Sx, Sy, Sz])


# ---------------------------------------------------------------- moving multiscale window
def multiscale_shift(kind, sx, ny, nz, label, S, org, nx, cell, left, mL, right, mR, enter,
                     rounds, seed, step, sys_id=0, t=None, mode: int = CONE_PRINTED):
    """One move of the multiscale simulation window by one coarse cell (cx
    lattice columns) along +x (Sec. II, Fig. 1), in the order:
      1. trailing end: the cx atomistic columns [org, org + cx) are averaged
         (Eq. 6) into the new last cell column of the left region, whose
         first column leaves for the track;
      2. the atomistic window moves: org -> org + cx;
      3. leading end: the right region's first cell column enters the
         atomistic window by thermalisation: the magnetic sites of columns
         [org + nx, org + nx + cx) (old origin) take cone spins around
         m_e(T) m of their cell (Eq. 6 read backwards), at time t (default
         step dt);
      4. the right region moves down one cell; its last column takes the
         directions `enter` [ny*nz, 3] of the track ahead.
    left / right: MM regions or None (then mL / mR are ignored).  Returns
    (S, new origin, mL, mR, the left region's leaving column or None)."""
    cx, cy, cz = cell
    S = np.array(S, dtype=np.float64, copy=True).reshape(3, -1)
    leave = None
    if left is not None:
        sums = coarse_grain(kind, sx, ny, nz, label, S, org, cx, cx, cy, cz)
        mL, leave = left.shift(mL, sums, stride=4)
    if right is not None:
        tt = step * right._p.dt if t is None else t
        mface = right.face_moment(mR, 0, tt)
        S = cone_columns(kind, sx, ny, nz, label, S, org + nx, cx, cx, cy, cz, mface, rounds,
                         seed, step, sys_id, mode=mode)
        mR, _ = right.shift(mR, enter, stride=3)
    return S, org + cx, mL, mR, leave


def multiscale_demag(left, mL, sums, ncx_atoms, right, mR, t, dd, mu_s):
    """Eq. 7 on the multiscale window of Fig. 1 (Sec. II): the left region's
    cells, the atomistic window's coarse cells and the right region's cells
    laid along x as one mesh of equal cells of edges dd (NX = nL + ncx_atoms
    + nR cells along x, x fastest).  Cell magnetisation (A/m): M_S0 m_e(T) m
    in a region cell (T of the cell at time t), mu_s (sum m) / V in an
    atomistic cell (sums: [ncell, >= 3] coarse-grain sums of the window,
    cells x fastest); left / right may be None.  Returns (B_all, B_regions):
    mu0 H_d in tesla, [3, NX ny nz], from every cell and from the regions'
    cells alone (Eq. 7 by direct summation)."""
    some = left if left is not None else right
    ny, nz = some._p.ny, some._p.nz
    nL = left._p.nx if left is not None else 0
    nR = right._p.nx if right is not None else 0
    NX = nL + ncx_atoms + nR
    V = (dd[0] * dd[1]) * dd[2]
    Mall = np.zeros((3, NX * ny * nz))
    Mreg = np.zeros((3, NX * ny * nz))
    sums = np.asarray(sums, np.float64)
    for k in range(nz):
        for j in range(ny):
            row = NX * (j + ny * k)
            for i in range(ncx_atoms):
                Mall[:, row + nL + i] = mu_s * sums[i + ncx_atoms * (j + ny * k), :3] / V
            for reg, m, off in ((left, mL, 0), (right, mR, nL + ncx_atoms)):
                if reg is None:
                    continue
                me = reg.equilibrium(t)
                m = np.asarray(m, np.float64).reshape(3, -1)
                for i in range(reg._p.nx):
                    c = i + reg._p.nx * (j + ny * k)
                    v = reg._p.Ms0 * me[c] * m[:, c]
                    Mall[:, row + off + i] = v
                    Mreg[:, row + off + i] = v
    Ball = MU0 * demag_direct(Mall, NX, ny, nz, *dd)
    Breg = MU0 * demag_direct(Mreg, NX, ny, nz, *dd)
    return Ball, Breg


def mesh_part(B, NX, ny, nz, x0, nx):
    """Cells [x0, x0 + nx) along x of a field [3, NX ny nz]: [3, nx ny nz]."""
    return np.ascontiguousarray(np.asarray(B).reshape(3, nz, ny, NX)[:, :, :, x0:x0 + nx]
                                .reshape(3, -1))
