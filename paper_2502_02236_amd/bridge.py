"""Workload definitions -> libasd descriptors (argument marshalling only)."""
from __future__ import annotations

import numpy as np

import workloads as W

from . import asd as A


def params_for(w: W.Workload, precision: int, kernel: int = A.ASD_KERNEL_PLAIN,
               graph_steps: int = 0, rounds: int = 10, demag_cell=(0, 0, 0)) -> A.asd_params:
    p = A.asd_params()
    p.lattice = A.ASD_SC if w.kind == W.SC else A.ASD_L10
    p.precision = precision
    p.a, p.c = w.a, w.c
    p.n_shells = len(w.J)
    for k, j in enumerate(w.J):
        p.J[k] = j
    p.mu_s, p.alpha, p.gamma, p.dt, p.k_u = w.mu_s, w.alpha, w.gamma, w.dt, w.ku
    p.seed = w.seed
    p.philox_rounds = rounds
    p.kernel = kernel
    p.graph_steps = graph_steps
    for k in range(3):
        p.demag_cell[k] = demag_cell[k]
    return p


class SystemInputs:
    """Holds the host arrays a descriptor points to (alive until create returns)."""

    def __init__(self, w: W.Workload, seeds=None, labels=None, ku_grain=None, T_system=-1.0):
        self.w = w
        d = A.asd_system_desc()
        d.nx, d.ny, d.nz = w.nx, w.ny, w.nz
        d.bc_x, d.bc_y, d.bc_z = w.bc
        d.track_nx = w.track_nx
        self.seeds = None
        self.labels = None
        self.ku = None
        if labels is not None:
            self.labels = np.ascontiguousarray(labels, dtype=np.int32)
            d.labels = self.labels.ctypes.data_as(A.C.POINTER(A.C.c_int32))
        elif w.grains:
            self.seeds = np.ascontiguousarray(
                seeds if seeds is not None else W.voronoi_seeds(w), dtype=np.int32)
            d.n_seeds = len(self.seeds)
            d.seeds_xy = self.seeds.ctypes.data_as(A.C.POINTER(A.C.c_int32))
            d.voronoi_q = W.Q_UNITS
            d.boundary_w_units = w.w_units
        if ku_grain is not None:
            self.ku = np.ascontiguousarray(ku_grain, dtype=np.float64)
            d.k_u_grain = self.ku.ctypes.data_as(A.C.POINTER(A.C.c_double))
            d.n_k_u_grain = len(self.ku)
        d.T_system = T_system
        self.desc = d


def drive_for(w: W.Workload, T_amb=None) -> tuple:
    dr = A.asd_drive()
    for k in range(3):
        dr.B[k] = w.B[k]
    bits = None
    if w.bits:
        bits = np.ascontiguousarray(w.bits, dtype=np.uint8)
        dr.n_bits = len(bits)
        dr.bits = bits.ctypes.data_as(A.C.POINTER(A.C.c_uint8))
        dr.steps_per_bit = w.steps_per_bit
    dr.spot_mode = w.spot_mode
    dr.T_amb = w.T_amb if T_amb is None else T_amb
    dr.T_peak, dr.fwhm, dr.x0, dr.y0, dr.v = w.T_peak, w.fwhm, w.x0, w.y0, w.v
    return dr, bits


def make_handle(w: W.Workload, precision: int, kernel: int = A.ASD_KERNEL_PLAIN, graph_steps=0,
                n_systems: int = 1, seeds=None, labels=None, ku_grain=None, T_amb=None,
                device="cuda:0", demag_cell=(0, 0, 0)) -> A.Handle:
    """A handle stepping n_systems copies of workload w (same grains, system ids 0..n-1)."""
    ins = [SystemInputs(w, seeds=seeds, labels=labels, ku_grain=ku_grain) for _ in range(n_systems)]
    h = A.Handle(params_for(w, precision, kernel, graph_steps, demag_cell=demag_cell),
                 [i.desc for i in ins], device=device)
    dr, bits = drive_for(w, T_amb)
    h.set_drive(dr)
    h._inputs = ins
    return h
