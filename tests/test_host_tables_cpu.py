"""Host logic of the library against the oracle, on the CPU: grain labels and
neighbour tables are bit-exact (these are the tables the kernels run on)."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle_build import oracle_labels
from paper_2502_02236_amd import asd as A
from paper_2502_02236_amd import bridge


def _pair(w):
    return bridge.params_for(w, A.ASD_FP32), bridge.SystemInputs(w)


@pytest.mark.parametrize("name,w", [
    ("slab", W.c2_granular_slab().scaled(nz=2)),
    ("l10", W.c3_l10_window().scaled(nz=2)),
    ("track", W.c5_track_window().scaled(nz=2)),
    ("slab_small_grains", W.c2_granular_slab().scaled(nx=60, ny=52, nz=3, grain_pitch=3e-9)),
])
def test_host_labels_match_oracle(name, w):
    p, si = _pair(w)
    n = w.n_sites if not w.track_nx else (w.track_nx * w.ny * w.nz)
    got = A.asd_host_grain_labels(p, si.desc, n)
    np.testing.assert_array_equal(got, oracle_labels(w))


@pytest.mark.parametrize("name,w", [
    ("sc_periodic", W.c1_plain_sc()),
    ("sc_open", W.c1_plain_sc().scaled(bc=(0, 0, 0), nx=7, ny=5, nz=4)),
    ("sc_track", W.c5_track_window().scaled(nx=9, ny=6, nz=3, track_nx=15)),
    ("l10_periodic", W.c3_l10_window().scaled(nx=6, ny=5, nz=4)),
    ("l10_open", W.c3_l10_window().scaled(nx=5, ny=4, nz=3, bc=(0, 0, 0))),
    ("l10_two_shells", W.c3_l10_window().scaled(nx=6, ny=5, nz=4, J=(6.0e-21, 1.2e-21))),
])
def test_host_neighbours_match_oracle(name, w):
    p, si = _pair(w)
    row, col, sh = A.asd_host_neighbours(p, si.desc)
    nx = w.track_nx or w.nx
    per = [int(b == W.BC_PERIODIC) for b in w.bc]
    r2, c2, s2 = oracle.neighbours(w.kind, nx, w.ny, w.nz, per, w.a, w.c, w.shell_radii)
    np.testing.assert_array_equal(row, r2)
    np.testing.assert_array_equal(col, c2)
    np.testing.assert_array_equal(sh, s2)


def test_thin_boundaries_are_reported():
    """Grain boundaries thinner than the neighbour range would let two grains
    exchange-couple through a bond: the library reports it (the kernels rely on
    non-magnetic boundaries)."""
    w = W.c2_granular_slab().scaled(nx=40, ny=40, nz=1, boundary_w=0.1e-9)
    p, si = _pair(w)
    import ctypes as C
    lab = np.empty(w.n_sites, dtype=np.int32)
    rc = A.lib().asd_host_grain_labels(C.byref(p), C.byref(si.desc), lab.ctypes.data_as(C.c_void_p))
    assert rc == A.ASD_EUNSUPPORTED
