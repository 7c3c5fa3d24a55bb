"""GPU parity of the demagnetising field (Eq. 7 on the coarse cells of Eq. 6).

The library convolves by zero-padded FFTs with the spectrum of Newell's tensor;
the oracle sums Eq. 7 directly.  Bars:
  * the field per coarse cell: FP64 within the tensor's own rounding bar
    (fp64_field_tol, 1e-11 of mu0 Ms for the small meshes), FP32 within 5e-7 of
    mu0 Ms.  The FP64 bar is set by the tensor itself: each entry is a 27-term
    difference of Newell's functions, whose terms grow like R^3 while the entry
    falls like R^-3, so two correct evaluations in a different order differ by
    ~27 eps (R/d)^3 / 4 pi per entry: ~1e-14 at the R <= 10 cells of the small
    meshes, up to ~1e-9 across a 256-cell mesh.  FP32: the cell sums
    and the FFT stages (radix 4, one radix-2 stage for odd log2 P) each round
    at ~6e-8 relative.
  * spins after Heun steps with the field: the FP64 and FP32 bars of the
    other parity tests (1e-12, 1e-4 per component).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from oracle_build import demag_cells, oracle_labels, oracle_system, track_stray, window_mask
from paper_2502_02236_amd import asd as A
from paper_2502_02236_amd import bridge

pytestmark = pytest.mark.gpu

FIELD_TOL = {A.ASD_FP64: 1e-11, A.ASD_FP32: 5e-7}
SPIN_TOL = {A.ASD_FP64: 1e-12, A.ASD_FP32: 1e-4}


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


def mu0_ms(w):
    zc = w.a if w.kind == W.SC else w.c
    per = 1 if w.kind == W.SC else 2
    return oracle.MU0 * w.mu_s * per / (w.a * w.a * zc)


def sc_slab(**kw):
    w = W.c2_granular_slab().scaled(nx=37, ny=29, nz=7, x0=5e-9, y0=4e-9, grain_pitch=4.0e-9,
                                    steps=40)
    return w.scaled(**kw)


def l10_slab(**kw):
    w = W.c3_l10_window().scaled(nx=13, ny=11, nz=6, x0=2e-9, y0=2e-9, grain_pitch=3.0e-9,
                                 steps=40)
    return w.scaled(**kw)


def track(**kw):
    w = W.c5_track_window().scaled(nx=30, ny=20, nz=5, track_nx=48, steps_per_bit=25,
                                   x0=4.5e-9, y0=3e-9, grain_pitch=3.0e-9)
    return w.scaled(**kw)


# (name, workload, coarse cell, systems)
FIELD_CASES = [
    ("sc_4x4x2_ragged", sc_slab(), (4, 4, 2), 1),
    ("sc_1x1x1_atomistic", sc_slab(nx=9, ny=7, nz=4), (1, 1, 1), 1),
    ("sc_single_layer", sc_slab(), (5, 3, 7), 2),
    ("sc_one_cell", sc_slab(nx=8, ny=6, nz=3), (8, 6, 3), 1),
    ("l10_3x3x2", l10_slab(), (3, 3, 2), 2),
    ("track_window_5x4x5", track(), (5, 4, 5), 2),
    # meshes 5 x 4 x ncz: z transforms of 16, 32 and 64 points
    ("sc_ncz7", sc_slab(nx=10, ny=8, nz=7), (2, 2, 1), 1),
    ("sc_ncz11", sc_slab(nx=10, ny=8, nz=11), (2, 2, 1), 1),
    ("sc_ncz15", sc_slab(nx=10, ny=8, nz=15), (2, 2, 1), 1),
    ("sc_ncz20", sc_slab(nx=10, ny=8, nz=20), (2, 2, 1), 2),
    # the largest mesh along x (256 cells, FFT length 512) and a long y axis
    ("sc_max_x_256", sc_slab(nx=256, ny=8, nz=3, grains=False), (1, 2, 3), 1),
    ("sc_y_255", sc_slab(nx=4, ny=255, nz=2, grains=False, bc=(1, 0, 0)), (2, 1, 1), 1),
]


def fp64_field_tol(dn, dd):
    """FP64 bar for a mesh of dn cells of size dd: a tensor entry at
    displacement R is a 27-term difference of Newell's functions whose terms are
    ~R^3 while the entry is ~R^-3, so two correct evaluations in a different
    order differ by up to ~27 eps (R / d_min)^3 / 4 pi of mu0 Ms; the bar takes
    that at the mesh's longest displacement, and never less than 1e-11."""
    eps = np.finfo(np.float64).eps
    R = math.sqrt(sum(((n - 1) * d) ** 2 for n, d in zip(dn, dd))) / min(dd)
    return max(1e-11, 27 * eps * R ** 3 / (4 * math.pi))


def random_state(w, labels, seed):
    S = W.random_spins(len(labels), seed)
    S[:, labels < 0] = 0.0
    return S


@pytest.mark.parametrize("prec", [A.ASD_FP64, A.ASD_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("name,w,cell,n_sys", FIELD_CASES, ids=[c[0] for c in FIELD_CASES])
def test_demag_field_matches_direct_sum(name, w, cell, n_sys, prec):
    say(f"[demag field] {name} cell={cell} systems={n_sys} prec={prec}")
    h = bridge.make_handle(w, prec, n_systems=n_sys, demag_cell=cell)
    lab = h.labels()
    states = [random_state(w, lab, 11 + s) for s in range(n_sys)]
    if name.startswith("track"):
        h.shift_window(7)  # the mesh follows the window
    for s, S in enumerate(states):
        h.set_spins(S, s)
    got, mesh = h.demag_field()
    dn, dd, dcell = demag_cells(w, cell, origin=7 if name.startswith("track") else 0)
    assert mesh == tuple(dn)
    scale = mu0_ms(w)
    for s, S in enumerate(states):
        ref = oracle.demag_field(S, dcell, dn, dd, w.mu_s)
        if name.startswith("track"):  # + the field of the frozen track
            ref = ref + track_stray(w, cell, 7, S)
        err = float(np.max(np.abs(got[s] - ref))) / scale
        tol = fp64_field_tol(dn, dd) if prec == A.ASD_FP64 else FIELD_TOL[prec]
        say(f"  system {s}: max |B_gpu - B_oracle| / mu0 Ms = {err:.3e} (bar {tol:.1e}; "
            f"|B| max {np.max(np.abs(ref)):.3f} T)")
        assert err <= tol, (name, s, err)
    h.close()


@pytest.mark.parametrize("prec", [A.ASD_FP64, A.ASD_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("origin", [0, 3, 10, 18])
def test_track_stray_field_matches_direct_sum(prec, origin):
    """Field of the frozen track at the window cells, for window origins aligned
    and not aligned with the coarse cells, up to the far end of the track."""
    w = track()
    cell = (4, 5, 2)
    h = bridge.make_handle(w, prec, demag_cell=cell, n_systems=2)
    lab = h.labels()
    states = [random_state(w, lab, 31 + s) for s in range(2)]
    if origin:
        h.shift_window(origin)
    for s, S in enumerate(states):
        h.set_spins(S, s)
    got, _ = h.demag_field()
    dn, dd, dcell = demag_cells(w, cell, origin)
    for s, S in enumerate(states):
        stray = track_stray(w, cell, origin, S)
        ref = oracle.demag_field(S, dcell, dn, dd, w.mu_s) + stray
        err = float(np.max(np.abs(got[s] - ref))) / mu0_ms(w)
        say(f"[stray] origin={origin} prec={prec} system {s}: err {err:.3e}, "
            f"|stray| max {np.max(np.abs(stray)):.4f} T")
        assert err <= FIELD_TOL[prec]
        assert np.max(np.abs(stray)) > 1e-3  # the track's field is not negligible
    h.close()


def test_demag_uniform_plate_is_minus_mu0_ms():
    """Saturated thin plate, one coarse cell per lattice cell across a wide window:
    far from the edges the field is close to -mu0 Ms along z (thin-film limit)."""
    w = sc_slab(nx=64, ny=64, nz=1, grains=False, bc=(0, 0, 0))
    h = bridge.make_handle(w, A.ASD_FP64, demag_cell=(1, 1, 1))
    got, mesh = h.demag_field()  # spins start at +z
    B = got[0].reshape(3, 1, 64, 64)
    centre = B[2, 0, 28:36, 28:36]
    assert np.all(centre < -0.9 * mu0_ms(w)) and np.all(centre > -mu0_ms(w))
    h.close()


# (name, workload, coarse cell, systems, precision)
STEP_CASES = [
    ("sc_fp64", sc_slab(), (4, 4, 2), 1, A.ASD_FP64),
    ("sc_fp32", sc_slab(), (4, 4, 2), 2, A.ASD_FP32),
    ("l10_fp64", l10_slab(), (3, 3, 2), 1, A.ASD_FP64),
    ("l10_fp32", l10_slab(), (3, 3, 3), 1, A.ASD_FP32),
    # 20 planes of cells (z transforms of 64 points)
    ("sc_fp64_ncz20", sc_slab(nz=20), (4, 4, 1), 1, A.ASD_FP64),
]


@pytest.mark.parametrize("variant", [0, 1, 2], ids=["recompute", "stash", "cellrows"])
@pytest.mark.parametrize("name,w,cell,n_sys,prec", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_heun_with_demag_matches_oracle(name, w, cell, n_sys, prec, variant):
    """Variant 2 forms the cell sums in the step kernels: with graph segments of
    ten steps, nine of every ten field evaluations start from those sums."""
    steps = 40
    say(f"[demag heun] {name} cell={cell} variant={variant} steps={steps}")
    h = bridge.make_handle(w, prec, n_systems=n_sys, demag_cell=cell, graph_steps=10)
    h.set_variant(A.ASD_KERNEL_PLAIN, variant)
    lab = h.labels()
    S0 = [random_state(w, lab, 21 + s) for s in range(n_sys)]
    for s in range(n_sys):
        h.set_spins(S0[s], s)
    h.step(steps)
    dn, dd, dcell = demag_cells(w, cell)
    for s in range(n_sys):
        sysm = oracle_system(w, labels=oracle_labels(w), sys_id=s)
        sysm.set_demag((dn, dd, dcell))
        ref = sysm.heun(S0[s], 0, steps)
        err = float(np.max(np.abs(h.get_spins(s).astype(np.float64) - ref)))
        say(f"  system {s}: max |dS| = {err:.3e}")
        assert err <= SPIN_TOL[prec], (name, s, err)
        # the field mattered: without it the oracle lands far from both
        if s == 0:
            plain = oracle_system(w, labels=oracle_labels(w), sys_id=s).heun(S0[s], 0, steps)
            assert float(np.max(np.abs(plain - ref))) > 100 * max(err, 1e-15)
    h.close()


@pytest.mark.parametrize("kernel,variant,once", [(A.ASD_KERNEL_PLAIN, 0, False),
                                                 (A.ASD_KERNEL_PLAIN, 2, False),
                                                 (A.ASD_KERNEL_FUSED, 0, False),
                                                 (A.ASD_KERNEL_FUSED, 0, True)],
                         ids=["recompute", "cellrows", "fused_stages", "fused_once"])
@pytest.mark.parametrize("prec,cell", [(A.ASD_FP64, (5, 4, 5)), (A.ASD_FP32, (5, 4, 5)),
                                       (A.ASD_FP64, (4, 3, 2)), (A.ASD_FP32, (7, 6, 3))],
                         ids=["fp64_5x4x5", "fp32_5x4x5", "fp64_4x3x2", "fp32_7x6x3_ragged"])
def test_track_with_demag_and_shifts(prec, cell, kernel, variant, once):
    """Moving window: the demagnetising mesh moves with the window and the frozen
    track's stray field is recomputed after every shift; graph-captured segments
    (the demag kernels are plain launches, no memset nodes) replayed."""
    w = track()
    shifts = [(10, 1), (20, 2)]
    steps = 40
    h = bridge.make_handle(w, prec, demag_cell=cell, graph_steps=10, kernel=kernel)
    h.set_variant(kernel, variant)
    if once:
        h.set_demag_reading(A.ASD_DEMAG_ONCE)
    lab = h.labels()
    S0 = random_state(w, lab, 5)
    h.set_spins(S0)
    done = 0
    for at, cols in shifts + [(steps, 0)]:
        h.step(at - done)
        done = at
        if cols:
            h.shift_window(cols)
    org = 0
    sysm = oracle_system(w, labels=lab, active=window_mask(w, 0), origin=0)
    S = np.array(S0, dtype=np.float64)
    done = 0
    for at, cols in shifts + [(steps, 0)]:
        dn, dd, dcell = demag_cells(w, cell, origin=org)
        sysm.set_demag((dn, dd, dcell), stray=track_stray(w, cell, org, S), once=once)
        S = sysm.heun(S, done, at - done)
        done = at
        if cols:
            org += cols
            sysm.set_active(window_mask(w, org), org)
    err = float(np.max(np.abs(h.get_spins().astype(np.float64) - S)))
    say(f"[demag track] prec={prec} cell={cell} max |dS| = {err:.3e}")
    assert err <= SPIN_TOL[prec]
    h.close()


@pytest.mark.parametrize("prec", [A.ASD_FP64, A.ASD_FP32], ids=["fp64", "fp32"])
def test_cell_rows_match_two_pass_over_100_steps(prec):
    """The cell-row kernels against the two-pass kernels that sum the spins in
    the field pass, 100 steps from the same state: three workgroups per layer
    of cells along x (the last one ragged), ragged cells along y and z, graph
    segments of ten steps and a tail of plain launches.  The per-site
    arithmetic is the same; only the order of the cell sums differs."""
    w = sc_slab(nx=150, ny=13, nz=5)
    cell = (2, 3, 2)
    out = {}
    for variant in (0, 2):
        h = bridge.make_handle(w, prec, demag_cell=cell, graph_steps=10)
        h.set_variant(A.ASD_KERNEL_PLAIN, variant)
        S0 = random_state(w, h.labels(), 77)
        h.set_spins(S0)
        h.step(95)
        h.step(5)
        out[variant] = h.get_spins().astype(np.float64)
        h.close()
    err = float(np.max(np.abs(out[2] - out[0])))
    bar = 1e-12 if prec == A.ASD_FP64 else 1e-4
    say(f"[cell rows vs two-pass] prec={prec}: max |dS| after 100 steps = {err:.3e} (bar {bar:.0e})")
    assert err <= bar


# (name, workload, coarse cell, precision, fused variants): tiles narrower than
# a cell (14 interior columns), z chunks of 8 and 11 planes cutting layers of
# cells, one chunk, and the widest tiles
FUSED_STAGE_CASES = [
    ("sc_fp64_chunks", sc_slab(nz=20), (4, 3, 3), A.ASD_FP64, [0, 1, 5]),
    ("sc_fp32_chunks", sc_slab(nz=20), (4, 3, 3), A.ASD_FP32, [0, 2, 12, 14]),
    ("sc_fp32_2sys", sc_slab(), (5, 4, 2), A.ASD_FP32, [0, 9]),
    ("sc_fp32_wide_cells", sc_slab(nx=70), (20, 7, 7), A.ASD_FP32, [2, 14]),
]


@pytest.mark.parametrize("name,w,cell,prec,variants", FUSED_STAGE_CASES,
                         ids=[c[0] for c in FUSED_STAGE_CASES])
def test_fused_stages_with_demag_match_oracle(name, w, cell, prec, variants):
    """The fused kernel as predictor and corrector stages with the field between
    them: each stage adds its field at the site's cell and writes per-tile parts
    of the cell sums for the next evaluation.  Graph segments of ten steps: nine
    of every ten evaluations start from those parts."""
    steps = 30
    n_sys = 2 if "2sys" in name else 1
    dn, dd, dcell = demag_cells(w, cell)
    refs = []
    S0 = None
    for v in variants:
        h = bridge.make_handle(w, prec, n_systems=n_sys, demag_cell=cell, graph_steps=10,
                               kernel=A.ASD_KERNEL_FUSED)
        h.set_variant(A.ASD_KERNEL_FUSED, v)
        lab = h.labels()
        if S0 is None:
            S0 = [random_state(w, lab, 31 + s) for s in range(n_sys)]
            for s in range(n_sys):
                sysm = oracle_system(w, labels=oracle_labels(w), sys_id=s)
                sysm.set_demag((dn, dd, dcell))
                refs.append(sysm.heun(S0[s], 0, steps))
        for s in range(n_sys):
            h.set_spins(S0[s], s)
        h.step(steps)
        for s in range(n_sys):
            err = float(np.max(np.abs(h.get_spins(s).astype(np.float64) - refs[s])))
            say(f"[fused stages] {name} variant {v} ({h.variant_name()}) system {s}: "
                f"max |dS| = {err:.3e}")
            assert err <= SPIN_TOL[prec], (name, v, s, err)
        h.close()


@pytest.mark.parametrize("prec", [A.ASD_FP64, A.ASD_FP32], ids=["fp64", "fp32"])
def test_fused_stages_match_two_pass_over_100_steps(prec):
    """The fused stage kernels against the two-pass kernels over 100 steps from
    the same state (FP64 within 1e-12)."""
    w = sc_slab(nx=150, ny=13, nz=9)
    cell = (2, 3, 2)
    out = {}
    for kernel, variant in ((A.ASD_KERNEL_PLAIN, 0), (A.ASD_KERNEL_FUSED, 0)):
        h = bridge.make_handle(w, prec, demag_cell=cell, graph_steps=10, kernel=kernel)
        h.set_variant(kernel, variant)
        S0 = random_state(w, h.labels(), 78)
        h.set_spins(S0)
        h.step(95)
        h.step(5)
        out[kernel] = h.get_spins().astype(np.float64)
        h.close()
    err = float(np.max(np.abs(out[A.ASD_KERNEL_FUSED] - out[A.ASD_KERNEL_PLAIN])))
    bar = 1e-12 if prec == A.ASD_FP64 else 1e-4
    say(f"[fused stages vs two-pass] prec={prec}: max |dS| after 100 steps = {err:.3e}")
    assert err <= bar


# the field evaluated once per step and held through both stages:
# (name, workload, coarse cell, precision, kernel, variant)
ONCE_CASES = [
    ("sc_fp64_recompute", sc_slab(), (4, 4, 2), A.ASD_FP64, A.ASD_KERNEL_PLAIN, 0),
    ("sc_fp64_cellrows", sc_slab(), (4, 4, 2), A.ASD_FP64, A.ASD_KERNEL_PLAIN, 2),
    ("sc_fp64_fused_chunks", sc_slab(nz=20), (4, 3, 3), A.ASD_FP64, A.ASD_KERNEL_FUSED, 0),
    ("sc_fp32_fused_wide", sc_slab(nz=20), (4, 3, 3), A.ASD_FP32, A.ASD_KERNEL_FUSED, 14),
    ("sc_fp32_fused_narrow", sc_slab(), (5, 4, 2), A.ASD_FP32, A.ASD_KERNEL_FUSED, 2),
    ("l10_fp64_cellrows", l10_slab(), (3, 3, 2), A.ASD_FP64, A.ASD_KERNEL_PLAIN, 2),
]


@pytest.mark.parametrize("name,w,cell,prec,kernel,variant", ONCE_CASES,
                         ids=[c[0] for c in ONCE_CASES])
def test_demag_once_per_step_matches_oracle(name, w, cell, prec, kernel, variant):
    """ASD_DEMAG_ONCE against the oracle's held field: the fused kernel runs the
    step in one launch with the field of S and writes the cell sums of the new
    spins for the next step's field; graph segments of ten steps."""
    steps = 30
    h = bridge.make_handle(w, prec, demag_cell=cell, graph_steps=10, kernel=kernel)
    h.set_variant(kernel, variant)
    h.set_demag_reading(A.ASD_DEMAG_ONCE)
    if kernel == A.ASD_KERNEL_FUSED:
        assert h.variant_name().endswith(", 3>")
    lab = h.labels()
    S0 = random_state(w, lab, 61)
    h.set_spins(S0)
    h.step(steps)
    dn, dd, dcell = demag_cells(w, cell)
    sysm = oracle_system(w, labels=oracle_labels(w))
    sysm.set_demag((dn, dd, dcell), once=True)
    ref = sysm.heun(S0, 0, steps)
    err = float(np.max(np.abs(h.get_spins().astype(np.float64) - ref)))
    say(f"[demag once] {name} ({h.variant_name()}): max |dS| = {err:.3e}")
    assert err <= SPIN_TOL[prec], (name, err)
    # the reading matters: the field at both stages lands far outside the FP64 bar
    if prec == A.ASD_FP64:
        each = oracle_system(w, labels=oracle_labels(w))
        each.set_demag((dn, dd, dcell))
        assert float(np.max(np.abs(each.heun(S0, 0, steps) - ref))) > 100 * max(err, 1e-13)
    h.close()


def test_demag_once_fused_matches_two_pass_over_100_steps():
    """FP64: the one-launch fused step with the held field against the two-pass
    kernels with the same reading, 100 steps (within 1e-12); then back to the
    field at both stages on the same handle."""
    w = sc_slab(nx=150, ny=13, nz=9)
    cell = (2, 3, 2)
    out = {}
    for kernel in (A.ASD_KERNEL_PLAIN, A.ASD_KERNEL_FUSED):
        h = bridge.make_handle(w, A.ASD_FP64, demag_cell=cell, graph_steps=10, kernel=kernel)
        h.set_variant(kernel, 0)
        h.set_demag_reading(A.ASD_DEMAG_ONCE)
        S0 = random_state(w, h.labels(), 79)
        h.set_spins(S0)
        h.step(95)
        h.step(5)
        out[kernel] = h.get_spins().astype(np.float64)
        h.set_demag_reading(A.ASD_DEMAG_EACH_STAGE)
        assert "1>+k_fused_sc" in h.variant_name() or kernel == A.ASD_KERNEL_PLAIN
        h.close()
    err = float(np.max(np.abs(out[A.ASD_KERNEL_FUSED] - out[A.ASD_KERNEL_PLAIN])))
    say(f"[demag once fused vs two-pass] max |dS| after 100 steps = {err:.3e}")
    assert err <= 1e-12


def test_demag_reading_errors():
    w = sc_slab()
    h = bridge.make_handle(w, A.ASD_FP32, demag_cell=(2, 2, 2))
    with pytest.raises(A.AsdError) as e:
        h.set_demag_reading(2)
    assert e.value.code == A.ASD_EINVAL
    h.close()
    h = bridge.make_handle(w, A.ASD_FP32)
    with pytest.raises(A.AsdError) as e:
        h.set_demag_reading(A.ASD_DEMAG_ONCE)
    assert e.value.code == A.ASD_ESTATE
    h.close()


def test_track_stray_field_at_the_largest_track():
    """The track mesh at its limit: 254 coarse columns along the stored track."""
    w = track(track_nx=254 * 2, nx=40, ny=6, nz=2, grains=False)
    cell = (2, 3, 2)
    for prec in (A.ASD_FP64, A.ASD_FP32):
        h = bridge.make_handle(w, prec, demag_cell=cell)
        lab = h.labels()
        S = random_state(w, lab, 41)
        h.shift_window(101)
        h.set_spins(S)
        got, _ = h.demag_field()
        dn, dd, dcell = demag_cells(w, cell, 101)
        ref = oracle.demag_field(S, dcell, dn, dd, w.mu_s) + track_stray(w, cell, 101, S)
        err = float(np.max(np.abs(got[0] - ref))) / mu0_ms(w)
        nt = -(-w.track_nx // cell[0]) + 2
        tol = fp64_field_tol((nt, dn[1], dn[2]), dd) if prec == A.ASD_FP64 else FIELD_TOL[prec]
        say(f"[stray max track] prec={prec}: err {err:.3e} (bar {tol:.1e})")
        assert err <= tol
        h.close()
    with pytest.raises(A.AsdError) as e:
        bridge.make_handle(track(track_nx=254 * 2 + 1, nx=40, ny=6, nz=2, grains=False), A.ASD_FP32,
                           demag_cell=cell)
    assert e.value.code == A.ASD_EUNSUPPORTED


def test_demag_error_paths():
    w = sc_slab()
    with pytest.raises(A.AsdError) as e:
        bridge.make_handle(w, A.ASD_FP32, demag_cell=(2, 0, 2))
    assert e.value.code == A.ASD_EINVAL
    with pytest.raises(A.AsdError) as e:
        bridge.make_handle(w.scaled(nx=600), A.ASD_FP32, demag_cell=(2, 1, 1))
    assert e.value.code == A.ASD_EUNSUPPORTED
    # the fused stage kernels: SC with open z; L1_0 and periodic z take the two-pass kernels
    for wl in (l10_slab(), w.scaled(bc=(0, 0, 1))):
        with pytest.raises(A.AsdError) as e:
            bridge.make_handle(wl, A.ASD_FP32, kernel=A.ASD_KERNEL_FUSED, demag_cell=(2, 2, 2))
        assert e.value.code == A.ASD_EUNSUPPORTED
        h = bridge.make_handle(wl, A.ASD_FP32, kernel=A.ASD_KERNEL_AUTO, demag_cell=(2, 2, 2))
        assert h.variant() == (A.ASD_KERNEL_PLAIN, 2)
        assert h.variant_name().startswith("k_cell_step")
        with pytest.raises(A.AsdError) as e:
            h.set_variant(A.ASD_KERNEL_FUSED, 0)
        assert e.value.code == A.ASD_EUNSUPPORTED
        h.close()
    h = bridge.make_handle(w, A.ASD_FP32, kernel=A.ASD_KERNEL_AUTO, demag_cell=(2, 2, 2))
    assert h.variant() == (A.ASD_KERNEL_FUSED, 0)
    h.set_variant(A.ASD_KERNEL_PLAIN, 2)
    assert h.variant_name().startswith("k_cell_step")
    h.close()
    h = bridge.make_handle(w, A.ASD_FP32)
    with pytest.raises(A.AsdError) as e:
        h.demag_field()
    assert e.value.code == A.ASD_ESTATE
    # the cell-row kernels need the field, and cells at most 64 lattice cells wide
    with pytest.raises(A.AsdError) as e:
        h.set_variant(A.ASD_KERNEL_PLAIN, 2)
    assert e.value.code == A.ASD_EUNSUPPORTED
    h.close()
    h = bridge.make_handle(w.scaled(nx=130), A.ASD_FP32, demag_cell=(65, 2, 2))
    assert h.variant() == (A.ASD_KERNEL_PLAIN, 0)
    with pytest.raises(A.AsdError) as e:
        h.set_variant(A.ASD_KERNEL_PLAIN, 2)
    assert e.value.code == A.ASD_EUNSUPPORTED
    h.close()
    # systems of different window sizes cannot share the mesh
    ins = [bridge.SystemInputs(w), bridge.SystemInputs(w.scaled(nx=w.nx - 1))]
    with pytest.raises(A.AsdError) as e:
        A.Handle(bridge.params_for(w, A.ASD_FP32, demag_cell=(2, 2, 2)), [i.desc for i in ins])
    assert e.value.code == A.ASD_EUNSUPPORTED
