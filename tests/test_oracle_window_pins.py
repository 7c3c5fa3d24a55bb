"""Pins of the oracle's moving multiscale window (Sec. II, Fig. 1): the
uniform-cap reading of the cone thermalisation (its spins average back to the
magnetisation they were drawn from, cos theta uniform on [2m - 1, 1]), the
move of a micromagnetic region by one cell, the reduced magnetisation
m_e(T) m that a region hands to the atoms, and the whole window move checked
against what it must do in the limits where its result is fixed: saturated
cells rebuild exactly, averaged columns become the left region's new cells,
the regions' cells move by exactly one column.
"""
import math

import numpy as np
import pytest

import oracle

GAMMA = 1.76e11
MS0, K0, TC = 5.2e5, 2.2e6, 710.0
A0 = 6.7e-21 / (2 * 0.3e-9)
MU_S = 2.99550525e-23


def region(n, **kw):
    args = dict(n=n, h=(0.6e-9, 0.6e-9, 0.6e-9), Ms0=MS0, A0=A0, K0=K0, lam=0.1, gamma=GAMMA,
                Tc=TC, mu_s=MU_S, dt=1e-15)
    args.update(kw)
    return oracle.MM(**args)


def random_unit(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(3, n))
    return v / np.linalg.norm(v, axis=0)


# ------------------------------------------------------------------ cap cone
@pytest.mark.parametrize("m", [0.0, 0.15, 0.5, 0.8, 0.97])
def test_cap_cone_cos_uniform_and_mean_returns_m(m):
    """ORC_CONE_CAP: cos of the polar angle to the cell direction is uniform
    on [2m - 1, 1] (Kolmogorov-Smirnov), the azimuth uniform, so the mean spin
    is m n (within 5 sigma over 6000 draws): thermalise then average returns
    the magnetisation, unlike the printed cone."""
    from scipy import stats
    n = np.array([0.3, -0.4, 0.866])
    n /= np.linalg.norm(n)
    N = 6000
    S = np.array([oracle.cone_spin(m * n, 10, 5, i, 3, 1, mode=oracle.CONE_CAP) for i in range(N)])
    if m == 0.0:  # zero magnetisation: the cap is the whole sphere, measured from z
        n = np.array([0.0, 0.0, 1.0])
    assert np.max(np.abs(np.linalg.norm(S, axis=1) - 1)) < 1e-15
    c = S @ n
    lo = 2 * m - 1
    assert c.min() >= lo - 1e-12
    assert stats.kstest((c - lo) / (1 - lo), "uniform").pvalue > 1e-3
    mean = S.mean(0)
    sig = S.std(0) / math.sqrt(N)
    assert np.all(np.abs(mean - m * n) < 5 * sig + 1e-12)
    a = np.array([1.0, 0.0, 0.0])
    e1 = np.cross(n, a)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(n, e1)
    phi = np.arctan2(S @ e2, S @ e1) % (2 * math.pi)
    assert stats.kstest(phi / (2 * math.pi), "uniform").pvalue > 1e-3


def test_cap_cone_saturated_cell_gives_its_direction():
    """m = 1: the cap shrinks to the direction itself (both readings)."""
    n = np.array([0.6, 0.0, -0.8])
    for mode in (oracle.CONE_CAP, oracle.CONE_PRINTED):
        for i in range(20):
            s = oracle.cone_spin(n, 10, 1, i, 0, 0, mode=mode)
            assert np.max(np.abs(s - n)) < 3e-16


def test_cap_cone_columns_round_trip():
    """Thermalise columns with the cap reading, then coarse-grain them (Eq. 6
    both ways): each cell returns its reduced magnetisation, magnitude and
    direction, within 4 sigma at 3200 sites per cell."""
    sx, ny, nz = 12, 40, 40
    n = sx * ny * nz
    lab = np.zeros(n, np.int32)
    mcell = np.array([[0.0, 0.0, 0.9], [0.5, 0.0, -0.5], [0.0, -0.3, 0.0]])
    S = oracle.cone_columns(oracle.SC, sx, ny, nz, lab, np.zeros((3, n)), 3, 6, 2, ny, nz, mcell,
                            10, 7, 11, 0, mode=oracle.CONE_CAP)
    out = oracle.coarse_grain(oracle.SC, sx, ny, nz, lab, S, 3, 6, 2, ny, nz)
    for c in range(3):
        d = out[c, :3] / out[c, 3]
        assert np.max(np.abs(d - mcell[c])) < 4 * 0.6 / math.sqrt(3200)
    # the printed reading is the same spins' polar angles stretched differently:
    # same sites and counters, different cells' magnitudes
    P = oracle.cone_columns(oracle.SC, sx, ny, nz, lab, np.zeros((3, n)), 3, 6, 2, ny, nz, mcell,
                            10, 7, 11, 0)
    outp = oracle.coarse_grain(oracle.SC, sx, ny, nz, lab, P, 3, 6, 2, ny, nz)
    assert np.linalg.norm(outp[0, :3] / outp[0, 3]) > 0.95  # printed: sin(tmax)/tmax, not 0.9


# ------------------------------------------------------------------ region move
def test_region_shift_moves_every_cell_one_column_down():
    """Cell (i, j, k) takes cell (i + 1, j, k); the first column leaves; the last
    column takes the normalised entering vectors (stride 4: the Eq. 6 sums; a
    zero vector gives +z)."""
    nx, ny, nz = 5, 3, 2
    r = region((nx, ny, nz))
    m = random_unit(nx * ny * nz, 1)
    enter = np.zeros((ny * nz, 4))
    enter[:, :3] = random_unit(ny * nz, 2).T * 3.5
    enter[:, 3] = 7.0
    enter[4, :3] = 0.0
    out, leave = r.shift(m, enter, stride=4)
    M, O = m.reshape(3, nz, ny, nx), out.reshape(3, nz, ny, nx)
    assert np.array_equal(O[:, :, :, :-1], M[:, :, :, 1:])
    np.testing.assert_array_equal(leave, M[:, :, :, 0].reshape(3, -1).T)
    want = enter[:, :3] / np.linalg.norm(enter[:, :3], axis=1, keepdims=True).clip(1e-300)
    want[4] = (0.0, 0.0, 1.0)
    np.testing.assert_allclose(O[:, :, :, -1].reshape(3, -1).T, want, rtol=0, atol=2e-16)


def test_face_moment_is_equilibrium_magnetisation_times_direction():
    """M / M_S^0 of a face cell = m_e(T) m with T of the cell (Sec. II): uniform
    ambient temperature, then a locked spot (cells nearer its centre hotter,
    so a smaller m_e)."""
    nx, ny, nz = 4, 6, 2
    m = random_unit(nx * ny * nz, 3)
    r = region((nx, ny, nz), T_amb=500.0)
    fm = r.face_moment(m, 0, 0.0)
    me = oracle.mm_me(500.0, TC, 0.0)
    np.testing.assert_allclose(np.linalg.norm(fm, axis=1), me, rtol=1e-15)
    M = m.reshape(3, nz, ny, nx)
    np.testing.assert_allclose(fm, me * M[:, :, :, 0].reshape(3, -1).T, rtol=1e-15)
    hot = region((nx, ny, nz), T_amb=300.0, T_peak=800.0, fwhm=3e-9, spot_mode=oracle.SPOT_LOCKED,
                 x0=0.3e-9, y0=1.8e-9, B=(0.0, 0.0, 0.8))
    fm = hot.face_moment(m, 0, 0.0)
    b = MU_S * 0.8 / 1.380649e-23
    for j in range(ny):
        T = hot.temperature(0, j, 0.0)
        assert abs(np.linalg.norm(fm[j]) - oracle.mm_me(T, TC, b)) < 1e-15
    mags = np.linalg.norm(fm[:ny], axis=1)
    assert np.argmin(mags) in (2, 3)  # y0 = 1.8 nm is the boundary of cells 2 and 3
    last = hot.face_moment(m, 1, 0.0)
    np.testing.assert_allclose(
        last / np.linalg.norm(last, axis=1, keepdims=True), M[:, :, :, -1].reshape(3, -1).T,
        rtol=0, atol=1e-15)


# ------------------------------------------------------------------ whole move
@pytest.mark.parametrize("mode", [oracle.CONE_PRINTED, oracle.CONE_CAP])
def test_window_move_limits(mode):
    """The window move at T = 0 (m_e = 1, so thermalisation rebuilds a cell's
    direction: exactly but for the rounding of |m| = 1 - O(eps), which both
    readings turn into a polar angle of O(sqrt eps), below 1e-7): the
    entering atomistic columns carry the right region's first cells'
    directions on their magnetic sites (grain-boundary sites stay 0), the left region's new last column is the direction of the
    averaged leaving atoms, the old first column leaves, and the origin
    advances by one coarse cell."""
    cx, cy, cz = 2, 2, 2
    nx, ny, nz = 8, 4, 4
    sx = nx + 6 * cx
    n = sx * ny * nz
    rng = np.random.default_rng(4)
    lab = np.zeros(n, np.int32)
    lab[rng.random(n) < 0.2] = -1
    S = random_unit(n, 5)
    S[:, lab < 0] = 0.0
    org = 2 * cx
    L = region((3, ny // cy, nz // cz))
    R = region((4, ny // cy, nz // cz))
    mL, mR = random_unit(L.n, 6), random_unit(R.n, 7)
    enter = random_unit(R._p.ny * R._p.nz, 8).T
    sums = oracle.coarse_grain(oracle.SC, sx, ny, nz, lab, S, org, cx, cx, cy, cz)
    S2, org2, mL2, mR2, leave = oracle.multiscale_shift(
        oracle.SC, sx, ny, nz, lab, S, org, nx, (cx, cy, cz), L, mL, R, mR, enter, 10, 9, 123,
        mode=mode)
    assert org2 == org + cx
    # atoms: only columns [org + nx, org + nx + cx) changed, to their cells' directions
    A, A2 = S.reshape(3, nz, ny, sx), S2.reshape(3, nz, ny, sx)
    cols = slice(org + nx, org + nx + cx)
    keep = np.ones(sx, bool)
    keep[cols] = False
    assert np.array_equal(A[:, :, :, keep], A2[:, :, :, keep])
    lab3 = lab.reshape(nz, ny, sx)
    face = R.face(0, mR)  # [ny/cy * nz/cz, 3]
    for z in range(nz):
        for y in range(ny):
            for x in range(org + nx, org + nx + cx):
                v = A2[:, z, y, x]
                if lab3[z, y, x] < 0:
                    assert np.all(v == 0)
                else:
                    c = (y // cy) + (ny // cy) * (z // cz)
                    assert np.max(np.abs(v - face[c])) < 1e-7
    # regions
    ML, ML2 = mL.reshape(3, -1, L._p.nx), mL2.reshape(3, -1, L._p.nx)
    assert np.array_equal(ML2[:, :, :-1], ML[:, :, 1:])
    np.testing.assert_array_equal(leave, ML[:, :, 0].T)
    d = sums[:, :3] / np.linalg.norm(sums[:, :3], axis=1, keepdims=True)
    np.testing.assert_allclose(ML2[:, :, -1].T, d, rtol=0, atol=2e-16)
    MR, MR2 = mR.reshape(3, -1, R._p.nx), mR2.reshape(3, -1, R._p.nx)
    assert np.array_equal(MR2[:, :, :-1], MR[:, :, 1:])
    np.testing.assert_allclose(MR2[:, :, -1].T, enter, rtol=0, atol=2e-16)


def test_window_move_thermalises_with_the_cell_temperature():
    """At a finite temperature the entering spins spread around the cell
    direction, and with the cap reading their average over a large cell
    returns m_e(T) m (the magnetisation the region held)."""
    cx, cy, cz = 4, 40, 40
    nx, ny, nz = 4, 40, 40
    sx = nx + 3 * cx
    n = sx * ny * nz
    lab = np.zeros(n, np.int32)
    S = np.zeros((3, n))
    S[2] = 1.0
    R = region((2, 1, 1), T_amb=650.0)
    mR = np.zeros((3, 2))
    mR[0] = 1.0
    enter = np.array([[0.0, 0.0, 1.0]])
    S2, org2, _, mR2, _ = oracle.multiscale_shift(
        oracle.SC, sx, ny, nz, lab, S, cx, nx, (cx, cy, cz), None, None, R, mR, enter, 10, 3, 0,
        mode=oracle.CONE_CAP)
    me = oracle.mm_me(650.0, TC, 0.0)
    out = oracle.coarse_grain(oracle.SC, sx, ny, nz, lab, S2, cx + nx, cx, cx, cy, cz)
    avg = out[0, :3] / out[0, 3]
    assert 0.3 < me < 0.7
    assert np.max(np.abs(avg - np.array([me, 0.0, 0.0]))) < 4 * 0.6 / math.sqrt(cx * cy * cz)
    assert np.array_equal(mR2[:, 0], mR[:, 1]) and np.array_equal(mR2[:, 1], [0.0, 0.0, 1.0])
