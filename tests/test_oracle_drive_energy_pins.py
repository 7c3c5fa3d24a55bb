"""Pins of the oracle's drive, reductions and energy against closed forms and
plain definitions written differently from the oracle's code:

* the laser spot of Sec. III (Fig. 2): a circular Gaussian fixed by its peak,
  its ambient temperature and its full width at half maximum, whose centre
  moves at v (continuous mode) or is locked to the window origin;
* the bit-timed write-field polarity (Sec. II: bits are written by flipping
  the field): bit floor(n / steps_per_bit) mod n_bits;
* the per-grain moment sums of Eq. 6 against numpy's bincount and math.fsum;
* the energy of the Hamiltonian of Eqs. 2-3 plus the Zeeman term: the aligned
  periodic lattice in closed form, and -dE/dS_i = mu_s B_i (the field the Heun
  stages use) by central differences, which are exact for a quadratic form;
* the micromagnetic cell temperature (same spot, cell centres) and the face
  neighbour of a region when the atomistic face cell holds no magnetic site.

A plausible slip in any of these functions (FWHM taken as the standard
deviation, exp(-r^2/s^2), the wrong centre, the polarity off by one bit, a
dropped or doubled exchange half, a missing anisotropy factor 2) fails a test
here.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle_build import oracle_system

LN2 = math.log(2.0)


def _spot_workload(kind=W.SC, **kw):
    base = dict(nx=40, ny=12, nz=2, bc=(W.BC_PERIODIC, W.BC_PERIODIC, W.BC_OPEN),
                spot_mode=W.SPOT_MOVING, T_amb=300.0, T_peak=800.0, fwhm=4e-9, x0=3e-9,
                y0=1.8e-9, v=10.0)
    if kind == W.L10:
        base.update(kind=W.L10, a=0.385e-9, c=0.371e-9, J=(6.0e-21, 1.2e-21, 0.5e-21, 0.2e-21))
    base.update(kw)
    return W.Workload("spot", **base)


def _closed_form_T(px, py, xc, yc, w):
    """The Gaussian written through its FWHM: T_amb + dT 2^(-4 r^2 / FWHM^2)."""
    r2 = (px - xc) ** 2 + (py - yc) ** 2
    return w.T_amb + (w.T_peak - w.T_amb) * np.power(2.0, -4.0 * r2 / w.fwhm ** 2)


@pytest.mark.parametrize("kind", [W.SC, W.L10])
@pytest.mark.parametrize("mode", [W.SPOT_MOVING, W.SPOT_LOCKED])
def test_spot_temperature_closed_form(kind, mode):
    w = _spot_workload(kind, spot_mode=mode)
    origin = 7
    s = oracle_system(w, origin=origin)
    px, py = oracle.site_positions(w.kind, w.nx, w.ny, w.nz, w.a)
    for step in (0, 1, 123, 4567):
        if mode == W.SPOT_MOVING:
            xc = w.x0 + w.v * step * w.dt
        else:
            xc = origin * w.hx + w.x0  # the window origin in lattice x units
        T = s.temperature(step)
        np.testing.assert_allclose(T, _closed_form_T(px, py, xc, w.y0, w), rtol=2e-15, atol=0)
        assert np.all(T >= w.T_amb) and np.all(T <= w.T_peak)


def test_spot_peak_half_maximum_and_far_field():
    """Exactly T_peak at the centre; (T_peak + T_amb) / 2 at r = FWHM/2 along x
    and along y; T_amb far away.  Sites are placed at those points."""
    w = _spot_workload(nx=4, ny=1, nz=1, spot_mode=W.SPOT_MOVING, v=0.0)
    n = 5
    h = 0.5 * w.fwhm
    px = np.array([w.x0, w.x0 + h, w.x0, w.x0 - h, w.x0 + 25 * w.fwhm])
    py = np.array([w.y0, w.y0, w.y0 - h, w.y0, w.y0])
    s = oracle.System(row_ptr=np.zeros(n + 1, np.int64), col=np.zeros(1, np.int32),
                      shell=np.zeros(1, np.int8), label=np.zeros(n, np.int32), px=px, py=py,
                      ctr0=np.arange(n, dtype=np.uint32), n_shells=0, J=(), mu_s=w.mu_s,
                      alpha=w.alpha, gamma=w.gamma, dt=w.dt, ku=0.0, spot_mode=W.SPOT_MOVING,
                      T_amb=w.T_amb, T_peak=w.T_peak, fwhm=w.fwhm, x0=w.x0, y0=w.y0, v=0.0)
    T = s.temperature(0)
    assert T[0] == w.T_peak
    half = 0.5 * (w.T_peak + w.T_amb)
    for k in (1, 2, 3):
        assert abs(T[k] - half) <= 2e-15 * half, T[k]
    assert T[4] == w.T_amb
    # a uniform system ignores the spot parameters
    s2 = oracle_system(_spot_workload(spot_mode=W.SPOT_NONE))
    assert np.all(s2.temperature(50) == 300.0)


def test_locked_spot_follows_the_window_origin():
    """The hottest site of a locked spot sits at origin * hx + x0 (hx = a for SC,
    a / 2 for L1_0) and moves one column per unit of origin."""
    for kind in (W.SC, W.L10):
        w = _spot_workload(kind, spot_mode=W.SPOT_LOCKED, x0=0.0, y0=0.0, nx=30, ny=4, nz=1)
        px, py = oracle.site_positions(w.kind, w.nx, w.ny, w.nz, w.a)
        for origin in (0, 3, 11):
            s = oracle_system(w, origin=origin)
            T = s.temperature(99)
            hot = np.flatnonzero(T == T.max())
            d2 = (px - origin * w.hx) ** 2 + py ** 2
            near = np.flatnonzero(d2 <= d2.min() * (1 + 1e-12) + 1e-40)
            np.testing.assert_array_equal(hot, near)
            # the centre falls on a site whenever origin * hx is a lattice x position
            if kind == W.SC or origin % 2 == 0:
                assert T.max() == w.T_peak


def test_polarity_schedule():
    bits = (1, 0, 0, 1, 1)
    spb = 7
    w = W.c1_plain_sc().scaled(bits=bits, steps_per_bit=spb)
    s = oracle_system(w)
    for n in range(0, 3 * spb * len(bits) + 5):
        expect = 1.0 if bits[(n // spb) % len(bits)] else -1.0
        assert s.polarity(n) == expect, n
    # flips exactly at the bit boundaries, wraps after n_bits bits
    assert s.polarity(spb - 1) == 1.0 and s.polarity(spb) == -1.0
    assert s.polarity(3 * spb - 1) == -1.0 and s.polarity(3 * spb) == 1.0
    assert s.polarity(5 * spb - 1) == 1.0 and s.polarity(5 * spb) == 1.0   # wrap to bit 0
    assert s.polarity(6 * spb) == -1.0
    big = 10**12 + 3
    assert s.polarity(big) == (1.0 if bits[(big // spb) % 5] else -1.0)
    # no pattern: +1 always
    s0 = oracle_system(W.c1_plain_sc())
    assert s0.polarity(0) == 1.0 and s0.polarity(10**9) == 1.0
    # the polarity multiplies the write field in the field the stages use
    S = np.zeros((3, w.n_sites))
    S[2] = 1.0
    for n in (0, spb):
        B = s.field(S, n, sites=[3 * 16 * 16])[0]   # z = 3: six neighbours
        Bz_free = 6 * w.J[0] / w.mu_s + 2 * w.ku / w.mu_s
        assert abs(B[2] - (Bz_free + s.polarity(n) * w.B[2])) < 1e-12 * Bz_free


def test_mm_polarity_and_temperature():
    bits = (0, 1, 1)
    p = oracle.MM(n=(12, 5, 2), h=(1e-9, 2e-9, 2e-9), Ms0=5.2e5, A0=6.8e-12, K0=2.2e6,
                  lam=0.1, gamma=1.76e11, Tc=710.0, mu_s=6.5e-23, dt=2e-14, B=(0, 0, 0.8),
                  bits=bits, steps_per_bit=4, spot_mode=W.SPOT_MOVING, T_amb=300.0,
                  T_peak=800.0, fwhm=6e-9, x0=4.5e-9, y0=3e-9, v=20.0)
    for n in range(30):
        assert p.polarity(n) == (1.0 if bits[(n // 4) % 3] else -1.0)
    w = _spot_workload(fwhm=6e-9, x0=4.5e-9, y0=3e-9, v=20.0)
    for t in (0.0, 1e-12, 3.3e-11):
        xc = 4.5e-9 + 20.0 * t
        for i in range(12):
            for j in range(5):
                T = p.temperature(i, j, t)
                ref = _closed_form_T(np.array((i + 0.5) * 1e-9), np.array((j + 0.5) * 2e-9),
                                     xc, 3e-9, w)
                assert abs(T - float(ref)) <= 2e-15 * T
    # the cell whose centre is the spot centre at t = 0: (4 + 1/2) nm, (1 + 1/2) 2 nm
    assert abs(p.temperature(4, 1, 0.0) - 800.0) < 1e-12


# ------------------------------------------------------------------ Eq. 6 moment sums
@pytest.mark.parametrize("masked", [False, True])
def test_magnetisation_is_the_per_label_sum(masked):
    """Per-grain (sum Sx, sum Sy, sum Sz, count) over magnetic (and, with a
    window mask, active) sites, against numpy's bincount and math.fsum."""
    rng = np.random.default_rng(77)
    w = W.c1_plain_sc().scaled(nx=12, ny=10, nz=6)
    n, G = w.n_sites, 9
    lab = rng.integers(-1, G, size=n).astype(np.int32)
    active = (rng.uniform(size=n) < 0.7).astype(np.uint8) if masked else None
    s = oracle_system(w, labels=lab, active=active)
    S = rng.normal(size=(3, n)) * rng.uniform(0.1, 3.0, size=n)
    pg, tot = s.magnetisation(S, G)
    use = (lab >= 0) & (True if active is None else active.astype(bool))
    for k in range(3):
        ref = np.bincount(lab[use], weights=S[k, use], minlength=G)
        np.testing.assert_allclose(pg[:, k], ref, rtol=1e-13, atol=1e-13)
        assert abs(tot[k] - math.fsum(S[k, use])) <= 1e-15 * math.fsum(np.abs(S[k, use]))
        for g in range(G):   # compensated sums: the correctly rounded value
            assert abs(pg[g, k] - math.fsum(S[k, use & (lab == g)])) <= 2 * np.spacing(
                abs(pg[g, k]) + 1e-300)
    np.testing.assert_array_equal(pg[:, 3], np.bincount(lab[use], minlength=G))
    assert tot[3] == use.sum()


# ------------------------------------------------------------------ energy (Eqs. 2-3 + Zeeman)
def test_energy_of_the_aligned_periodic_lattice():
    """All spins along +z on a periodic lattice, B along +z:
    E_ex = -(1/2) N sum_s z_s J_s (SC: -3 N J; L1_0 shells of 4, 2, 4, 8),
    E_an = -N k_u, E_Z = -N mu_s B."""
    Bz = 0.8
    sc = W.Workload("cube", nx=6, ny=6, nz=6, bc=(1, 1, 1), B=(0.0, 0.0, Bz))
    l10 = W.Workload("l10", kind=W.L10, nx=4, ny=4, nz=4, bc=(1, 1, 1), a=0.385e-9, c=0.371e-9,
                     J=(6.0e-21, 1.2e-21, 0.5e-21, 0.2e-21), B=(0.0, 0.0, Bz))
    for w, zJ in ((sc, 6 * sc.J[0]), (l10, 4 * l10.J[0] + 2 * l10.J[1] + 4 * l10.J[2]
                                     + 8 * l10.J[3])):
        N = w.n_sites
        S = np.zeros((3, N))
        S[2] = 1.0
        E = oracle_system(w).energy(S, 0)
        assert abs(E[0] / (-0.5 * N * zJ) - 1) < 1e-14
        assert abs(E[1] / (-N * w.ku) - 1) < 1e-14
        assert abs(E[2] / (-N * w.mu_s * Bz) - 1) < 1e-14
        assert abs(E[3] - (E[0] + E[1] + E[2])) <= 1e-15 * abs(E[3])
        # reversing every spin keeps exchange and anisotropy, flips the Zeeman term
        Er = oracle_system(w).energy(-S, 0)
        assert Er[0] == E[0] and Er[1] == E[1] and Er[2] == -E[2]


def _gradient_check(s, S, mu_s, sites, step):
    """-dE/dS_i by central differences (exact for a quadratic form up to
    rounding) against mu_s times the field of the Heun stages."""
    B = s.field(S, step, sites=sites)
    h = 0.25
    for r, i in enumerate(sites):
        for k in range(3):
            Sp, Sm = S.copy(), S.copy()
            Sp[k, i] += h
            Sm[k, i] -= h
            g = -(s.energy(Sp, step)[3] - s.energy(Sm, step)[3]) / (2 * h)
            scale = mu_s * np.max(np.abs(B[r])) + 1e-30
            assert abs(g - mu_s * B[r, k]) <= 1e-9 * scale, (i, k, g, mu_s * B[r, k])


@pytest.mark.parametrize("kind", [W.SC, W.L10])
def test_energy_gradient_is_the_stage_field(kind):
    """B_i = -dE/d(mu_s S_i) for the exchange (pairs within one grain), the
    anisotropy (per-grain k_u) and the polarised write field, at arbitrary
    (not unit) spins on a periodic lattice with grain boundaries."""
    if kind == W.SC:
        w = W.Workload("g", nx=8, ny=7, nz=4, bc=(1, 1, 0), B=(0.1, -0.2, 0.7),
                       bits=(0, 1), steps_per_bit=3)
    else:
        w = W.Workload("g", kind=W.L10, nx=5, ny=4, nz=4, bc=(1, 1, 0), a=0.385e-9, c=0.371e-9,
                       J=(6.0e-21, 1.2e-21, 0.5e-21, 0.2e-21), B=(0.1, -0.2, 0.7),
                       bits=(0, 1), steps_per_bit=3)
    rng = np.random.default_rng(5)
    n = w.n_sites
    lab = rng.integers(-1, 3, size=n).astype(np.int32)
    kug = w.ku * (1 + 0.3 * rng.uniform(-1, 1, size=3))
    s = oracle_system(w, labels=lab, ku_grain=kug)
    S = rng.normal(size=(3, n))
    S[:, lab < 0] = 0.0
    sites = [i for i in rng.choice(n, size=12, replace=False) if lab[i] >= 0]
    for step in (0, 4):   # both polarities
        _gradient_check(s, S, w.mu_s, sites, step)


def test_energy_of_a_window_splits_its_edge_bonds():
    """With a window mask the energy counts each bond between the window and
    the frozen track once per end: E(window) + E(track) = E(whole lattice),
    and for sites whose neighbours all lie in the window -dE/dS_i is the field."""
    w = W.Workload("t", nx=10, ny=6, nz=3, bc=(W.BC_TRACK, 0, 0), track_nx=24,
                   B=(0.0, 0.0, 0.8))
    rng = np.random.default_rng(9)
    n = 24 * 6 * 3
    S = rng.normal(size=(3, n))
    S /= np.linalg.norm(S, axis=0)
    lab = np.zeros(n, np.int32)
    x = np.arange(n) % 24
    win = ((x >= 6) & (x < 16)).astype(np.uint8)
    geom = None
    whole = oracle_system(w, labels=lab).energy(S, 0)
    inside = oracle_system(w, labels=lab, active=win, origin=6).energy(S, 0)
    outside = oracle_system(w, labels=lab, active=(1 - win).astype(np.uint8)).energy(S, 0)
    for k in range(4):
        assert abs(inside[k] + outside[k] - whole[k]) <= 1e-13 * abs(whole[k]), k
    del geom
    s = oracle_system(w, labels=lab, active=win, origin=6)
    interior = [i for i in range(n) if 8 <= x[i] < 14][::7]
    _gradient_check(s, S, w.mu_s, interior, 0)


# ------------------------------------------------------------------ region face with no atoms
def _region(**kw):
    args = dict(n=(5, 3, 2), h=(1e-9, 1e-9, 2e-9), Ms0=5.2e5, A0=6.8e-12, K0=2.2e6, lam=0.1,
                gamma=1.76e11, Tc=710.0, mu_s=6.5e-23, dt=2e-14, B=(0.0, 0.0, -0.8),
                spot_mode=W.SPOT_NONE, T_amb=300.0)
    args.update(kw)
    return oracle.MM(**args)


def test_region_face_cell_without_atoms_is_an_open_face():
    """An atomistic face cell that holds no magnetic site (a grain-boundary cell)
    has no magnetisation (its Eq. 6 sum is zero) and so no exchange with the
    region: the region's boundary cell behind it evolves as at an open face.
    A face neighbour equal to the boundary cell's own direction adds nothing
    (the stencil difference vanishes)."""
    rng = np.random.default_rng(4)
    m0 = rng.normal(size=(3, 30)) * 0.3
    m0[2] += 1
    m0 /= np.linalg.norm(m0, axis=0)
    ref = _region()
    open_face = ref.rk4(m0, 0, 20)
    zero = _region()
    zero.set_ghost(1, np.zeros((6, 3)))
    np.testing.assert_array_equal(zero.rk4(m0, 0, 20), open_face)
    # a uniform state with a face neighbour along the same direction stays put
    u = np.zeros((3, 30))
    u[2] = 1.0
    same = _region(B=(0.0, 0.0, 0.0))
    same.set_ghost(0, np.tile([0.0, 0.0, 1.0], (6, 1)))
    np.testing.assert_array_equal(same.rk4(u, 0, 10), u)
    # a single empty face cell only decouples the cell behind it: with every
    # other face neighbour equal to the current boundary direction, the first
    # step differs from the open face only through the coupled cells' stencil
    part = _region()
    g = open_face.reshape(3, 2, 3, 5)[:, :, :, 4].reshape(3, -1).T.copy()
    g[2] = 0.0
    part.set_ghost(1, g)
    one = part.rk4(m0, 0, 1)
    assert np.any(one != ref.rk4(m0, 0, 1))
