"""Pins of the oracle's micromagnetic region (LLG by RK4 on a finite-difference
mesh, Eqs. 4-5, temperature-dependent parameters of Sec. II) against closed
forms: the Langevin function and the Curie-Weiss equation it defines, damped
precession of a uniform state and RK4's fourth order, the precession frequency
of a spin wave on the six-point stencil (whose long-wave limit is Eq. 11), and
the temperature scaling of the anisotropy and damping against the atomistic
oracle's single spin.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle_build import free_spins_system

GAMMA = 1.76e11
MS0, K0, TC = 5.2e5, 2.2e6, 710.0
A0 = 6.8e-21 / (2 * 0.5e-9)  # Eq. 9, A = J / 2a
MU_S = MS0 * (0.5e-9) ** 3


def mm(n=(4, 3, 2), h=(1e-9, 1e-9, 2e-9), **kw):
    args = dict(n=n, h=h, Ms0=MS0, A0=A0, K0=K0, lam=0.1, gamma=GAMMA, Tc=TC, mu_s=MU_S,
                dt=1e-15)
    args.update(kw)
    return oracle.MM(**args)


def test_langevin_function():
    """Against coth x - 1/x in 40-digit decimal arithmetic, on both sides of the
    switch from the series to the closed form at 0.1.  Bound: just above the
    switch coth x and 1/x cancel to 1/300 of their size, so the closed form keeps
    about 300 eps of relative error (7e-14); the series through x^11 leaves 2e-17."""
    from decimal import Decimal, getcontext
    getcontext().prec = 40
    for x in (1e-6, 0.01, 0.0999, 0.1, 0.1001, 0.5, 2.0, 30.0):
        X = Decimal(x)
        e = (2 * X).exp()
        ref = float((e + 1) / (e - 1) - 1 / X)
        assert abs(oracle.langevin(x) - ref) <= (1e-13 if x >= 0.1 else 1e-15) * ref, x


def test_equilibrium_magnetisation_solves_curie_weiss():
    """m_e = L(3 T_C m_e / T + b / T): residual, limits (1 - T / 3 T_C at low T,
    (5/3)(1 - T/T_C) for m_e^2 just below T_C, 0 above T_C without field, > 0 with)."""
    for T in (50.0, 300.0, 600.0, 700.0):
        for b in (0.0, 5.0):
            m = oracle.mm_me(T, TC, b)
            assert abs(m - oracle.langevin((3 * TC * m + b) / T)) < 1e-14
    assert oracle.mm_me(0.0, TC) == 1.0
    for T in (1.0, 5.0):
        assert abs(oracle.mm_me(T, TC) - (1 - T / (3 * TC))) < 3 * (T / TC) ** 2
    for d in (1e-3, 1e-4):
        m = oracle.mm_me(TC * (1 - d), TC)
        assert abs(m * m / (5 / 3 * d) - 1) < 5 * d
    assert oracle.mm_me(800.0, TC) == 0.0
    assert 0 < oracle.mm_me(800.0, TC, 2.0) < oracle.mm_me(800.0, TC, 5.0)
    Ts = np.linspace(10, 700, 40)
    ms = [oracle.mm_me(T, TC) for T in Ts]
    assert np.all(np.diff(ms) < 0)


def closed_form(theta0, phi0, B, alpha, t):
    gp = GAMMA / (1 + alpha * alpha)
    th = 2 * math.atan(math.tan(theta0 / 2) * math.exp(-alpha * gp * B * t))
    ph = phi0 + gp * B * t
    return np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])


def test_uniform_damped_precession_and_fourth_order():
    """Uniform state, no anisotropy, T = 0 (alpha = lambda): every cell follows the
    closed-form damped precession; the RK4 error falls 16x per halving of dt."""
    theta0, phi0, B, lam = 2.5, 0.3, 5.0, 0.1
    t = 2e-12
    errs = []
    for dt in (40e-15, 20e-15, 10e-15):
        steps = int(round(t / dt))
        r = mm(K0=0.0, B=(0.0, 0.0, B), dt=dt, periodic=(1, 1, 1))
        m0 = np.array([math.sin(theta0) * math.cos(phi0), math.sin(theta0) * math.sin(phi0),
                       math.cos(theta0)])
        m = r.rk4(np.repeat(m0[:, None], r.n, axis=1), 0, steps)
        assert np.max(np.abs(m - m[:, :1])) < 1e-15
        errs.append(np.max(np.abs(m[:, 0] - closed_form(theta0, phi0, B, lam, t))))
    assert errs[-1] < 1e-9
    for e0, e1 in zip(errs, errs[1:]):
        assert abs(math.log2(e0 / e1) - 4) < 0.3, errs


def test_spin_wave_frequency_on_the_stencil():
    """Small transverse wave m = (e cos kx, e sin kx, 1) on a periodic chain at
    T = 0, lambda = 0: it precesses at w = gamma [B + 2K/Ms + (2A/Ms)(2/h^2)(1 - cos kh)]
    (Eq. 4 on the six-point stencil with Eq. 5); for kh -> 0 this is Eq. 11's
    w0 + gamma (2A/Ms) k^2."""
    nx, hx, B = 64, 1e-9, 1.0
    steps, dt = 400, 1e-15
    eps = 1e-4
    x = np.arange(nx)
    for q in (1, 4, 9):
        k = 2 * math.pi * q / (nx * hx)
        r = mm(n=(nx, 1, 1), h=(hx, 1e-9, 2e-9), lam=0.0, B=(0.0, 0.0, B), dt=dt,
               periodic=(1, 1, 1))
        m0 = np.stack([eps * np.cos(k * x * hx), eps * np.sin(k * x * hx), np.ones(nx)])
        m0 /= np.linalg.norm(m0, axis=0)
        m = r.rk4(m0, 0, steps)
        a0 = np.angle((m0[0] + 1j * m0[1]) * np.exp(-1j * k * x * hx)).mean()
        a1 = np.angle((m[0] + 1j * m[1]) * np.exp(-1j * k * x * hx)).mean()
        w_num = (a1 - a0) / (steps * dt)  # m_x + i m_y turns as exp(+i w t) about +z
        w = GAMMA * (B + 2 * K0 / MS0 + (2 * A0 / MS0) * (2 / hx ** 2) * (1 - math.cos(k * hx)))
        assert abs(w_num / w - 1) < 1e-6, (q, w_num, w)
        if q == 1:
            w11 = GAMMA * (B + 2 * K0 / MS0 + (2 * A0 / MS0) * k * k)
            assert abs(w / w11 - 1) < 1e-3


def test_temperature_scaling_matches_a_single_spin():
    """Uniform state at a uniform T: exchange vanishes and each cell is a spin with
    anisotropy field 2 K0 m_e^2 / Ms0 and damping lambda (1 - T / 3 T_C).  The
    atomistic oracle's single spin (Heun, no noise) with k_u = mu_s K0 m_e^2 / Ms0
    and that damping follows the same path to the Heun error."""
    T, B, lam = 400.0, 2.0, 0.1
    me = oracle.mm_me(T, TC, MU_S * B / W.KB)
    alpha = lam * (1 - T / (3 * TC))
    th, ph = 0.7, 0.1
    m0 = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    steps, dt = 2000, 1e-15
    r = mm(B=(0.0, 0.0, B), dt=dt, periodic=(1, 1, 1), T_amb=T)
    m = r.rk4(np.repeat(m0[:, None], r.n, axis=1), 0, steps)[:, 0]
    s = free_spins_system(1, mu_s=MU_S, alpha=alpha, gamma=GAMMA, dt=dt,
                          ku=MU_S * K0 * me * me / MS0, B=(0.0, 0.0, B), T=0.0)
    ref = s.heun(m0[:, None], 0, steps)[:, 0]
    assert np.max(np.abs(m - ref)) < 1e-6
    moved = np.max(np.abs(ref - m0))
    assert moved > 0.05
    # with the 0 K parameters instead the path differs
    s0 = free_spins_system(1, mu_s=MU_S, alpha=lam, gamma=GAMMA, dt=dt, ku=MU_S * K0 / MS0,
                           B=(0.0, 0.0, B), T=0.0)
    assert np.max(np.abs(s0.heun(m0[:, None], 0, steps)[:, 0] - m)) > 1e-3


def test_unit_length_and_energy_descent_with_exchange():
    """Random start at T = 0 with damping: |m| = 1 after every step and the
    exchange + anisotropy + Zeeman energy of the mesh decreases."""
    n = (6, 5, 3)
    h = (1e-9, 1e-9, 2e-9)
    r = mm(n=n, h=h, B=(0.0, 0.0, 0.5), lam=0.5, dt=5e-15)
    rng = np.random.default_rng(1)
    m = rng.normal(size=(3, r.n))
    m /= np.linalg.norm(m, axis=0)

    def energy(m):
        M = m.reshape(3, n[2], n[1], n[0])
        e = 0.0
        for ax, hh in ((3, h[0]), (2, h[1]), (1, h[2])):
            d = np.diff(M, axis=ax)
            e += A0 * (d ** 2).sum() / hh ** 2
        e -= K0 * (M[2] ** 2).sum()
        e -= MS0 * 0.5 * M[2].sum()
        return e
    e0 = energy(m)
    prev = e0
    for k in range(10):
        m = r.rk4(m, 40 * k, 40)
        assert np.max(np.abs(np.linalg.norm(m, axis=0) - 1)) < 1e-14
        e = energy(m)
        assert e < prev
        prev = e


def test_x_face_coupling_converges_to_the_unsplit_mesh():
    """A periodic mesh cut in two along x, each half seeing the other's boundary
    cells (taken at the start of every step) through its x faces: as dt halves the
    coupled halves approach the uncut mesh linearly (the lag is first order), and
    with the faces removed they do not."""
    n, h = (8, 3, 2), (1e-9, 1e-9, 2e-9)
    rng = np.random.default_rng(3)
    m0 = rng.normal(size=(3, 16 * 3 * 2)) * 0.3
    m0[2] += 1
    m0 /= np.linalg.norm(m0, axis=0)
    M0 = m0.reshape(3, 2, 3, 16)
    t_end = 200e-15
    errs = []
    for dt in (4e-15, 2e-15, 1e-15):
        steps = int(round(t_end / dt))
        full = mm(n=(16, 3, 2), h=h, dt=dt, B=(0.0, 0.0, 0.5), periodic=(1, 0, 0))
        ref = full.rk4(m0, 0, steps).reshape(3, 2, 3, 16)
        L = mm(n=n, h=h, dt=dt, B=(0.0, 0.0, 0.5))
        R = mm(n=n, h=h, dt=dt, B=(0.0, 0.0, 0.5))
        a = np.ascontiguousarray(M0[:, :, :, :8]).reshape(3, -1)
        b = np.ascontiguousarray(M0[:, :, :, 8:]).reshape(3, -1)
        for k in range(steps):
            fa0, fa1, fb0, fb1 = L.face(0, a), L.face(1, a), R.face(0, b), R.face(1, b)
            L.set_ghost(0, fb1)  # periodic: left's -x neighbour is right's last column
            L.set_ghost(1, fb0)
            R.set_ghost(0, fa1)
            R.set_ghost(1, fa0)
            a, b = L.rk4(a, k, 1), R.rk4(b, k, 1)
        got = np.concatenate([a.reshape(3, 2, 3, 8), b.reshape(3, 2, 3, 8)], axis=3)
        errs.append(np.max(np.abs(got - ref)))
    assert errs[-1] < 5e-3
    for e0, e1 in zip(errs, errs[1:]):
        assert abs(math.log2(e0 / e1) - 1) < 0.25, errs
    # without the faces the halves drift apart from the uncut mesh
    L = mm(n=n, h=h, dt=1e-15, B=(0.0, 0.0, 0.5))
    a = L.rk4(np.ascontiguousarray(M0[:, :, :, :8]).reshape(3, -1), 0, 200)
    drift = np.max(np.abs(a.reshape(3, 2, 3, 8) - ref[:, :, :, :8]))
    assert drift > 10 * errs[-1]


@pytest.mark.parametrize("kind,cell", [(oracle.SC, (3, 4, 2)), (oracle.L10, (2, 3, 3))])
def test_set_columns_writes_each_cell_direction(kind, cell):
    """The regions' faces written into atomistic columns: every magnetic site of
    a coarse cell takes the cell's unit direction (+z for a zero cell), the
    non-magnetic sites stay zero and the other columns are untouched; so
    coarse-graining the written columns gives count x direction."""
    sx, ny, nz = 11, 7, 5
    cx, cy, cz = cell
    per = 1 if kind == oracle.SC else 2
    n = per * sx * ny * nz
    rng = np.random.default_rng(12)
    lab = np.where(rng.uniform(size=n) < 0.2, -1, 0).astype(np.int32)
    S0 = rng.normal(size=(3, n))
    S0 /= np.linalg.norm(S0, axis=0)
    S0[:, lab < 0] = 0.0
    x0, ncols = 4, 5
    ncell = -(-ncols // cx) * -(-ny // cy) * -(-nz // cz)
    mcell = rng.normal(size=(ncell, 3)) * rng.uniform(0.1, 2.0, size=(ncell, 1))
    mcell[1] = 0.0
    S = oracle.set_columns(kind, sx, ny, nz, lab, S0, x0, ncols, cx, cy, cz, mcell)
    unit = mcell / np.maximum(np.linalg.norm(mcell, axis=1), 1e-300)[:, None]
    unit[1] = (0.0, 0.0, 1.0)
    site = np.arange(n)
    x = (site // per) % sx
    y = (site // per // sx) % ny
    z = site // per // sx // ny
    inside = (x >= x0) & (x < x0 + ncols)
    c = (x - x0) // cx + -(-ncols // cx) * (y // cy + -(-ny // cy) * (z // cz))
    mag = lab >= 0
    np.testing.assert_array_equal(S[:, ~inside], S0[:, ~inside])
    np.testing.assert_array_equal(S[:, inside & ~mag], 0.0)
    w = inside & mag
    np.testing.assert_allclose(S[:, w], unit[c[w]].T, rtol=0, atol=1e-15)
    out = oracle.coarse_grain(kind, sx, ny, nz, lab, S, x0, ncols, cx, cy, cz)
    counts = np.bincount(c[w], minlength=ncell)
    np.testing.assert_array_equal(out[:, 3], counts)
    np.testing.assert_allclose(out[:, :3], counts[:, None] * unit, rtol=1e-13, atol=1e-13)
