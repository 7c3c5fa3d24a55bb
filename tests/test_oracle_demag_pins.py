"""Pins of the oracle's demagnetising field (Eq. 7, Newell tensor) against
closed forms that do not use Newell's functions: Aharoni's demagnetising
factors of a rectangular prism, the point-dipole field at large distance, the
exact parities of the tensor, and the shape anisotropy of a uniformly
magnetised cell seen by a macrospin.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle_build import demag_cells, free_spins_system, oracle_system, track_stray


def aharoni_Dz(a, b, c):
    """Demagnetising factor along z of a uniformly magnetised prism with edges
    2a, 2b, 2c along x, y, z (A. Aharoni, J. Appl. Phys. 83, 3432 (1998))."""
    r = math.sqrt(a * a + b * b + c * c)
    ab, bc, ac = math.hypot(a, b), math.hypot(b, c), math.hypot(a, c)
    t = ((b * b - c * c) / (2 * b * c) * math.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * math.log((r - b) / (r + b))
         + b / (2 * c) * math.log((ab + a) / (ab - a)) + a / (2 * c) * math.log((ab + b) / (ab - b))
         + c / (2 * a) * math.log((bc - b) / (bc + b)) + c / (2 * b) * math.log((ac - a) / (ac + a))
         + 2 * math.atan(a * b / (c * r)) + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r + c / (a * b) * (ac + bc)
         - ((a * a + b * b) ** 1.5 + (b * b + c * c) ** 1.5 + (c * c + a * a) ** 1.5)
         / (3 * a * b * c))
    return t / math.pi


def prism_factors(dx, dy, dz):
    """(Dx, Dy, Dz) of a dx x dy x dz prism by Aharoni's formula, axes relabelled."""
    a, b, c = dx / 2, dy / 2, dz / 2
    return aharoni_Dz(b, c, a), aharoni_Dz(c, a, b), aharoni_Dz(a, b, c)


def dipole_tensor(X, Y, Z, V):
    """-V (3 r r / r^2 - I) / (4 pi r^3) as (xx, yy, zz, xy, xz, yz): the field of
    a point moment V M is H = -N M."""
    r = np.array([X, Y, Z], dtype=float)
    rr = np.linalg.norm(r)
    u = r / rr
    D = -V * (3 * np.outer(u, u) - np.eye(3)) / (4 * math.pi * rr ** 3)
    return np.array([D[0, 0], D[1, 1], D[2, 2], D[0, 1], D[0, 2], D[1, 2]])


@pytest.mark.parametrize("edges", [(1.0, 1.0, 1.0), (1.0, 2.0, 0.5), (2.0, 6.0, 0.4),
                                   (4.0, 1.4, 2.6), (0.3e-9, 0.3e-9, 0.9e-9)])
def test_self_term_is_the_prism_demagnetising_factor(edges):
    """A cell's tensor on itself is the demagnetising tensor of the prism: diagonal,
    equal to Aharoni's factors, trace 1."""
    N = oracle.newell_tensor(0.0, 0.0, 0.0, *edges)
    D = prism_factors(*edges)
    np.testing.assert_allclose(N[:3], D, rtol=0, atol=5e-14)
    assert abs(N[:3].sum() - 1.0) < 5e-15
    assert np.all(np.abs(N[3:]) < 1e-15)


def test_self_term_limits():
    """Cube 1/3 each; a thin plate has Nzz -> 1, a long rod Nzz -> 0 and Nxx = Nyy -> 1/2."""
    np.testing.assert_allclose(oracle.newell_tensor(0, 0, 0, 1, 1, 1)[:3], 1 / 3, atol=1e-15)
    # 1 - Nzz of a plate of aspect t falls like t ln(1/t)
    gaps = [1 - oracle.newell_tensor(0, 0, 0, 1.0, 1.0, t)[2] for t in (1e-2, 1e-3, 1e-4)]
    assert gaps[0] < 0.05 and gaps[1] < 0.006 and gaps[2] < 0.0008
    assert gaps[0] > gaps[1] > gaps[2] > 0
    rod = oracle.newell_tensor(0, 0, 0, 1e-3, 1e-3, 1.0)
    assert rod[2] < 2e-3 and abs(rod[0] - 0.5) < 1e-3 and rod[0] == pytest.approx(rod[1], abs=1e-15)


def test_parities_and_relabelling():
    """Diagonal terms are even in every coordinate; N_xy is odd in X and Y and even in Z
    (likewise N_xz, N_yz); swapping x and y swaps N_xx and N_yy and N_xz and N_yz.
    Tolerance: each entry is a 27-term difference of values ~R^3 / (4 pi V) ~ 10,
    so evaluation order moves it by ~27 * 1e-16 * 10 ~ 3e-14 absolute."""
    d = (1.0, 1.3, 0.7)
    X, Y, Z = 2.0, -1.3, 1.4
    N = oracle.newell_tensor(X, Y, Z, *d)
    for sx, sy, sz in [(-1, 1, 1), (1, -1, 1), (1, 1, -1), (-1, -1, -1)]:
        M = oracle.newell_tensor(sx * X, sy * Y, sz * Z, *d)
        np.testing.assert_allclose(M[:3], N[:3], rtol=0, atol=1e-13)
        np.testing.assert_allclose(M[3], sx * sy * N[3], rtol=0, atol=1e-13)
        np.testing.assert_allclose(M[4], sx * sz * N[4], rtol=0, atol=1e-13)
        np.testing.assert_allclose(M[5], sy * sz * N[5], rtol=0, atol=1e-13)
    S = oracle.newell_tensor(Y, X, Z, d[1], d[0], d[2])
    np.testing.assert_allclose(S[[1, 0, 2, 3, 5, 4]], N, rtol=0, atol=1e-13)


@pytest.mark.parametrize("edges,order", [((1.0, 1.0, 1.0), 4), ((1.0, 1.5, 0.6), 2)])
def test_far_field_is_the_point_dipole(edges, order):
    """At distance R the cell-averaged tensor approaches the point-dipole tensor with
    relative error O((d/R)^2), O((d/R)^4) for a cube (its quadrupole vanishes)."""
    V = edges[0] * edges[1] * edges[2]
    u = np.array([0.6, 0.48, 0.64])
    errs = []
    for R in (5.0, 10.0, 20.0):
        X, Y, Z = R * u
        N = oracle.newell_tensor(X, Y, Z, *edges)
        D = dipole_tensor(X, Y, Z, V)
        errs.append(np.max(np.abs(N - D)) / np.max(np.abs(D)))
    assert errs[2] < (0.5 if order == 2 else 0.02) * (1 / 20) ** order * 20
    for e0, e1 in zip(errs, errs[1:]):
        assert abs(math.log2(e0 / e1) - order) < 0.3


def test_direct_sum_single_cell_gives_dipole_field():
    """One magnetised cell in the mesh: Eq. 7 gives its field at every other cell;
    far from it this is the point-dipole field of the moment V M (catches a
    transposed component or a wrong displacement index)."""
    nx, ny, nz, d = 14, 11, 9, (1.0, 1.2, 0.8)
    n = nx * ny * nz
    M = np.zeros((3, n))
    j = 0 + nx * (1 + ny * 2)  # cell (0, 1, 2)
    m = np.array([0.3, -0.5, 0.8]) * 1e6
    M[:, j] = m
    H = oracle.demag_direct(M, nx, ny, nz, *d)
    V = d[0] * d[1] * d[2]
    for (ix, iy, iz) in [(13, 10, 8), (13, 1, 2), (0, 10, 8), (9, 10, 0), (13, 4, 8)]:
        i = ix + nx * (iy + ny * iz)
        r = np.array([(0 - ix) * d[0], (1 - iy) * d[1], (2 - iz) * d[2]])  # r_j - r_i
        D = dipole_tensor(*r, V)
        T = np.array([[D[0], D[3], D[4]], [D[3], D[1], D[5]], [D[4], D[5], D[2]]])
        expect = -T @ m
        R = np.linalg.norm(r) / max(d)
        assert np.linalg.norm(H[:, i] - expect) <= 2.0 / R ** 2 * np.linalg.norm(expect), (ix, iy, iz)
    # the cell's own field is its prism factor
    D = prism_factors(*d)
    np.testing.assert_allclose(H[:, j], -np.array(D) * m, rtol=1e-12)


def test_direct_sum_uniform_body_mean_field():
    """Uniform M over a box of cells: the mean of Eq. 7 over the cells is
    -D_body M with D_body the box's demagnetising factors (Aharoni), since the
    cell-averaged tensors of all pairs add up to the body's own."""
    nx, ny, nz, d = 9, 6, 4, (1.0, 1.3, 0.7)
    n = nx * ny * nz
    Db = prism_factors(nx * d[0], ny * d[1], nz * d[2])
    for m in ([1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0], [0.3, -0.4, 0.5]):
        m = np.array(m) * 8e5
        M = np.repeat(m[:, None], n, axis=1)
        H = oracle.demag_direct(M, nx, ny, nz, *d)
        np.testing.assert_allclose(H.mean(axis=1), -np.array(Db) * m, rtol=0, atol=1e-9 * 8e5)


def test_heun_with_demag_is_macrospin_with_shape_anisotropy():
    """A uniformly magnetised SC block that is one coarse cell, at T = 0: exchange
    keeps it uniform and the demagnetising field -mu0 Ms N m adds the shape
    anisotropy mu0 Ms^2 (Nxx - Nzz) V / 2 to k_u (Nxx = Nyy), so every spin follows
    a free spin with k_eff = k_u - mu_s mu0 Ms (Nzz - Nxx) / 2, step for step."""
    w = W.c1_plain_sc().scaled(nx=6, ny=6, nz=2, bc=(0, 0, 0), B=(0.0, 0.0, -0.5), T_amb=0.0,
                               ku=2.6e-22)
    sysm = oracle_system(w)
    n = w.n_sites
    dd = (w.nx * w.a, w.ny * w.a, w.nz * w.a)
    sysm.set_demag(((1, 1, 1), dd, np.zeros(n, np.int32)))
    th, ph = 0.4, 0.2
    s0 = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    S = np.repeat(s0[:, None], n, axis=1)
    steps = 400
    Sg = sysm.heun(S, 0, steps)
    N = oracle.newell_tensor(0, 0, 0, *dd)
    Ms = w.mu_s / w.a ** 3
    keff = w.ku - w.mu_s * oracle.MU0 * Ms * (N[2] - N[0]) / 2
    free = free_spins_system(1, mu_s=w.mu_s, alpha=w.alpha, gamma=w.gamma, dt=w.dt, ku=keff,
                             B=w.B, T=0.0)
    Sf = free.heun(s0[:, None], 0, steps)[:, 0]
    assert np.max(np.abs(Sg - Sg[:, :1])) < 1e-13  # stays uniform
    assert np.max(np.abs(Sg[:, 0] - Sf)) < 1e-11
    # the demagnetising field changed the motion (flat block: k_eff < k_u)
    assert keff < w.ku
    nodemag = oracle_system(w).heun(S, 0, steps)
    assert np.max(np.abs(nodemag[:, 0] - Sf)) > 1e-6


@pytest.mark.parametrize("origin,cell", [(0, (3, 2, 2)), (5, (3, 2, 2)), (7, (4, 3, 5))])
def test_track_stray_plus_window_field_is_whole_track_field(origin, cell):
    """Superposition on the window's cells: the field of the window's own sites
    (window mesh) plus the frozen track's (track mesh aligned with it) equals
    the field of all stored sites on the track mesh, read at the window cells."""
    w = W.c5_track_window().scaled(nx=14, ny=6, nz=5, track_nx=26, grains=False)
    n = w.track_nx * w.ny * w.nz
    S = W.random_spins(n, 3)
    dn, dd, dcell = demag_cells(w, cell, origin)
    own = oracle.demag_field(S, dcell, dn, dd, w.mu_s)
    stray = track_stray(w, cell, origin, S)
    # all stored sites on the track mesh
    cx, cy, cz = cell
    idx = np.arange(n)
    xw, y, z = idx % w.track_nx - origin, (idx // w.track_nx) % w.ny, idx // (w.track_nx * w.ny)
    i0 = -(-origin // cx)
    it = xw // cx + i0
    nt = int(it.max()) + 1
    dall = (it + nt * (y // cy + dn[1] * (z // cz))).astype(np.int32)
    Ball = oracle.demag_field(S, dall, (nt, dn[1], dn[2]), dd, w.mu_s)
    i, j, k = np.meshgrid(np.arange(dn[0]), np.arange(dn[1]), np.arange(dn[2]), indexing="ij")
    win = (i + i0 + nt * (j + dn[1] * k)).transpose(2, 1, 0).reshape(-1)
    np.testing.assert_allclose(own + stray, Ball[:, win], rtol=0, atol=1e-12)
    assert np.max(np.abs(stray)) > 1e-3


def test_field_once_per_step_is_a_field_held_through_the_step():
    """Reading in which the demagnetising field is evaluated once per step: one
    coarse cell covering a block gives one field, B_d(S_n), at every site; held
    through both Heun stages it must act exactly like a uniform applied field of
    that value (polarity +1), to rounding.  A slip that re-evaluates the field
    at S' (the other reading), drops it from a stage, or takes it from another
    configuration, moves the spins by far more than rounding."""
    w = W.c1_plain_sc().scaled(nx=5, ny=4, nz=3, bc=(0, 0, 0), B=(0.05, -0.02, 0.3), T_amb=300.0)
    n = w.n_sites
    dd = (w.nx * w.a, w.ny * w.a, w.nz * w.a)
    rng = np.random.default_rng(11)
    S0 = rng.normal(size=(3, n))
    S0 /= np.linalg.norm(S0, axis=0)
    one = ((1, 1, 1), dd, np.zeros(n, np.int32))
    Bd = oracle.demag_field(S0, np.zeros(n, np.int32), (1, 1, 1), dd, w.mu_s)[:, 0]
    assert np.max(np.abs(Bd)) > 1e-3  # a random state still has a net moment
    once = oracle_system(w)
    once.set_demag(one, once=True)
    S_once = once.heun(S0, 0, 1)
    held = oracle_system(w.scaled(B=tuple(np.asarray(w.B) + Bd)))
    S_held = held.heun(S0, 0, 1)
    assert np.max(np.abs(S_once - S_held)) < 1e-13
    each = oracle_system(w)
    each.set_demag(one)
    S_each = each.heun(S0, 0, 1)
    assert np.max(np.abs(S_each - S_once)) > 1e3 * np.max(np.abs(S_once - S_held))
    # several steps: the held field is re-evaluated at the start of each step
    S2 = once.heun(S0, 0, 2)
    Bd1 = oracle.demag_field(S_once, np.zeros(n, np.int32), (1, 1, 1), dd, w.mu_s)[:, 0]
    S2_held = oracle_system(w.scaled(B=tuple(np.asarray(w.B) + Bd1))).heun(S_held, 1, 1)
    assert np.max(np.abs(S2 - S2_held)) < 1e-12
