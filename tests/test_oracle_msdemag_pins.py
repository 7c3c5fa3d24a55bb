"""Pins of the oracle's demagnetising field of the multiscale window (Sec. II,
Eq. 7, Fig. 1): the field a micromagnetic region holds through its RK4 step
acts exactly like an applied field; the window's meshes laid along x as one
mesh reproduce, for a uniformly magnetised body at T = 0 whose atomistic and
micromagnetic parts carry the same magnetisation, the field of that body
computed as a single mesh; the regions' part scales with m_e(T); the right
region sits on the far side of the atoms (mirror symmetry); the split into
the regions' part and the rest adds up.
"""
import numpy as np
import pytest

import oracle

GAMMA = 1.76e11
A = 0.3e-9
MU_S = 2.99550525e-23
TC = 710.0
CELL = (2, 3, 2)
DD = (CELL[0] * A, CELL[1] * A, CELL[2] * A)


def region(nx, ny, nz, **kw):
    args = dict(n=(nx, ny, nz), h=DD, Ms0=MU_S / A ** 3, A0=6.7e-21 / (2 * A), K0=2.6e-22 / A ** 3,
                lam=0.1, gamma=GAMMA, Tc=TC, mu_s=MU_S, dt=1e-15)
    args.update(kw)
    return oracle.MM(**args)


def random_unit(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(3, n))
    return v / np.linalg.norm(v, axis=0)


def test_held_field_acts_as_an_applied_field():
    """A held field along x equals a write field along x, step for step and
    bit for bit (mu_s = 0 so that m_e does not see the write field; the field
    enters after the exchange and anisotropy terms, which have no x part
    beyond the exchange one)."""
    n = (4, 3, 2)
    m0 = random_unit(24, 1)
    Bx = 0.37
    a = region(*n, mu_s=0.0, T_amb=300.0)
    a.set_field(np.stack([np.full(24, Bx), np.zeros(24), np.zeros(24)]))
    b = region(*n, mu_s=0.0, T_amb=300.0, B=(Bx, 0.0, 0.0))
    ma, mb = a.rk4(m0, 0, 25), b.rk4(m0, 0, 25)
    np.testing.assert_array_equal(ma, mb)
    # and it matters: without it the region moves elsewhere
    c = region(*n, mu_s=0.0, T_amb=300.0)
    assert np.max(np.abs(c.rk4(m0, 0, 25) - ma)) > 1e-6
    # removing it restores the plain region
    a.set_field(None)
    np.testing.assert_array_equal(a.rk4(m0, 0, 25), c.rk4(m0, 0, 25))


def uniform_window(nL, ncxA, nR, ny, nz, direction=(0.0, 0.0, 1.0), T=0.0):
    d = np.asarray(direction, np.float64)
    L = region(nL, ny, nz, T_amb=T) if nL else None
    R = region(nR, ny, nz, T_amb=T) if nR else None
    mL = np.tile(d[:, None], (1, nL * ny * nz)) if nL else None
    mR = np.tile(d[:, None], (1, nR * ny * nz)) if nR else None
    nsite = CELL[0] * CELL[1] * CELL[2]
    sums = np.zeros((ncxA * ny * nz, 4))
    sums[:, :3] = nsite * d
    sums[:, 3] = nsite
    return L, mL, sums, R, mR


@pytest.mark.parametrize("direction", [(0.0, 0.0, 1.0), (0.6, 0.0, 0.8), (0.0, 1.0, 0.0)])
def test_uniform_body_across_meshes_equals_one_mesh(direction):
    """At T = 0 (m_e = 1) with M_S0 = mu_s / a^3, a fully magnetic atomistic
    cell of aligned spins and a region cell along the same direction carry the
    same magnetisation; the window laid out as one mesh must then give the
    field of one uniformly magnetised box (computed as a single mesh), within
    rounding.  A wrong cell volume, a missing M_S0 or m_e, or a misplaced mesh
    breaks it."""
    nL, ncxA, nR, ny, nz = 3, 4, 2, 3, 2
    L, mL, sums, R, mR = uniform_window(nL, ncxA, nR, ny, nz, direction)
    Ball, Breg = oracle.multiscale_demag(L, mL, sums, ncxA, R, mR, 0.0, DD, MU_S)
    NX = nL + ncxA + nR
    Ms = MU_S / A ** 3
    M = np.tile((Ms * np.asarray(direction))[:, None], (1, NX * ny * nz))
    ref = oracle.MU0 * oracle.demag_direct(M, NX, ny, nz, *DD)
    scale = oracle.MU0 * Ms
    assert np.max(np.abs(Ball - ref)) < 1e-13 * scale
    # the regions' part plus the atoms' part is the whole
    M_at = M.copy()
    for c in range(NX * ny * nz):
        if not (nL <= c % NX < nL + ncxA):
            M_at[:, c] = 0.0
    B_at = oracle.MU0 * oracle.demag_direct(M_at, NX, ny, nz, *DD)
    assert np.max(np.abs(Breg + B_at - Ball)) < 1e-13 * scale
    # inside a body magnetised along z the field opposes M
    if direction == (0.0, 0.0, 1.0):
        assert np.all(Ball[2] < 0)


def test_region_part_scales_with_equilibrium_magnetisation():
    """Uniform T below T_C: the regions' magnetisation is M_S0 m_e(T) m, so
    their field is m_e(T) times the T = 0 one (m_e from the Curie-Weiss root,
    pinned elsewhere); the atoms' part does not depend on the regions' T."""
    nL, ncxA, nR, ny, nz = 2, 3, 2, 2, 2
    L0, mL, sums, R0, mR = uniform_window(nL, ncxA, nR, ny, nz, (0.0, 0.6, 0.8), T=0.0)
    LT, _, _, RT, _ = uniform_window(nL, ncxA, nR, ny, nz, (0.0, 0.6, 0.8), T=520.0)
    me = oracle.mm_me(520.0, TC, 0.0)
    assert 0.2 < me < 0.9
    _, B0 = oracle.multiscale_demag(L0, mL, sums, ncxA, R0, mR, 0.0, DD, MU_S)
    ball_T, BT = oracle.multiscale_demag(LT, mL, sums, ncxA, RT, mR, 0.0, DD, MU_S)
    np.testing.assert_allclose(BT, me * B0, rtol=1e-13, atol=1e-16)
    ball_0, _ = oracle.multiscale_demag(L0, mL, sums, ncxA, R0, mR, 0.0, DD, MU_S)
    NX = nL + ncxA + nR
    atoms = [c for c in range(NX * ny * nz) if nL <= c % NX < nL + ncxA]
    np.testing.assert_allclose((ball_T - BT)[:, atoms], (ball_0 - B0)[:, atoms], rtol=1e-12,
                               atol=1e-15)


def test_right_region_mirrors_left_region():
    """Equal regions either side of an empty atomistic window, magnetised along
    z: their field in the window is mirror-symmetric about its centre (B_z
    even, B_x odd along x); a right region placed anywhere but beyond the
    atoms breaks the symmetry."""
    nL = nR = 3
    ncxA, ny, nz = 5, 3, 2
    L, mL, sums, R, mR = uniform_window(nL, ncxA, nR, ny, nz)
    sums[:] = 0.0
    _, Breg = oracle.multiscale_demag(L, mL, sums, ncxA, R, mR, 0.0, DD, MU_S)
    NX = nL + ncxA + nR
    B = Breg.reshape(3, nz, ny, NX)[:, :, :, nL:nL + ncxA]
    scale = np.abs(B).max()
    assert scale > 0
    np.testing.assert_allclose(B[2], B[2][:, :, ::-1], rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(B[0], -B[0][:, :, ::-1], rtol=0, atol=1e-13 * scale)
    assert np.abs(B[0]).max() > 1e-3 * scale
    # mesh_part picks the cells of one mesh in its own order
    part = oracle.mesh_part(Breg, NX, ny, nz, nL, ncxA)
    np.testing.assert_array_equal(part.reshape(3, nz, ny, ncxA), B)
