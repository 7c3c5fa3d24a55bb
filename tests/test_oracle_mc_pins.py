"""Pins of the oracle's Metropolis Monte Carlo (the exchange calibration of
Sec. III with Eq. 8) against closed forms of equilibrium statistical mechanics:
the Langevin function of free spins, Boltzmann quadrature of an anisotropic
spin in a field, the exact nearest-neighbour correlation of the classical
Heisenberg ring, and energy descent at zero temperature.  Statistical bars:
4 standard errors of block means plus 0.005.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle_build import checkerboard, free_spins_system, oracle_system

MU_S = 3.23 * W.MU_B
GAMMA = 1.76e11


def block_stats(samples):
    a = np.asarray(samples)
    return a.mean(), a.std(ddof=1) / math.sqrt(len(a))


def run_blocks(sysm, S, colour, burn, blocks, per_block, observable):
    S = sysm.mc(S, colour, 0, burn)
    out = []
    for b in range(blocks):
        S = sysm.mc(S, colour, burn + b * per_block, per_block)
        out.append(observable(S))
    return out


def test_mc_free_spins_follow_the_langevin_function():
    """Uncoupled spins in B z: <S_z> = coth x - 1/x with x = mu_s B / kB T."""
    n = 4096
    for B, T in ((5.0, 10.0), (20.0, 30.0)):
        s = free_spins_system(n, mu_s=MU_S, alpha=1.0, gamma=GAMMA, dt=1e-15, ku=0.0,
                              B=(0.0, 0.0, B), T=T, seed=41)
        x = MU_S * B / (W.KB * T)
        expect = 1 / math.tanh(x) - 1 / x
        S = np.stack([np.zeros(n), np.zeros(n), np.ones(n)])
        m, err = block_stats(run_blocks(s, S, np.zeros(n, np.int8), 20, 10, 20,
                                        lambda S: S[2].mean()))
        assert abs(m - expect) < 4 * err + 0.005, (B, T, m, expect, err)


def test_mc_anisotropic_spin_matches_boltzmann_quadrature():
    """<S_z>, <S_z^2> of exp[(k_u cos^2 t + mu_s B cos t) / kB T] over the sphere."""
    n, B, T, ku = 4096, 20.0, 100.0, 2.6e-22
    s = free_spins_system(n, mu_s=MU_S, alpha=1.0, gamma=GAMMA, dt=1e-15, ku=ku,
                          B=(0.0, 0.0, B), T=T, seed=42)
    beta = 1 / (W.KB * T)
    wfun = lambda c: math.exp(beta * (ku * c * c + MU_S * B * c))
    Z = integrate.quad(wfun, -1, 1)[0]
    m1 = integrate.quad(lambda c: c * wfun(c), -1, 1)[0] / Z
    m2 = integrate.quad(lambda c: c * c * wfun(c), -1, 1)[0] / Z
    S = np.stack([np.zeros(n), np.zeros(n), np.ones(n)])
    obs = run_blocks(s, S, np.zeros(n, np.int8), 30, 10, 20,
                     lambda S: (S[2].mean(), (S[2] ** 2).mean()))
    for k, ref in enumerate((m1, m2)):
        m, err = block_stats([o[k] for o in obs])
        assert abs(m - ref) < 4 * err + 0.005, (k, m, ref, err)


def test_mc_heisenberg_ring_correlation():
    """Classical Heisenberg ring (even length, periodic) at zero field:
    <S_i . S_i+1> = coth K - 1/K with K = J / kB T."""
    n, J = 2048, 6.7e-21
    for K in (0.5, 1.0, 2.0):
        T = J / (W.KB * K)
        w = W.Workload("ring", nx=n, ny=1, nz=1, bc=(1, 0, 0), J=(J,), ku=0.0,
                       B=(0.0, 0.0, 0.0), T_amb=T, seed=43)
        sysm = oracle_system(w)
        S = W.random_spins(n, 7)
        m, err = block_stats(run_blocks(sysm, S, checkerboard(w), 200, 10, 60,
                                        lambda S: (S * np.roll(S, -1, axis=1)).sum(0).mean()))
        expect = 1 / math.tanh(K) - 1 / K
        assert abs(m - expect) < 4 * err + 0.005, (K, m, expect, err)


def test_mc_zero_temperature_never_raises_the_energy():
    """At T = 0 only moves that do not raise the site energy are accepted, so the
    total energy (the oracle's independent energy sum) never increases."""
    w = W.c2_granular_slab().scaled(nx=12, ny=10, nz=4, grains=False, spot_mode=W.SPOT_NONE,
                                    T_amb=0.0, B=(0.0, 0.0, -0.8))
    sysm = oracle_system(w, T_amb=0.0)
    S = W.random_spins(w.n_sites, 9)
    col = checkerboard(w)
    e = [sysm.energy(S, 0)[3]]
    for t in range(8):
        S = sysm.mc(S, col, t, 1)
        e.append(sysm.energy(S, t + 1)[3])
    assert all(b <= a + 1e-30 for a, b in zip(e, e[1:]))
    assert e[-1] < e[0]
    assert np.max(np.abs(np.linalg.norm(S, axis=0) - 1)) < 1e-15


def test_mc_trial_directions_are_uniform_at_infinite_temperature():
    """With a vanishing Hamiltonian every move is accepted, so after one sweep each
    spin is its trial direction: uniform on the sphere (S_z uniform on (-1, 1),
    azimuth uniform)."""
    from scipy import stats
    n = 8000
    s = free_spins_system(n, mu_s=MU_S, alpha=1.0, gamma=GAMMA, dt=1e-15, ku=0.0,
                          B=(0.0, 0.0, 0.0), T=300.0, seed=44)
    S = s.mc(np.stack([np.zeros(n), np.zeros(n), np.ones(n)]), np.zeros(n, np.int8), 5, 1)
    assert stats.kstest((S[2] + 1) / 2, "uniform").pvalue > 1e-3
    phi = np.arctan2(S[1], S[0]) % (2 * math.pi)
    assert stats.kstest(phi / (2 * math.pi), "uniform").pvalue > 1e-3


@pytest.mark.parametrize("kind,dims,bc", [(W.SC, (6, 4, 4), (1, 1, 1)), (W.SC, (5, 3, 3), (0, 0, 0)),
                                          (W.L10, (4, 4, 4), (1, 1, 1)), (W.L10, (5, 3, 3), (0, 0, 0))])
def test_mc_colours_never_pair_neighbours(kind, dims, bc):
    """The Monte Carlo colours form independent sets of the neighbour graph (all
    four L1_0 shells), so one colour can be updated at once."""
    import oracle
    nx, ny, nz = dims
    w = W.Workload("c", kind=kind, nx=nx, ny=ny, nz=nz, bc=bc,
                   a=0.385e-9 if kind == W.L10 else 0.3e-9, c=0.371e-9 if kind == W.L10 else 0.3e-9,
                   J=(6.0e-21, 1.2e-21, 0.5e-21, 0.2e-21) if kind == W.L10 else (6.7e-21,))
    row, col, _ = oracle.neighbours(kind, nx, ny, nz, list(bc), w.a, w.c, w.shell_radii)
    colour = checkerboard(w)
    assert colour.max() == (1 if kind == W.SC else 7)
    for i in range(len(colour)):
        for k in range(row[i], row[i + 1]):
            assert colour[col[k]] != colour[i], (i, col[k])


def test_mc_l10_zero_temperature_descent():
    """L1_0, four shells, T = 0: the oracle's independent energy never increases."""
    w = W.c3_l10_window().scaled(nx=6, ny=6, nz=4, grains=False, spot_mode=W.SPOT_NONE,
                                 T_amb=0.0, bc=(1, 1, 0))
    sysm = oracle_system(w, T_amb=0.0)
    S = W.random_spins(w.n_sites, 4)
    col = checkerboard(w)
    e = [sysm.energy(S, 0)[3]]
    for t in range(6):
        S = sysm.mc(S, col, t, 1)
        e.append(sysm.energy(S, t + 1)[3])
    assert all(b <= a + 1e-30 for a, b in zip(e, e[1:])) and e[-1] < e[0]
