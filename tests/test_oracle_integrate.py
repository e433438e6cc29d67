"""Pins of the oracle's kick-drift-kick leapfrog against the mechanics it must obey."""
import math

import numpy as np

import oracle
from oracle import integrate
from paper_0909_0541_amd import inputs


def kepler_pair(a=1.0, e=0.5):
    """Two equal masses (total 1) at apoapsis of a relative orbit with
    semi-major axis a and eccentricity e, centre of mass at rest at 0."""
    ra = a * (1.0 + e)
    va = math.sqrt((1.0 - e) / (a * (1.0 + e)))  # G M = 1
    pos = np.array([[0.5 * ra, 0.0, 0.0], [-0.5 * ra, 0.0, 0.0]])
    vel = np.array([[0.0, 0.5 * va, 0.0], [0.0, -0.5 * va, 0.0]])
    return pos, vel, np.array([0.5, 0.5])


def test_kepler_energy_closed_form_and_one_period():
    pos, vel, m = kepler_pair()
    eps = 1e-6
    a0, p0 = integrate.forces(pos, m, eps, 0.0, 2)
    k0, u0 = integrate.energy(vel, m, p0)
    # E = -G m1 m2 / (2 a) for the bound pair
    assert abs((k0 + u0) - (-0.125)) < 1e-10
    period = 2.0 * math.pi  # 2 pi sqrt(a^3 / (G M))
    steps = 4000
    x, v, a, p = integrate.leapfrog(pos, vel, m, eps, 0.0, 2, period / steps, steps, acc=a0)
    k1, u1 = integrate.energy(v, m, p)
    assert abs((k1 + u1) - (k0 + u0)) < 1e-4 * 0.125
    assert np.max(np.abs(x - pos)) < 1e-3  # back at apoapsis after one period
    # momentum of an isolated pair stays zero
    assert np.max(np.abs((m[:, None] * v).sum(axis=0))) < 1e-14


def test_time_reversibility():
    pos, m, vel = inputs.plummer(256, 21, with_vel=True)
    eps, theta, n_crit, dt = 1e-2, 0.5, 16, 1e-3
    x, v, a, _ = integrate.leapfrog(pos, vel, m, eps, theta, n_crit, dt, 10)
    assert np.max(np.abs(x - pos)) > 1e-3  # it moved
    xb, vb, _, _ = integrate.leapfrog(x, -v, m, eps, theta, n_crit, dt, 10, acc=a)
    assert np.max(np.abs(xb - pos)) < 1e-12
    assert np.max(np.abs(vb + vel)) < 1e-12


def test_free_particle_and_momentum_with_direct_forces():
    x, v, _, _ = integrate.leapfrog(np.array([[0.1, 0.2, 0.3]]), np.array([[1.0, -2.0, 0.5]]), np.array([1.0]),
                                    1e-2, 0.0, 1, 0.25, 8)
    assert np.allclose(x, [[2.1, -3.8, 1.3]], rtol=0, atol=1e-14)
    pos, m, vel = inputs.plummer(64, 22, with_vel=True)
    x, v, _, _ = integrate.leapfrog(pos, vel, m, 1e-2, 0.0, 8, 1e-3, 20)
    p0 = (m[:, None] * vel).sum(axis=0)
    p1 = (m[:, None] * v).sum(axis=0)
    assert np.max(np.abs(p1 - p0)) < 1e-14


def test_energy_matches_definition_on_plummer():
    pos, m, vel = inputs.plummer(512, 23, with_vel=True)
    acc, pot = oracle.direct(pos, m, 1e-3)
    k, u = integrate.energy(vel, m, pot)
    # virial equilibrium of a Plummer sphere: 2K + U ~ 0 within sampling noise
    assert abs(2 * k + u) < 0.15 * abs(u)
    # the pairwise potential energy counted once per pair
    d = pos[:, None, :] - pos[None, :, :]
    r = np.sqrt((d * d).sum(-1) + 1e-6)
    np.fill_diagonal(r, np.inf)
    u_pairs = -0.5 * np.sum(m[:, None] * m[None, :] / r)
    assert abs(u - u_pairs) < 1e-12 * abs(u)
