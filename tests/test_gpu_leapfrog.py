"""FP64 state and kick-drift-kick leapfrog on the GPU against the FP64 oracle."""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import to_dev
from oracle import integrate
from paper_0909_0541_amd import inputs
from test_oracle_integrate import kepler_pair

pytestmark = pytest.mark.gpu


def test_kick_drift_bit_exact(gpu):
    bh = gpu
    rng = np.random.default_rng(5)
    n = 10007
    v = rng.normal(size=(n, 3))
    x = rng.normal(size=(n, 3))
    a = rng.normal(size=(n, 3)).astype(np.float32)
    c = bh.Context()
    dv, dx, da = to_dev(v), to_dev(x), to_dev(a, torch.float32)
    c.kick(dv, da, 0.37)
    c.drift(dx, dv, 0.011)
    v1 = v + 0.37 * a.astype(np.float64)
    x1 = x + 0.011 * v1
    assert np.array_equal(dv.cpu().numpy(), v1)
    assert np.array_equal(dx.cpu().numpy(), x1)


def test_energy_sums(gpu):
    bh = gpu
    pos, m, vel = inputs.plummer(50000, 31, with_vel=True)
    pot = np.random.default_rng(2).uniform(-2, -0.5, 50000).astype(np.float32)
    c = bh.Context()
    e = c.energy(to_dev(vel), to_dev(m), to_dev(pot, torch.float32)).cpu().numpy()
    k, u = integrate.energy(vel, m, pot.astype(np.float64))
    assert abs(e[0] - k) <= 1e-11 * abs(k) and abs(e[1] - u) <= 1e-11 * abs(u)


def _gpu_forces(c, x, m, eps, theta, n_crit):
    c.build_tree(x, m)
    c.make_groups(n_crit)
    return c.compute_forces(eps, theta)


def test_leapfrog_matches_oracle_and_manual_steps(gpu):
    bh = gpu
    pos, m, vel = inputs.plummer(4096, 32, with_vel=True)
    eps, theta, n_crit, dt, steps = 1.0 / 256, 0.6, 64, 1e-3, 5
    c = bh.Context()
    x, v, dm = to_dev(pos), to_dev(vel), to_dev(m)
    acc, pot = _gpu_forces(c, x, dm, eps, theta, n_crit)
    amax = float(acc.abs().max())
    # the same steps by hand through the single-step entry points
    c2 = bh.Context()
    x2, v2 = x.clone(), v.clone()
    a2, p2 = acc.clone(), pot.clone()
    c.leapfrog(x, v, dm, eps, theta, n_crit, dt, steps, acc, pot)
    for _ in range(steps):
        c2.kick(v2, a2, 0.5 * dt)
        c2.drift(x2, v2, dt)
        a2, p2 = _gpu_forces(c2, x2, dm, eps, theta, n_crit)
        c2.kick(v2, a2, 0.5 * dt)
    assert torch.equal(x, x2) and torch.equal(v, v2) and torch.equal(acc, a2) and torch.equal(pot, p2)
    assert c.get_stats().error_flags == 0
    xo, vo, ao, po = integrate.leapfrog(pos, vel, m, eps, theta, n_crit, dt, steps)
    # FP32 forces within 1e-5 * max|a| per step (the force parity bar, taken
    # against the largest force) bound the drift of velocities and positions
    dv = np.max(np.abs(v.cpu().numpy() - vo))
    dx = np.max(np.abs(x.cpu().numpy() - xo))
    assert dv <= steps * dt * 1e-5 * amax, dv
    assert dx <= steps * steps * dt * dt * 1e-5 * amax, dx


def test_leapfrog_time_reversible(gpu):
    bh = gpu
    pos, m, vel = inputs.plummer(2048, 33, with_vel=True)
    eps, theta, n_crit, dt = 1.0 / 128, 0.6, 64, 1e-3
    c = bh.Context()
    x, v, dm = to_dev(pos), to_dev(vel), to_dev(m)
    acc, pot = _gpu_forces(c, x, dm, eps, theta, n_crit)
    c.leapfrog(x, v, dm, eps, theta, n_crit, dt, 10, acc, pot)
    assert float((x - to_dev(pos)).abs().max()) > 1e-3
    v.neg_()
    c.leapfrog(x, v, dm, eps, theta, n_crit, dt, 10, acc, pot)
    assert float((x - to_dev(pos)).abs().max()) < 1e-9
    assert float((v + to_dev(vel)).abs().max()) < 1e-7


def test_kepler_orbit_energy_and_period(gpu):
    bh = gpu
    pos, vel, m = kepler_pair()
    eps, steps = 1e-6, 4000
    c = bh.Context()
    x, v, dm = to_dev(pos), to_dev(vel), to_dev(m)
    acc, pot = _gpu_forces(c, x, dm, eps, 0.5, 2)
    e0 = c.energy(v, dm, pot).cpu().numpy().sum()
    assert abs(e0 + 0.125) < 1e-7  # -m1 m2 / (2a), FP32 potential
    c.leapfrog(x, v, dm, eps, 0.5, 2, 2.0 * math.pi / steps, steps, acc, pot)
    e1 = c.energy(v, dm, pot).cpu().numpy().sum()
    assert abs(e1 - e0) < 1e-4 * 0.125
    assert float((x - to_dev(pos)).abs().max()) < 1e-3


def test_leapfrog_argument_errors(gpu):
    bh = gpu
    c = bh.Context()
    x = to_dev(np.zeros((4, 3)))
    v = to_dev(np.zeros((4, 3)))
    m = to_dev(np.ones(4))
    a = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    p = torch.zeros(4, dtype=torch.float32, device="cuda")
    with pytest.raises(bh.BHError):
        c.leapfrog(x, v, m, 0.1, 0.5, 8, 1e-3, -1, a, p)
    with pytest.raises(bh.BHError):
        c.leapfrog(x, v, m, 0.1, 0.5, 0, 1e-3, 1, a, p)
    with pytest.raises(bh.BHError):
        c.leapfrog(x, v, m, 0.1, 0.5, 8, float("nan"), 1, a, p)
    c.leapfrog(x, v, m, 0.1, 0.5, 8, 1e-3, 0, a, p)  # zero steps: nothing happens
