"""A whole step captured in a HIP graph and replayed: every replay must equal
the eager step bit for bit, with the program's own eager work and
synchronisations between replays."""
import numpy as np
import pytest
import torch

from gpu_helpers import to_dev
from paper_0909_0541_amd import inputs

pytestmark = pytest.mark.gpu


def _eager(bh, off, pos, mass, n_crit, eps, theta):
    c = bh.Context()
    if len(off) == 2:
        c.build_tree(pos, mass)
        c.make_groups(n_crit)
        a, p = c.compute_forces(float(eps[0]), float(theta[0]))
    else:
        c.build_batch(off, pos, mass)
        c.make_groups(n_crit)
        a, p = c.compute_forces_batch(eps, theta)
    torch.cuda.synchronize()
    return a.clone(), p.clone()


def _cases():
    p, m = inputs.clustered(30000, 41, n_halos=30)[:2]
    bp, bm, boff, beps = inputs.batch_systems(seed=9, n_systems=10, n_min=500, n_max=8000)
    return [("single", np.array([0, p.shape[0]]), p, m, 64, np.array([1e-3]), np.array([0.6])),
            ("batch", boff, bp, bm, 32, beps, np.full(10, 0.7))]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_replays_equal_eager(gpu, case):
    bh = gpu
    name, off, pos, mass, n_crit, eps, theta = case
    dpos, dmass = to_dev(pos), to_dev(mass)
    a0, p0 = _eager(bh, off, dpos, dmass, n_crit, eps, theta)
    c = bh.Context()
    acc, pot = c.graph_capture(off, dpos, dmass, n_crit, eps, theta)
    torch.cuda.synchronize()
    assert torch.equal(acc, a0) and torch.equal(pot, p0), "eager step of the capture"
    for k in range(4):
        acc.fill_(float("nan"))
        pot.zero_()
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        c.graph_launch()
        c.sync()
        assert torch.equal(acc, a0) and torch.equal(pot, p0), f"replay {k}"
        assert float(junk) == float(junk)
    assert c.get_stats().error_flags == 0


def test_replay_on_moved_particles(gpu):
    bh = gpu
    pos, mass, vel = inputs.plummer(20000, 42, with_vel=True)
    dpos, dmass, dvel = to_dev(pos), to_dev(mass), to_dev(vel)
    off = np.array([0, 20000])
    c = bh.Context()
    acc, pot = c.graph_capture(off, dpos, dmass, 64, [1 / 256], [0.6])
    for k in range(3):
        c.drift(dpos, dvel, 1e-3)  # move the particles in place
        c.graph_launch()
        c.sync()
        a1, p1 = _eager(bh, off, dpos, dmass, 64, np.array([1 / 256]), np.array([0.6]))
        assert torch.equal(acc, a1) and torch.equal(pot, p1), f"step {k}"


def test_launch_without_capture(gpu):
    bh = gpu
    c = bh.Context()
    with pytest.raises(bh.BHError):
        c.graph_launch()


@pytest.mark.parametrize("opts", [{"quadrupole": True}, {"curve": 1}, {"quadrupole": True, "curve": 1}],
                         ids=["quadrupole", "peano_hilbert", "both"])
def test_replays_equal_eager_with_options(gpu, opts):
    bh = gpu
    pos, mass = inputs.clustered(30000, 43, n_halos=30)[:2]
    off = np.array([0, pos.shape[0]])
    dpos, dmass = to_dev(pos), to_dev(mass)
    e = bh.Context(**opts)
    e.build_tree(dpos, dmass)
    e.make_groups(64)
    a0, p0 = e.compute_forces(1e-3, 0.7)
    a0, p0 = a0.clone(), p0.clone()
    c = bh.Context(**opts)
    acc, pot = c.graph_capture(off, dpos, dmass, 64, np.array([1e-3]), np.array([0.7]))
    torch.cuda.synchronize()
    assert torch.equal(acc, a0) and torch.equal(pot, p0), "eager step of the capture"
    for k in range(3):
        acc.fill_(float("nan"))
        torch.cuda.synchronize()
        c.graph_launch()
        c.sync()
        assert torch.equal(acc, a0) and torch.equal(pot, p0), f"replay {k}"
    assert c.get_stats().error_flags == 0
