"""Peano-Hilbert order (bh_options.curve = 1) against the oracle built in
the same order: keys and permutation bit-exact, the tree (topology and FP64
moments, summed over the children in curve order on both sides) bit-exact,
groups and list lengths exact, forces to the parity bar; a batch equals its
systems run alone bit for bit; and Morton order stays the default."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import check_forces, gpu_nodes, oracle_nonchain_nodes, to_dev
from paper_0909_0541_amd import inputs

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(5)
    dup = np.concatenate([np.tile([[0.1, 0.2, 0.3]], (300, 1)), rng.uniform(-1, 1, (700, 3))])
    lattice = np.stack(np.meshgrid(*[np.arange(6.0)] * 3, indexing="ij"), -1).reshape(-1, 3)
    return {
        "plummer_8k": (inputs.plummer(8192, 1, with_vel=False)[0], 1.0 / 256, 0.75, 64),
        "clustered_20k": (inputs.clustered(20000, 2, n_halos=40)[0], 1e-4, 0.6, 256),
        "duplicates_1k": (dup, 0.01, 0.7, 16),
        "lattice_216": (lattice, 0.05, 0.9, 8),
        "tiny_3": (np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 2.0, 0.5]]), 0.1, 0.5, 1),
    }


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
def test_hilbert_matches_oracle(gpu, name):
    pos, eps, theta, n_crit = CASES[name]
    mass = np.random.default_rng(1).uniform(0.5, 1.5, pos.shape[0]) / pos.shape[0]
    t = oracle.Tree(pos, mass, curve=1)
    c = gpu.Context(curve=1)
    c.build_tree(to_dev(pos), to_dev(mass))
    keys, perm = c.export_sorted()
    keys_o, perm_o = t.sorted()
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), keys_o)
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), perm_o)
    got, _, _ = gpu_nodes(c)
    expect = oracle_nonchain_nodes(t)
    assert set(got) == set(expect)
    bad = [k for k in got if got[k] != expect[k]]
    assert not bad, f"{len(bad)} nodes differ, e.g. {bad[0]}"
    G = c.make_groups(n_crit)
    assert t.groups(n_crit) == G
    acc, pot = c.compute_forces(eps, theta)
    st = c.get_stats()
    assert st.error_flags == 0
    ref = t.forces(eps, theta)
    _, _, ll, _ = c.export_groups(lists=True)
    assert np.array_equal(ll.cpu().numpy(), ref["list_len"])
    assert st.interactions == ref["interactions"]
    check_forces(acc.cpu().numpy().astype(np.float64), pot.cpu().numpy().astype(np.float64), ref)


def test_hilbert_order_differs_and_morton_is_default(gpu):
    pos = inputs.clustered(5000, 3, n_halos=8)[0]
    mass = np.full(5000, 1 / 5000)
    cm, ch = gpu.Context(), gpu.Context(curve=1)
    for c in (cm, ch):
        c.build_tree(to_dev(pos), to_dev(mass))
    km = cm.export_sorted()[0].cpu().numpy().view(np.uint64)
    kh = ch.export_sorted()[0].cpu().numpy().view(np.uint64)
    assert np.array_equal(km, oracle.Tree(pos, mass).sorted()[0])
    assert not np.array_equal(km, kh)
    with pytest.raises(gpu.BHError):
        cm.set_options(curve=2)


def test_hilbert_batch_equals_standalone(gpu):
    bh = gpu
    pos, mass, off, eps = inputs.batch_systems(seed=4, n_systems=5, n_min=2000, n_max=20000)
    theta = np.array([0.4, 0.6, 0.75, 1.0, 0.5])
    c = bh.Context(curve=1, split_visits=-1)
    dpos, dmass = to_dev(pos), to_dev(mass)
    c.build_batch(off, dpos, dmass)
    c.make_groups(64)
    a, p = c.compute_forces_batch(eps, theta)
    assert c.get_stats().error_flags == 0
    for k in range(len(off) - 1):
        lo, hi = int(off[k]), int(off[k + 1])
        s = bh.Context(curve=1, split_visits=-1)
        s.build_tree(dpos[lo:hi].contiguous(), dmass[lo:hi].contiguous())
        s.make_groups(64)
        sa, sp = s.compute_forces(float(eps[k]), float(theta[k]))
        assert torch.equal(sa, a[lo:hi]) and torch.equal(sp, p[lo:hi]), f"system {k}"


def test_hilbert_with_quadrupoles_and_neighbors(gpu):
    """The options compose: quadrupole sums in Peano-Hilbert order match the
    oracle's in that order, and the neighbour search gives the same counts
    and densities in either order."""
    pos, mass = inputs.clustered(15000, 12, n_halos=30)[:2]
    eps, theta, n_crit = 1e-3, 0.6, 64
    c = gpu.Context(curve=1, quadrupole=True)
    c.build_tree(to_dev(pos), to_dev(mass))
    G = c.make_groups(n_crit)
    acc, pot = c.compute_forces(eps, theta)
    assert c.get_stats().error_flags == 0
    t = oracle.Tree(pos, mass, curve=1)
    assert t.groups(n_crit) == G
    ref = t.forces(eps, theta, quadrupole=True)
    check_forces(acc.cpu().numpy().astype(np.float64), pot.cpu().numpy().astype(np.float64), ref)
    h = to_dev(np.full(pos.shape[0], 0.02))
    ch, rh = c.neighbors(h, count=True, rho=True)
    m = gpu.Context()
    m.build_tree(to_dev(pos), to_dev(mass))
    m.make_groups(n_crit)
    cm, rm = m.neighbors(h, count=True, rho=True)
    assert torch.equal(ch, cm)
    np.testing.assert_allclose(rh.cpu().numpy(), rm.cpu().numpy(), rtol=1e-12)


@pytest.mark.parametrize("n", [0, 1, 2, 65])
def test_options_small_and_empty_inputs(gpu, n):
    """Edge sizes with every option: Peano-Hilbert order with quadrupole sums
    against the oracle, and the neighbour search against brute force."""
    pos = np.random.default_rng(n + 3).normal(size=(n, 3))
    mass = np.full(n, 1.0)
    c = gpu.Context(curve=1, quadrupole=True)
    c.build_tree(to_dev(pos.reshape(n, 3)), to_dev(mass))
    G = c.make_groups(8)
    acc, pot = c.compute_forces(0.05, 0.6)
    h = np.full(n, 1.0)
    cnt, rho = c.neighbors(to_dev(h), count=True, rho=True)
    assert c.get_stats().error_flags == 0
    if n == 0:
        assert G == 0
        return
    t = oracle.Tree(pos, mass, curve=1)
    assert t.groups(8) == G
    ref = t.forces(0.05, 0.6, quadrupole=True)
    check_forces(acc.cpu().numpy().astype(np.float64), pot.cpu().numpy().astype(np.float64), ref)
    nref = oracle.neighbors(pos, mass, h)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), nref["count"])
    np.testing.assert_allclose(rho.cpu().numpy(), nref["rho"], rtol=1e-12)
