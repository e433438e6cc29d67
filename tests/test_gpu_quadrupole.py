"""Quadrupole option of the group path against the FP64 oracle.

The option keeps the lists of the monopole path (same opening test) and adds
to every cell entry the second-order term of the softened potential of its
particles.  Checks: the second moments of every cell match the oracle's
(computed there from each cell's own particles, here bottom-up by parallel
axes) to FP64 rounding; list lengths are exact and forces meet the parity bar
against the oracle's quadrupole sums, on single systems with and without
split walks, near-heavy large groups, and a batch; the quadrupole sums are
closer to direct summation than the monopole sums at the same theta; a batch
equals its systems run alone bit for bit; and the option's state errors.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import check_forces, to_dev
from paper_0909_0541_amd import inputs

pytestmark = pytest.mark.gpu


def _moment_cases():
    rng = np.random.default_rng(5)
    dup = np.concatenate([np.tile([[0.1, 0.2, 0.3]], (300, 1)), rng.uniform(-1, 1, (700, 3))])
    lattice = np.stack(np.meshgrid(*[np.arange(6.0)] * 3, indexing="ij"), -1).reshape(-1, 3)
    return {
        "plummer_8k": inputs.plummer(8192, 1, with_vel=False)[0],
        "clustered_20k": inputs.clustered(20000, 2, n_halos=40)[0],
        "duplicates_1k": dup,
        "lattice_216": lattice,
    }


MOMENT_CASES = _moment_cases()


@pytest.mark.parametrize("name", list(MOMENT_CASES))
def test_moments_match_oracle(gpu, name):
    pos = MOMENT_CASES[name]
    mass = np.random.default_rng(1).uniform(0.5, 1.5, pos.shape[0]) / pos.shape[0]
    c = gpu.Context(quadrupole=True)
    c.build_tree(to_dev(pos), to_dev(mass))
    ints, reals = c.export_nodes()
    mom = c.export_moments().cpu().numpy()
    ints, reals = ints.cpu().numpy(), reals.cpu().numpy()
    t = oracle.Tree(pos, mass)
    side = t.info()["side"]
    nd = t.nodes()
    S = t.second_moments()
    ref = {}
    for k in np.flatnonzero(nd["kind"] != oracle.KIND_PARTICLE):
        ref[(int(nd["first"][k]), int(nd["count"][k]))] = S[k]
    checked = 0
    for k in range(ints.shape[0]):
        kind, first, count = int(ints[k, 1]), int(ints[k, 2]), int(ints[k, 3])
        if kind in (1, 3):
            assert np.all(mom[k] == 0.0)
            continue
        want = ref[(first, count)]
        # FP64 rounding relative to the moments themselves, or to the cell's
        # mass times its size squared where the moments vanish (coincident
        # particles: both sides then hold rounding noise of the positions)
        l = reals[k, 4] if np.isfinite(reals[k, 4]) else side * 2.0 ** -21
        scale = max(want[0] + want[1] + want[2], reals[k, 0] * l * l, 1e-300)
        assert np.max(np.abs(mom[k] - want)) <= 1e-12 * scale, (k, mom[k], want)
        checked += 1
    assert checked == c.get_stats().n_cells


def _force_cases():
    p8, m8, _ = inputs.plummer(8192, 1, with_vel=False)
    pc, mc = inputs.clustered(20000, 9, n_halos=40)[:2]
    pb, mb = inputs.clustered(30000, 4, n_halos=20)[:2]
    return {
        "plummer_8k": (p8, m8, 1 / 256, 0.75, 64, None),
        "clustered_20k": (pc, mc, 1e-4, 0.6, 64, None),
        "clustered_20k_split": (pc, mc, 1e-4, 0.6, 64, 64),
        "large_groups_30k": (pb, mb, 1e-3, 0.8, 256, None),
        "small_groups_30k": (pb, mb, 1e-3, 0.5, 4, None),
    }


FORCE_CASES = _force_cases()


@pytest.mark.parametrize("name", list(FORCE_CASES))
def test_quadrupole_forces_match_oracle(gpu, name):
    pos, mass, eps, theta, n_crit, cap = FORCE_CASES[name]
    c = gpu.Context(quadrupole=True, split_visits=cap)
    c.build_tree(to_dev(pos), to_dev(mass))
    G = c.make_groups(n_crit)
    acc, pot = c.compute_forces(eps, theta)
    st = c.get_stats()
    assert st.error_flags == 0
    if cap is not None:
        assert st.n_split_groups > 0
    t = oracle.Tree(pos, mass)
    assert t.groups(n_crit) == G
    ref = t.forces(eps, theta, quadrupole=True)
    _, _, ll, _ = c.export_groups(lists=True)
    assert np.array_equal(ll.cpu().numpy(), ref["list_len"])
    assert st.interactions == ref["interactions"]
    info = check_forces(acc.cpu().numpy().astype(np.float64), pot.cpu().numpy().astype(np.float64), ref)
    print(name, info, flush=True)


def test_quadrupole_closer_to_direct(gpu):
    """Same lists, one more order of the expansion: the truncation error
    falls by a factor that shrinks with theta (about theta^3 against
    theta^2)."""
    pos, mass = inputs.plummer(20000, 3, with_vel=False)[:2]
    eps, n_crit = 1 / 256, 64
    idx = np.random.default_rng(2).choice(pos.shape[0], 2000, replace=False)
    da, dp = oracle.direct(pos, mass, eps, idx)
    ratio = {}
    for theta in (0.8, 0.5):
        err = {}
        for quad in (False, True):
            c = gpu.Context(quadrupole=quad)
            c.build_tree(to_dev(pos), to_dev(mass))
            c.make_groups(n_crit)
            a, p = c.compute_forces(eps, theta)
            a = a.cpu().numpy().astype(np.float64)[idx]
            rel = np.linalg.norm(a - da, axis=1) / np.linalg.norm(da, axis=1)
            err[quad] = float(np.sqrt(np.mean(rel ** 2)))
        ratio[theta] = err[True] / err[False]
        print("theta", theta, "rms relative force error: monopole", err[False], "quadrupole", err[True], flush=True)
    assert ratio[0.8] < 0.6
    assert ratio[0.5] < ratio[0.8]


def test_quadrupole_batch_equals_standalone(gpu):
    bh = gpu
    pos, mass, off, eps = inputs.batch_systems(seed=9, n_systems=5, n_min=2000, n_max=20000)
    theta = np.array([0.4, 0.6, 0.75, 1.0, 0.5])
    c = bh.Context(quadrupole=True, split_visits=-1)
    dpos, dmass = to_dev(pos), to_dev(mass)
    c.build_batch(off, dpos, dmass)
    c.make_groups(64)
    a, p = c.compute_forces_batch(eps, theta)
    assert c.get_stats().error_flags == 0
    for k in range(len(off) - 1):
        lo, hi = int(off[k]), int(off[k + 1])
        s = bh.Context(quadrupole=True, split_visits=-1)
        s.build_tree(dpos[lo:hi].contiguous(), dmass[lo:hi].contiguous())
        s.make_groups(64)
        sa, sp = s.compute_forces(float(eps[k]), float(theta[k]))
        assert torch.equal(sa, a[lo:hi]) and torch.equal(sp, p[lo:hi]), f"system {k}"


def test_quadrupole_option_errors(gpu):
    bh = gpu
    pos, mass, _ = inputs.plummer(3000, 6, with_vel=False)
    c = bh.Context()
    c.build_tree(to_dev(pos), to_dev(mass))
    c.make_groups(32)
    with pytest.raises(bh.BHError) as e:
        c.export_moments()
    assert e.value.status == -4
    c.set_options(quadrupole=True)
    with pytest.raises(bh.BHError) as e:  # tree built without moments
        c.compute_forces(0.01, 0.6)
    assert e.value.status == -4
    c.build_tree(to_dev(pos), to_dev(mass))
    c.make_groups(32)
    a, p = c.compute_forces(0.01, 0.6)
    with pytest.raises(bh.BHError) as e:  # the per-particle walk is monopole only
        c.compute_forces_particle(0.01, 0.6)
    assert e.value.status == -1
    # back to monopoles on the same tree: the plain sums again, bit for bit
    c.set_options(quadrupole=False)
    a0, p0 = c.compute_forces(0.01, 0.6)
    m = bh.Context()
    m.build_tree(to_dev(pos), to_dev(mass))
    m.make_groups(32)
    a1, p1 = m.compute_forces(0.01, 0.6)
    assert torch.equal(a0, a1) and torch.equal(p0, p1)
    assert not torch.equal(a, a1)
