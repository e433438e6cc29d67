"""Pins of the oracle's per-group features on configurations whose tree is known by hand."""
import numpy as np

import oracle
from oracle.features import TINY, all_features, group_features, probe_features


def _cluster(c, rng, k=4, r=1e-3):
    return np.asarray(c, dtype=np.float64) + rng.uniform(-r, r, (k, 3))


def _expected(all_pos, all_mass, idx, anc, eps):
    """f0..f5 and f11 from the definition, with the ancestor cells A_1, A_2
    given by hand as (particle index set, side); the probe features f6..f10
    are not part of group_features and stay 0."""
    p = all_pos[idx]
    m = all_mass[idx]
    lo, hi = p.min(axis=0), p.max(axis=0)
    cen = (lo + hi) / 2
    R = np.linalg.norm(hi - lo) / 2
    mg = m.sum()
    xg = (m[:, None] * p).sum(axis=0) / mg
    (s1, l1), (s2, _) = anc
    com1 = (all_mass[s1][:, None] * all_pos[s1]).sum(axis=0) / all_mass[s1].sum()
    f = np.zeros(12)
    f[:6] = [np.log2(len(idx)), np.log2(1 + R / eps), np.linalg.norm(xg - cen) / (R + eps), np.log2(l1 / (R + eps)),
             np.log2(all_mass[s1].sum() / mg), np.linalg.norm(com1 - cen) / l1]
    f[11] = np.log2(all_mass[s2].sum() / mg)
    return f


def test_two_clusters_root_is_every_ancestor():
    rng = np.random.default_rng(1)
    pos = np.concatenate([_cluster([0.0, 0.0, 0.0], rng), _cluster([1.0, 1.0, 1.0], rng)])
    mass = rng.uniform(0.5, 1.5, 8)
    t = oracle.Tree(pos, mass)
    assert t.groups(4) == 2
    info = t.info()
    side = info["side"]
    ext = (pos.max(axis=0) - pos.min(axis=0)).max()
    assert side == ext * (1 + 2.0 ** -20)
    eps = 1e-3
    f = group_features(t, eps)
    first, count, _, _ = t.group_info()
    _, perm = t.sorted()
    allidx = np.arange(8)
    for g in range(2):
        idx = perm[first[g]:first[g] + count[g]]
        exp = _expected(pos, mass, np.sort(idx), [(allidx, side)] * 2, eps)
        assert np.allclose(f[g], exp, rtol=1e-12, atol=1e-12), (g, f[g], exp)


def test_nested_clusters_skip_single_child_cells():
    rng = np.random.default_rng(2)
    # two superclusters, each of two clusters 0.1 apart along x
    a0 = _cluster([0.02, 0.02, 0.02], rng)
    a1 = _cluster([0.095, 0.02, 0.02], rng)
    b0 = _cluster([0.98, 0.98, 0.98], rng)
    b1 = _cluster([0.905, 0.98, 0.98], rng)
    pos = np.concatenate([a0, a1, b0, b1])
    mass = rng.uniform(0.5, 1.5, 16)
    t = oracle.Tree(pos, mass)
    assert t.groups(4) == 4
    side = t.info()["side"]
    eps = 1e-4
    f = group_features(t, eps)
    first, count, _, _ = t.group_info()
    _, perm = t.sorted()
    sets = {0: np.arange(0, 8), 1: np.arange(0, 8), 2: np.arange(8, 16), 3: np.arange(8, 16)}
    seen = set()
    for g in range(4):
        idx = np.sort(perm[first[g]:first[g] + count[g]])
        k = int(idx[0]) // 4  # which cluster
        seen.add(k)
        sup = sets[k]
        # the supercluster's split cell: the level-3 cube (side/8) holding both
        # of its clusters; above it only single-child cells up to the root
        anc = [(sup, side / 8), (np.arange(16), side)]
        exp = _expected(pos, mass, idx, anc, eps)
        assert np.allclose(f[g], exp, rtol=1e-12, atol=1e-12), (g, f[g], exp)
    assert seen == {0, 1, 2, 3}


def test_whole_system_group_has_no_ancestor():
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 1, (10, 3))
    mass = np.ones(10)
    t = oracle.Tree(pos, mass)
    assert t.groups(64) == 1
    f = group_features(t, 0.01)
    assert f[0, 0] == np.log2(10)
    assert np.all(f[0, 3:] == 0.0)
    pf = probe_features(t, 0.01)
    # a whole system is one member node: no field, one entry, inside mass = m_g
    assert pf[0, 0] == np.log2(TINY) and pf[0, 1] == np.log2(TINY)
    assert pf[0, 2] == 0.0 and pf[0, 3] == 0.0 and pf[0, 4] == 0.0


def test_coincident_group_uses_the_cell_above_the_bucket():
    pos = np.concatenate([np.zeros((6, 3)), np.ones((2, 3))])
    mass = np.ones(8)
    t = oracle.Tree(pos, mass)
    t.groups(4)
    f = group_features(t, 0.1)
    first, count, _, _ = t.group_info()
    for g in range(len(first)):
        assert np.isfinite(f[g]).all()
        # every group's first ancestor is the root (the buckets are skipped)
        assert np.isclose(f[g, 4], np.log2(8.0 / count[g]))


def test_probe_features_of_two_distant_clusters():
    """At theta = 1 each cluster sees the other as one cell, and its own
    cluster is one member node: two entries."""
    rng = np.random.default_rng(4)
    pos = np.concatenate([_cluster([0.0, 0.0, 0.0], rng), _cluster([1.0, 1.0, 1.0], rng)])
    mass = rng.uniform(0.5, 1.5, 8)
    t = oracle.Tree(pos, mass)
    assert t.groups(4) == 2
    eps = 1e-2
    f = all_features(t, eps)
    first, count, lo, hi = t.group_info()
    _, perm = t.sorted()
    for g in range(2):
        own = np.sort(perm[first[g]:first[g] + count[g]])
        other = np.setdiff1d(np.arange(8), own)
        cen = (pos[own].min(axis=0) + pos[own].max(axis=0)) / 2
        mo = mass[other].sum()
        d = (mass[other][:, None] * pos[other]).sum(axis=0) / mo - cen
        r2 = d @ d + eps * eps
        a = mo * np.linalg.norm(d) / r2 ** 1.5
        exp = [np.log2(a + TINY), np.log2(mo / r2 + TINY), 0.0, 1.0, 0.0]
        assert np.allclose(f[g, 6:11], exp, rtol=1e-12, atol=1e-12), (g, f[g, 6:11], exp)
