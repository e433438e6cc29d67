"""Pins of the oracle's per-group features on configurations whose tree is known by hand."""
import numpy as np

import oracle
from oracle.features import group_features


def _cluster(c, rng, k=4, r=1e-3):
    return np.asarray(c, dtype=np.float64) + rng.uniform(-r, r, (k, 3))


def _expected(members, all_pos, all_mass, idx, anc, side, eps):
    """Features from the definition, with the ancestor cells given by hand
    as (particle index set, side)."""
    p = all_pos[idx]
    m = all_mass[idx]
    lo, hi = p.min(axis=0), p.max(axis=0)
    cen = (lo + hi) / 2
    R = np.linalg.norm(hi - lo) / 2
    mg = m.sum()
    xg = (m[:, None] * p).sum(axis=0) / mg
    f = [np.log2(len(idx)), np.log2(1 + R / eps), np.linalg.norm(xg - cen) / (R + eps),
         np.log2(anc[0][1] / (R + eps))]
    for s, _ in anc:
        f.append(np.log2(all_mass[s].sum() / mg))
    for s, l in anc:
        com = (all_mass[s][:, None] * all_pos[s]).sum(axis=0) / all_mass[s].sum()
        f.append(np.linalg.norm(com - cen) / l)
    return np.array(f)


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
        exp = _expected(None, pos, mass, np.sort(idx), [(allidx, side)] * 4, side, eps)
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
        anc = [(sup, side / 8), (np.arange(16), side), (np.arange(16), side), (np.arange(16), side)]
        exp = _expected(None, pos, mass, idx, anc, side, eps)
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
