"""Pins of the oracle's oct-tree, groups, walk and tree sum.

Each check ties the oracle to something other than itself: an independent
brute-force construction of the tree (Sec. 3.1, by geometric cell membership
in exact rational arithmetic, no keys and no sorting), an independent
per-particle recursive walk written from Fig. "treewalk" with Eq. (2) as
printed, direct summation (theta -> 0 reduces the tree to Eq. (1)), and
invariants such as mass conservation of every interaction list.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import KIND_BUCKET, KIND_CELL, KIND_PARTICLE
from paper_0909_0541_amd import inputs


def _small_inputs():
    rng = np.random.default_rng(42)
    a = rng.uniform(-1, 1, (24, 3))
    b = np.concatenate([rng.normal(0, 0.01, (10, 3)), rng.uniform(-1, 1, (6, 3)),
                        np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])])  # one exact duplicate
    c = np.concatenate([rng.normal(0, 1e-5, (6, 3)) + 0.3, rng.uniform(0, 1, (10, 3))])
    return [a, b, c]


def _brute_force_nodes(pos, lo, side):
    """Node set of Sec. 3.1 by brute force: at level l a particle lies in cell
    floor((x - lo) 2^l / side) (exact rationals); a cell at level l exists if it
    is non-empty and its parent cell holds at least two particles; cells stop
    at one particle or at level 21.  Returns {(level, frozenset(members))}."""
    n = pos.shape[0]
    lo_f = [Fraction(float(v)) for v in lo]
    side_f = Fraction(float(side))
    exact = [[Fraction(float(pos[i, k])) for k in range(3)] for i in range(n)]
    nodes = set()
    frontier = {(): list(range(n))}  # key: path of cells, value: members
    nodes.add((0, frozenset(range(n))))
    level = 0
    cur = [list(range(n))] if n >= 2 else []
    while cur and level < 21:
        level += 1
        nxt = []
        for members in cur:
            cells = {}
            for i in members:
                c = tuple(int(((exact[i][k] - lo_f[k]) * (2 ** level) / side_f).__floor__()) for k in range(3))
                cells.setdefault(c, []).append(i)
            for c, mem in cells.items():
                nodes.add((level, frozenset(mem)))
                if len(mem) >= 2:
                    nxt.append(mem)
        cur = nxt
    del frontier
    return nodes


@pytest.mark.parametrize("case", range(3))
def test_tree_matches_brute_force(case):
    pos = _small_inputs()[case]
    mass = np.linspace(0.5, 1.5, pos.shape[0])
    t = oracle.Tree(pos, mass)
    info = t.info()
    lo, side = info["lo"], info["side"]
    # the root cube encloses every particle
    assert np.all(pos >= lo) and np.all(pos < lo + side)
    keys, perm = t.sorted()
    nd = t.nodes()
    got = set()
    for k in range(info["nnodes"]):
        members = frozenset(perm[nd["first"][k]:nd["first"][k] + nd["count"][k]].tolist())
        got.add((int(nd["level"][k]), members))
    assert got == _brute_force_nodes(pos, lo, side)


def test_tree_invariants_and_moments():
    pos, mass, _ = inputs.clustered(5000, 9, n_halos=20)
    mass = mass * np.random.default_rng(1).uniform(0.5, 1.5, mass.shape[0])
    t = oracle.Tree(pos, mass)
    info = t.info()
    keys, perm = t.sorted()
    assert np.all(np.diff(keys.astype(object)) >= 0)
    assert np.array_equal(np.sort(perm), np.arange(pos.shape[0]))
    nd = t.nodes()
    root = info["root"]
    assert nd["count"][root] == pos.shape[0]
    # root mass and centre of mass against numpy sums
    assert nd["mass"][root] == pytest.approx(mass.sum(), rel=1e-14)
    np.testing.assert_allclose(nd["com"][root], (mass[:, None] * pos).sum(0) / mass.sum(), rtol=1e-13, atol=1e-15)
    leaf_cover = np.zeros(pos.shape[0], dtype=int)
    for k in range(info["nnodes"]):
        lv, kind, first, count = nd["level"][k], nd["kind"][k], nd["first"][k], nd["count"][k]
        assert 0 <= lv <= 21
        if kind == KIND_PARTICLE:
            assert count == 1
            leaf_cover[first] += 1
            continue
        if kind == KIND_BUCKET:
            assert lv == 21 and count >= 2
            assert np.all(keys[first:first + count] == keys[first])
            leaf_cover[first:first + count] += 1
            continue
        ch = nd["children"][k][: nd["nchild"][k]]
        assert 1 <= len(ch) <= 8
        assert nd["count"][ch].sum() == count
        assert np.all(nd["level"][ch] == lv + 1)
        assert np.all(nd["parent"][ch] == k)
        # children are consecutive ranges in octant (Morton) order
        assert nd["first"][ch[0]] == first
        assert np.all(nd["first"][ch[1:]] == nd["first"][ch[:-1]] + nd["count"][ch[:-1]])
        assert nd["mass"][k] == pytest.approx(nd["mass"][ch].sum(), rel=1e-14)
        # centre of mass from the member particles
        idx = perm[first:first + count]
        com = (mass[idx, None] * pos[idx]).sum(0) / mass[idx].sum()
        np.testing.assert_allclose(nd["com"][k], com, rtol=1e-12, atol=1e-14 * info["side"])
        # the cell side halves per level and s is bounded by the half diagonal
        assert nd["l"][k] == info["side"] / 2.0 ** lv
        assert 0.0 <= nd["s"][k] <= 0.5 * np.sqrt(3.0) * nd["l"][k] * (1 + 1e-12)
    assert np.all(leaf_cover == 1)


def test_zero_and_one_particle():
    t = oracle.Tree(np.zeros((0, 3)), np.zeros(0))
    assert t.groups(8) == 0
    t = oracle.Tree(np.array([[1.0, 2.0, 3.0]]), np.array([2.0]))
    assert t.groups(8) == 1
    out = t.forces(0.1, 0.5)
    assert np.all(out["acc"] == 0.0) and np.all(out["pot"] == 0.0)
    assert out["interactions"] == 0


def test_coincident_particles_form_a_bucket():
    pos = np.tile([[0.25, -0.5, 1.0]], (40, 1))
    pos = np.concatenate([pos, [[3.0, 3.0, 3.0]]])
    mass = np.ones(41)
    t = oracle.Tree(pos, mass)
    nd = t.nodes()
    assert (nd["kind"] == KIND_BUCKET).sum() == 1
    b = np.flatnonzero(nd["kind"] == KIND_BUCKET)[0]
    assert nd["count"][b] == 40 and np.isinf(nd["l"][b])
    t.groups(16)
    f, c, _, _ = t.group_info()
    # the bucket's 40 particles are packed into groups of 16, 16, 8
    assert sorted(c.tolist()) == sorted([16, 16, 8, 1])
    eps = 0.05
    out = t.forces(eps, 0.8)
    a_dir, p_dir = oracle.direct(pos, mass, eps)
    np.testing.assert_allclose(out["acc"], a_dir, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out["pot"], p_dir, rtol=1e-12)


@pytest.mark.parametrize("n_crit", [1, 7, 64, 256])
def test_groups_partition_and_structure(n_crit):
    pos, mass, _ = inputs.clustered(6000, 3, n_halos=30)
    t = oracle.Tree(pos, mass)
    G = t.groups(n_crit)
    first, count, lo, hi = t.group_info()
    assert G == len(first)
    assert first[0] == 0 and np.all(first[1:] == first[:-1] + count[:-1]) and first[-1] + count[-1] == 6000
    assert np.all((count >= 1) & (count <= n_crit))
    keys, perm = t.sorted()
    spos = pos[perm]
    for g in range(G):
        p = spos[first[g]:first[g] + count[g]]
        assert np.array_equal(lo[g], p.min(0)) and np.array_equal(hi[g], p.max(0))
    # every group is a union of consecutive children of one node holding more
    # than n_crit particles, and a group cannot absorb the next sibling run
    nd = t.nodes()
    big = np.flatnonzero(nd["count"] > n_crit)
    bounds = {}
    for k in big:
        if nd["kind"][k] == KIND_BUCKET:
            edges = list(range(nd["first"][k], nd["first"][k] + nd["count"][k] + 1))
            sizes = [1] * nd["count"][k]
        else:
            ch = nd["children"][k][: nd["nchild"][k]]
            edges = [nd["first"][c] for c in ch] + [nd["first"][k] + nd["count"][k]]
            sizes = [nd["count"][c] for c in ch]
        for e, s in zip(edges[:-1], sizes):
            bounds[e] = (k, s)
    for g in range(G):
        assert first[g] in bounds, "group must start at a child boundary"
        parent, _ = bounds[first[g]]
        assert nd["count"][parent] > n_crit
        end = first[g] + count[g]
        if g + 1 < G and end in bounds and bounds[end][0] == parent:
            nxt_size = bounds[end][1]
            if nxt_size <= n_crit:
                assert count[g] + nxt_size > n_crit, "greedy packing would have absorbed the next child"


def _per_particle_walk(nd, root, x, theta):
    """Fig. "treewalk" for one particle with Eq. (2) as printed: a cell is far
    enough if l/theta + s < d, d the distance from the particle to the cell's
    centre of mass.  Returns the sorted list of node ids that interact."""
    out = []

    def rec(k):
        if nd["kind"][k] == KIND_PARTICLE:
            out.append(k)
            return
        if nd["kind"][k] == KIND_BUCKET:
            out.append(k)
            return
        d = np.sqrt(((nd["com"][k] - x) ** 2).sum())
        if nd["l"][k] / theta + nd["s"][k] < d:
            out.append(k)
            return
        for c in nd["children"][k][: nd["nchild"][k]]:
            rec(c)

    rec(root)
    return sorted(out)


@pytest.mark.parametrize("theta", [0.3, 0.6, 1.0])
def test_single_particle_groups_equal_paper_walk(theta):
    # with n_crit = 1 every group is one particle and the group criterion is
    # the paper's per-particle criterion, so the lists must be identical
    pos, mass, _ = inputs.plummer(600, 21, with_vel=False)
    t = oracle.Tree(pos, mass)
    assert t.groups(1) == 600
    nd = t.nodes()
    root = t.info()["root"]
    keys, perm = t.sorted()
    for g in range(0, 600, 37):
        _, part, node = t.group_list(g, theta)
        expect = _per_particle_walk(nd, root, pos[perm[g]], theta)
        assert sorted(set(node.tolist())) == expect


@pytest.mark.parametrize("theta", [0.2, 0.5, 0.75, 1.0])
def test_lists_conserve_mass_and_contain_members(theta):
    pos, mass, _ = inputs.clustered(8000, 4, n_halos=40)
    t = oracle.Tree(pos, mass)
    t.groups(64)
    first, count, lo, hi = t.group_info()
    out = t.forces(1e-3, theta)
    assert np.allclose(out["list_mass"], mass.sum(), rtol=1e-13)
    nd = t.nodes()
    rng = np.random.default_rng(0)
    keys, perm = t.sorted()
    spos = pos[perm]
    for g in rng.choice(t.ngroups, 25, replace=False):
        xyzm, part, node = t.group_list(g, theta)
        assert xyzm.shape[0] == out["list_len"][g]
        # each member's own particle entry appears exactly once
        own = part[(part >= first[g]) & (part < first[g] + count[g])]
        assert np.array_equal(np.sort(own), np.arange(first[g], first[g] + count[g]))
        # conservativeness: every accepted cell is far enough for every member
        # under Eq. (2) as printed (distance from the particle to the com)
        cells = node[part < 0]
        mem = spos[first[g]:first[g] + count[g]]
        for k in cells:
            d = np.sqrt(((mem - nd["com"][k]) ** 2).sum(1))
            assert np.all(nd["l"][k] / theta + nd["s"][k] < d)


def test_theta_zero_is_direct_summation():
    for pos, mass, eps in [(inputs.plummer(1500, 8, with_vel=False)[0], None, 0.01),
                           (inputs.clustered(1500, 8, n_halos=5)[0], None, 1e-4),
                           (inputs.uniform_cube(1000, 8)[0], None, 0.05)]:
        mass = np.random.default_rng(3).uniform(0.2, 2.0, pos.shape[0])
        t = oracle.Tree(pos, mass)
        t.groups(32)
        out = t.forces(eps, 0.0)
        assert np.all(out["list_len"] == pos.shape[0])
        assert out["interactions"] == pos.shape[0] * (pos.shape[0] - 1)
        a, p = oracle.direct(pos, mass, eps)
        scale = np.abs(a).max()
        np.testing.assert_allclose(out["acc"], a, rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(out["pot"], p, rtol=1e-12)


def test_error_shrinks_with_theta():
    # smaller theta opens more cells: more interactions and a smaller error
    pos, mass, _ = inputs.plummer(4000, 17, with_vel=False)
    eps = 0.01
    a, _ = oracle.direct(pos, mass, eps)
    t = oracle.Tree(pos, mass)
    t.groups(32)
    rms, inter = [], []
    for th in [1.0, 0.7, 0.5, 0.3]:
        out = t.forces(eps, th)
        e = np.linalg.norm(out["acc"] - a, axis=1) / np.linalg.norm(a, axis=1)
        rms.append(np.sqrt((e * e).mean()))
        inter.append(out["interactions"])
    assert all(x > y for x, y in zip(rms, rms[1:])), rms
    assert all(x < y for x, y in zip(inter, inter[1:])), inter
    assert rms[0] < 0.05


def test_group_and_per_particle_walks_agree_on_force_for_tight_theta():
    # two valid readings of the same method (group vs per-particle lists) give
    # forces that agree to the accuracy of the method at small theta
    pos, mass, _ = inputs.uniform_sphere(3000, 6)
    t1 = oracle.Tree(pos, mass)
    t1.groups(1)
    t64 = oracle.Tree(pos, mass)
    t64.groups(64)
    o1 = t1.forces(0.01, 0.25)
    o64 = t64.forces(0.01, 0.25)
    a, _ = oracle.direct(pos, mass, 0.01)
    e1 = np.linalg.norm(o1["acc"] - a, axis=1) / np.linalg.norm(a, axis=1)
    e64 = np.linalg.norm(o64["acc"] - a, axis=1) / np.linalg.norm(a, axis=1)
    assert np.sqrt((e64 ** 2).mean()) <= np.sqrt((e1 ** 2).mean()) * 1.05
    assert o64["interactions"] > o1["interactions"]


def test_invalid_inputs_rejected():
    with pytest.raises(ValueError):
        oracle.Tree(np.array([[0.0, np.nan, 0.0]]), np.ones(1))
    with pytest.raises(ValueError):
        oracle.Tree(np.zeros((2, 3)), np.array([1.0, -1.0]))
