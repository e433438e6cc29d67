"""Pins of the oracle's Peano-Hilbert ordering.

The index is checked against the defining properties of a Hilbert curve, not
against a copy of itself: it is a bijection from the cells of a grid onto
consecutive integers, consecutive indices are face-adjacent cells (Morton
order jumps), the curve starts at the origin cell, and every aligned cube of
any level is one contiguous index range (so the octal digits of the index
name the octree's cells).  The oracle's tree over Hilbert keys holds the same
cells as over Morton keys (the cells are geometric), and with one-particle
groups the same interaction lists, so forces agree to rounding.
"""
import numpy as np
import pytest

import oracle
from paper_0909_0541_amd import inputs

B = 21


def _grid_keys(bits, shift):
    n = 1 << bits
    out = {}
    for x in range(n):
        for y in range(n):
            for z in range(n):
                k = oracle.hilbert_key(x << shift, y << shift, z << shift) >> (3 * shift)
                out[k] = (x, y, z)
    return out


@pytest.mark.parametrize("bits,shift", [(3, B - 3), (4, 0), (2, 7)])
def test_bijection_and_adjacency(bits, shift):
    keys = _grid_keys(bits, shift)
    n3 = 1 << (3 * bits)
    assert sorted(keys) == list(range(n3))
    assert keys[0] == (0, 0, 0)
    steps = [np.abs(np.subtract(keys[i + 1], keys[i])).sum() for i in range(n3 - 1)]
    assert all(s == 1 for s in steps)


def test_morton_is_not_adjacent():
    # the same check fails for bit interleaving, so it has teeth
    def morton(x, y, z):
        k = 0
        for b in range(2, -1, -1):
            k = (k << 3) | (((x >> b) & 1) << 2) | (((y >> b) & 1) << 1) | ((z >> b) & 1)
        return k
    keys = {morton(x, y, z): (x, y, z) for x in range(8) for y in range(8) for z in range(8)}
    steps = [np.abs(np.subtract(keys[i + 1], keys[i])).sum() for i in range(511)]
    assert max(steps) > 1


def test_aligned_cubes_are_contiguous_ranges():
    rng = np.random.default_rng(3)
    for level in (1, 2, 5, 11, 20):
        side = 1 << (B - level)
        for _ in range(6):
            corner = rng.integers(0, 1 << level, 3) * side
            pts = corner + rng.integers(0, side, (40, 3))
            pre = {oracle.hilbert_key(*p) >> (3 * (B - level)) for p in pts}
            assert len(pre) == 1
            # a cell of the neighbouring cube along some axis has another prefix
            ax = rng.integers(0, 3)
            q = corner.copy()
            q[ax] = (q[ax] + side) % (1 << B)
            assert oracle.hilbert_key(*q) >> (3 * (B - level)) not in pre


def _cells(t):
    nd = t.nodes()
    _, perm = t.sorted()
    out = set()
    for k in range(nd["kind"].shape[0]):
        a, c = int(nd["first"][k]), int(nd["count"][k])
        out.add((int(nd["level"][k]), frozenset(perm[a:a + c].tolist())))
    return out


def test_same_cells_and_lists_as_morton():
    pos, mass = inputs.clustered(4000, 6, n_halos=10)[:2]
    tm, th = oracle.Tree(pos, mass, curve=0), oracle.Tree(pos, mass, curve=1)
    assert _cells(tm) == _cells(th)
    keys_h, perm_h = th.sorted()
    assert np.all(np.diff(keys_h.astype(np.uint64)) >= 0)
    assert tm.groups(1) == th.groups(1) == pos.shape[0]
    fm, fh = tm.forces(1e-3, 0.6), th.forces(1e-3, 0.6)
    assert fm["interactions"] == fh["interactions"]
    np.testing.assert_allclose(fh["acc"], fm["acc"], rtol=1e-11, atol=1e-11 * np.abs(fm["acc"]).max())
    np.testing.assert_allclose(fh["pot"], fm["pot"], rtol=1e-12)
    # with larger groups both orders give valid trees and every group is a
    # contiguous range of its own order
    G = th.groups(64)
    first, count, lo, hi = th.group_info()
    assert count.sum() == pos.shape[0] and np.all(first[1:] == (first + count)[:-1])
