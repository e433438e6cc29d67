"""FP64 reference of the 12 per-group features of the opening-angle network
(test infrastructure only).

For a group of c particles (a Morton range with bounding box [lo, hi], centre
c_g = (lo + hi)/2, half-diagonal R = |hi - lo|/2, mass m_g and centre of mass
x_g) and softening eps, with A_1 the smallest tree cell (not a bucket of equal
keys) that holds more than c particles and contains the group, and A_2 the
next cell above A_1 with at least two sub-cells (A_2 = A_1 at the root):

  f0  = log2 c
  f1  = log2(1 + R / eps)
  f2  = |x_g - c_g| / (R + eps)
  f3  = log2(l(A_1) / (R + eps))
  f4  = log2(m(A_1) / m_g)
  f5  = |com(A_1) - c_g| / l(A_1)
  f11 = log2(m(A_2) / m_g)

with l the cell side and com its centre of mass (Sec. 3.1); a group that is
a whole system has f3, f4, f5, f11 = 0.  The rest come from the group's
interaction list at theta = 1 (Eq. 2/3, the probe list), with d = com - c_g
for every entry whose centre of mass lies outside the box:

  f6  = log2(|sum m d / (|d|^2 + eps^2)^(3/2)| + 2^-100)   (probe field)
  f7  = log2(sum m / (|d|^2 + eps^2) + 2^-100)             (its scale)
  f8  = log2(1 + number of single-particle entries outside the box)
  f9  = log2(list length)
  f10 = log2(mass of the entries inside the box / m_g)

The features describe the group's size and density, how lopsided the mass
around it is, and how strongly the surrounding pull cancels at the group,
which decides how much relative error a given theta makes for it.
"""
from __future__ import annotations

import numpy as np

from . import KIND_BUCKET, KIND_CELL, KIND_PARTICLE


def group_features(tree, eps: float) -> np.ndarray:
    """[G, 12] FP64 features of the groups of an oracle Tree (groups() called)."""
    nd = tree.nodes()
    first, count, lo, hi = tree.group_info()
    keys, perm = tree.sorted()
    spos = tree.pos[perm]
    smass = tree.mass[perm]
    kind, parent, ncount, nchild = nd["kind"], nd["parent"], nd["count"], nd["nchild"]
    leaf_of = np.full(tree.n, -1, dtype=np.int64)
    pk = np.flatnonzero(kind == KIND_PARTICLE)
    leaf_of[nd["first"][pk]] = pk
    G = first.shape[0]
    out = np.zeros((G, 12))
    for g in range(G):
        f, c = int(first[g]), int(count[g])
        cen = (lo[g] + hi[g]) / 2.0
        e = hi[g] - lo[g]
        R = np.sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) / 2.0
        m = smass[f:f + c]
        mg = 0.0
        mx = np.zeros(3)
        for i in range(c):
            mg += m[i]
            mx += m[i] * spos[f + i]
        xg = mx / mg
        d = xg - cen
        out[g, 0] = np.log2(c)
        out[g, 1] = np.log2(1.0 + R / eps)
        out[g, 2] = np.sqrt(d @ d) / (R + eps)
        # A_1: smallest proper cell above the group holding more than c particles
        a = parent[leaf_of[f]]
        while a >= 0 and (kind[a] == KIND_BUCKET or ncount[a] <= c):
            a = parent[a]
        if a < 0:
            continue
        anc = [a]
        b = parent[a]
        while b >= 0 and kind[b] == KIND_CELL and nchild[b] == 1:
            b = parent[b]
        anc.append(b if b >= 0 else a)
        out[g, 3] = np.log2(nd["l"][anc[0]] / (R + eps))
        out[g, 4] = np.log2(nd["mass"][anc[0]] / mg)
        dc = nd["com"][anc[0]] - cen
        out[g, 5] = np.sqrt(dc @ dc) / nd["l"][anc[0]]
        out[g, 11] = np.log2(nd["mass"][anc[1]] / mg)
    return out


PROBE_THETA = 1.0
TINY = 2.0 ** -100


def probe_features(tree, eps: float) -> np.ndarray:
    """[G, 5] features f6..f10 from each group's theta = 1 interaction list."""
    first, count, lo, hi = tree.group_info()
    keys, perm = tree.sorted()
    smass = tree.mass[perm]
    eps2 = eps * eps
    G = first.shape[0]
    out = np.zeros((G, 5))
    for g in range(G):
        xyzm, part, _ = tree.group_list(g, PROBE_THETA)
        cen = (lo[g] + hi[g]) / 2.0
        mg = 0.0
        for i in range(int(first[g]), int(first[g] + count[g])):
            mg += smass[i]
        a = np.zeros(3)
        S = 0.0
        n_part = 0
        m_in = 0.0
        for k in range(xyzm.shape[0]):
            com, m = xyzm[k, :3], xyzm[k, 3]
            below = lo[g] - com
            above = com - hi[g]
            ek = np.maximum(0.0, np.maximum(below, above))
            if ek[0] * ek[0] + ek[1] * ek[1] + ek[2] * ek[2] == 0.0:
                m_in += m
                continue
            d = com - cen
            r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2
            a += m * d / (r2 * np.sqrt(r2))
            S += m / r2
            n_part += int(part[k] >= 0)
        out[g, 0] = np.log2(np.sqrt(a @ a) + TINY)
        out[g, 1] = np.log2(S + TINY)
        out[g, 2] = np.log2(1.0 + n_part)
        out[g, 3] = np.log2(xyzm.shape[0])
        out[g, 4] = np.log2(m_in / mg)
    return out


def all_features(tree, eps: float) -> np.ndarray:
    """The 12 features of every group, in the network's input order."""
    f = group_features(tree, eps)
    f[:, 6:11] = probe_features(tree, eps)
    return f

