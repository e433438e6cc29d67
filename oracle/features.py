"""FP64 reference of the 12 per-group features of the opening-angle network
(test infrastructure only).

For a group of c particles (a Morton range with bounding box [lo, hi], centre
c_g = (lo + hi)/2, half-diagonal R = |hi - lo|/2, mass m_g and centre of mass
x_g) and softening eps, with A_1 the smallest tree cell (not a bucket of equal
keys) that holds more than c particles and contains the group, and A_{k+1}
the next cell above A_k with at least two sub-cells (A_{k+1} = A_k at the
root):

  f0      = log2 c
  f1      = log2(1 + R / eps)
  f2      = |x_g - c_g| / (R + eps)
  f3      = log2(l(A_1) / (R + eps))
  f4..f7  = log2(m(A_k) / m_g),          k = 1..4
  f8..f11 = |com(A_k) - c_g| / l(A_k),   k = 1..4

with l the cell side and com its centre of mass (Sec. 3.1).  A group that is
a whole system has no A_1; then f3..f11 are 0.  The features describe how
the group sits in the mass around it (how big, how dense, how lopsided the
enclosing cells are), which is what decides how much error a given theta
makes for it (Eq. 2/3).
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
        anc = []
        for _ in range(4):
            anc.append(a)
            b = parent[a]
            while b >= 0 and kind[b] == KIND_CELL and nchild[b] == 1:
                b = parent[b]
            if b >= 0:
                a = b
        out[g, 3] = np.log2(nd["l"][anc[0]] / (R + eps))
        for k, a in enumerate(anc):
            out[g, 4 + k] = np.log2(nd["mass"][a] / mg)
            dc = nd["com"][a] - cen
            out[g, 8 + k] = np.sqrt(dc @ dc) / nd["l"][a]
    return out
