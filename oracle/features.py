"""FP64 reference of the 12 per-group features of the opening-angle network
(test infrastructure only).

For a group of c particles (a Morton range with bounding box [lo, hi], centre
c_g = (lo + hi)/2, half-diagonal R = |hi - lo|/2, mass m_g and centre of mass
x_g) and softening eps, with A_1 the smallest tree cell with at least two
sub-cells (not a bucket of equal keys) that holds more than c particles and
contains the group, and A_2 the next such cell above A_1 (A_2 = A_1 at the
root):

  f0  = log2 c
  f1  = log2(1 + R / eps)
  f2  = |x_g - c_g| / (R + eps)
  f3  = log2(l(A_1) / (R + eps))
  f4  = log2(m(A_1) / m_g)
  f5  = |com(A_1) - c_g| / l(A_1)
  f11 = log2(m(A_2) / m_g)

with l the cell side and com its centre of mass (Sec. 3.1); a group that is
a whole system has f3, f4, f5, f11 = 0.  The rest come from the group's
probe list (the group's walk at theta = 1, Eq. 2/3, where nodes made only of
members and cells smaller than R are taken whole), with d = com - c_g for
every entry whose centre of mass lies outside the box:

  f6  = log2(|sum m d / (|d|^2 + eps^2)^(3/2)| + 2^-100)   (probe field)
  f7  = log2(sum m / (|d|^2 + eps^2) + 2^-100)             (its scale)
  f8  = log2(1 + number of single-particle entries outside the box)
  f9  = log2(number of entries)
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
    # the smallest node above each particle: its leaf's parent, or its bucket
    # (members of a bucket of equal keys are not separate nodes)
    above = np.full(tree.n, -1, dtype=np.int64)
    pk = np.flatnonzero(kind == KIND_PARTICLE)
    above[nd["first"][pk]] = parent[pk]
    for b in np.flatnonzero(kind == KIND_BUCKET):
        above[nd["first"][b]:nd["first"][b] + ncount[b]] = b
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
        # A_1: smallest split cell above the group holding more than c particles
        a = above[f]
        while a >= 0 and (kind[a] == KIND_BUCKET or ncount[a] <= c or nchild[a] == 1):
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
    """[G, 5] features f6..f10 from each group's probe list.

    The probe list is the walk of Fig. "treewalk" for the group at theta = 1
    with two shortcuts: a node holding only members of the group is one entry
    that counts as inside, and a cell smaller than R (the box half-diagonal) is
    one entry without the opening test; otherwise particles are entries, a
    cell is an entry when d^2 > (l + s)^2 (d the distance from its centre of
    mass to the box) and is opened when not."""
    nd = tree.nodes()
    root = tree.info()["root"]
    first, count, lo, hi = tree.group_info()
    keys, perm = tree.sorted()
    spos = tree.pos[perm]
    smass = tree.mass[perm]
    kind, nfirst, ncount = nd["kind"], nd["first"], nd["count"]
    l, s, com, mass, children = nd["l"], nd["s"], nd["com"], nd["mass"], nd["children"]
    eps2 = eps * eps
    G = first.shape[0]
    out = np.zeros((G, 5))
    for g in range(G):
        f, c = int(first[g]), int(count[g])
        glo, ghi = lo[g], hi[g]
        cen = (glo + ghi) / 2.0
        e = ghi - glo
        lmin = np.sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) / 2.0
        mg = 0.0
        for i in range(f, f + c):
            mg += smass[i]
        a = np.zeros(3)
        S = 0.0
        n_part = 0
        n_entries = 0
        m_in = 0.0
        stack = [root]
        pend = []
        while stack:
            v = stack.pop()
            ek = np.maximum(0.0, np.maximum(glo - com[v], com[v] - ghi))
            d2 = ek[0] * ek[0] + ek[1] * ek[1] + ek[2] * ek[2]
            member = nfirst[v] >= f and nfirst[v] + ncount[v] <= f + c
            if member or kind[v] == KIND_PARTICLE or (kind[v] == KIND_CELL and l[v] < lmin):
                take = True
            elif kind[v] == KIND_BUCKET:
                take = False
            else:
                q = l[v] + s[v]
                take = d2 > q * q
            if not take:
                if kind[v] == KIND_BUCKET:
                    # a bucket's members are particle entries (Morton order)
                    for i in range(int(nfirst[v]), int(nfirst[v] + ncount[v])):
                        pend.append((spos[i], smass[i], f <= i < f + c, True))
                else:
                    stack.extend(int(k) for k in children[v] if k >= 0)
            else:
                pend.append((com[v], mass[v], member, kind[v] == KIND_PARTICLE))
            while pend:
                x, m, mem, is_part = pend.pop()
                ek = np.maximum(0.0, np.maximum(glo - x, x - ghi))
                n_entries += 1
                if mem or ek[0] * ek[0] + ek[1] * ek[1] + ek[2] * ek[2] == 0.0:
                    m_in += m
                    continue
                d = x - cen
                r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2
                a += m * d / (r2 * np.sqrt(r2))
                S += m / r2
                n_part += int(is_part)
        out[g, 0] = np.log2(np.sqrt(a @ a) + TINY)
        out[g, 1] = np.log2(S + TINY)
        out[g, 2] = np.log2(1.0 + n_part)
        out[g, 3] = np.log2(n_entries)
        out[g, 4] = np.log2(m_in / mg)
    return out


def all_features(tree, eps: float) -> np.ndarray:
    """The 12 features of every group, in the network's input order."""
    f = group_features(tree, eps)
    f[:, 6:11] = probe_features(tree, eps)
    return f

