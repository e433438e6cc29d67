"""Python wrapper of the FP64 oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It loads ``oracle/liboracle.so`` (built from
``bh_oracle.c`` by ``oracle/build.py``) with ctypes and exposes numpy-level
functions:

  direct(pos, mass, eps, idx=None)        -- Eq. (1) by direct summation
  Tree(pos, mass, curve=0)                -- oct-tree of Sec. 3.1 in Morton (0) or
                                             Peano-Hilbert (1) order
  hilbert_key(x, y, z)                    -- Peano-Hilbert index of a cell
  Tree.groups(n_crit)                     -- particle groups
  Tree.forces(eps, theta, theta_g=None, groups=None)
                                          -- grouped tree walk + Eq. (1) sums
  Tree.group_list(g, theta)               -- one group's interaction list
  Tree.second_moments()                   -- per-node second mass moments
  Tree.forces(..., quadrupole=True)       -- the same sums with quadrupole terms
  neighbors(pos, mass, h, lists=False)    -- brute-force neighbours and SPH density
  sph_kernel(r, h)                        -- the cubic spline kernel
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        i64, dbl, vp = C.c_int64, C.c_double, C.c_void_p
        L.oracle_direct.argtypes = [i64, vp, vp, dbl, i64, vp, vp, vp]
        L.oracle_direct.restype = C.c_int
        L.oracle_tree_build.argtypes = [i64, vp, vp]
        L.oracle_tree_build.restype = vp
        L.oracle_tree_build2.argtypes = [i64, vp, vp, C.c_int]
        L.oracle_tree_build2.restype = vp
        L.oracle_hilbert_key.argtypes = [i64, i64, i64]
        L.oracle_hilbert_key.restype = C.c_uint64
        L.oracle_tree_free.argtypes = [vp]
        L.oracle_tree_free.restype = None
        L.oracle_tree_groups.argtypes = [vp, C.c_int]
        L.oracle_tree_groups.restype = i64
        L.oracle_tree_forces.argtypes = [vp, dbl, dbl, vp, i64, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_tree_forces.restype = C.c_int
        L.oracle_tree_forces2.argtypes = [vp, dbl, dbl, vp, i64, vp, C.c_int, vp, vp, vp, vp, vp, vp]
        L.oracle_tree_forces2.restype = C.c_int
        L.oracle_tree_quadrupoles.argtypes = [vp]
        L.oracle_tree_quadrupoles.restype = None
        L.oracle_tree_node_quadrupole.argtypes = [vp, i64, vp]
        L.oracle_tree_node_quadrupole.restype = None
        L.oracle_tree_group_list.argtypes = [vp, i64, dbl, i64, vp, vp, vp]
        L.oracle_tree_group_list.restype = i64
        L.oracle_tree_info.argtypes = [vp, vp, vp, vp, vp]
        L.oracle_tree_info.restype = None
        L.oracle_tree_sorted.argtypes = [vp, vp, vp]
        L.oracle_tree_sorted.restype = None
        L.oracle_tree_nodes.argtypes = [vp, vp, vp, vp]
        L.oracle_tree_nodes.restype = None
        L.oracle_tree_group_info.argtypes = [vp, vp, vp, vp, vp]
        L.oracle_tree_group_info.restype = None
        L.oracle_sph_kernel.argtypes = [dbl, dbl]
        L.oracle_sph_kernel.restype = dbl
        L.oracle_neighbors.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_neighbors.restype = C.c_int
        L.oracle_neighbors_sel.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp]
        L.oracle_neighbors_sel.restype = C.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def direct(pos, mass, eps: float, idx=None):
    """FP64 direct summation of Eq. (1) for rows idx (all rows if None).
    Returns (acc [k,3], pot [k])."""
    pos = _f64(pos, (-1, 3))
    mass = _f64(mass)
    n = pos.shape[0]
    if idx is None:
        ns = n
        idxa = None
    else:
        idxa = np.ascontiguousarray(idx, dtype=np.int64)
        ns = idxa.shape[0]
    acc = np.zeros((ns, 3))
    pot = np.zeros(ns)
    rc = lib().oracle_direct(n, _p(pos), _p(mass), float(eps), ns, _p(idxa), _p(acc), _p(pot))
    if rc != 0:
        raise ValueError("oracle_direct failed")
    return acc, pot


KIND_CELL, KIND_PARTICLE, KIND_BUCKET = 0, 1, 2


class Tree:
    """The oracle's oct-tree over (pos, mass); see bh_oracle.c."""

    def __init__(self, pos, mass, curve: int = 0):
        """curve 0: Morton order; 1: Peano-Hilbert order."""
        self.pos = _f64(pos, (-1, 3))
        self.mass = _f64(mass)
        self.n = self.pos.shape[0]
        h = lib().oracle_tree_build2(self.n, _p(self.pos), _p(self.mass), int(curve))
        if not h:
            raise ValueError("oracle_tree_build rejected the input")
        self._h = h
        self.ngroups = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_tree_free(h)
            self._h = None

    def info(self):
        lo = np.zeros(3)
        side = C.c_double()
        nn = C.c_int64()
        root = C.c_int64()
        lib().oracle_tree_info(self._h, _p(lo), C.byref(side), C.byref(nn), C.byref(root))
        return {"lo": lo, "side": side.value, "nnodes": nn.value, "root": root.value}

    def sorted(self):
        keys = np.zeros(self.n, dtype=np.uint64)
        perm = np.zeros(self.n, dtype=np.int64)
        lib().oracle_tree_sorted(self._h, _p(keys), _p(perm))
        return keys, perm

    def nodes(self):
        """Node table: dict of arrays (level, kind, first, count, nchild,
        parent, mass, com [k,3], l, s, children [k,8])."""
        nn = self.info()["nnodes"]
        ints = np.zeros((nn, 6), dtype=np.int64)
        reals = np.zeros((nn, 6))
        ch = np.zeros((nn, 8), dtype=np.int64)
        lib().oracle_tree_nodes(self._h, _p(ints), _p(reals), _p(ch))
        return {"level": ints[:, 0], "kind": ints[:, 1], "first": ints[:, 2], "count": ints[:, 3],
                "nchild": ints[:, 4], "parent": ints[:, 5], "mass": reals[:, 0], "com": reals[:, 1:4],
                "l": reals[:, 4], "s": reals[:, 5], "children": ch}

    def groups(self, n_crit: int) -> int:
        g = lib().oracle_tree_groups(self._h, int(n_crit))
        if g < 0:
            raise ValueError("oracle_tree_groups failed")
        self.ngroups = int(g)
        return self.ngroups

    def group_info(self):
        G = self.ngroups
        first = np.zeros(G, dtype=np.int64)
        count = np.zeros(G, dtype=np.int64)
        lo = np.zeros((G, 3))
        hi = np.zeros((G, 3))
        lib().oracle_tree_group_info(self._h, _p(first), _p(count), _p(lo), _p(hi))
        return first, count, lo, hi

    def second_moments(self):
        """Second mass moments about each node's centre of mass, [nnodes, 6]
        in the order xx, yy, zz, xy, xz, yz (zero for particles)."""
        lib().oracle_tree_quadrupoles(self._h)
        nn = self.info()["nnodes"]
        out = np.zeros((nn, 6))
        row = np.zeros(6)
        for k in range(nn):
            lib().oracle_tree_node_quadrupole(self._h, k, _p(row))
            out[k] = row
        return out

    def forces(self, eps: float, theta: float, theta_g=None, groups=None, lists_only: bool = False,
               quadrupole: bool = False):
        """Grouped tree forces.  Returns dict with acc [n,3], pot [n] and
        acc_abs [n] (sum of term magnitudes), all in input order with NaN rows
        for particles outside the selected groups, plus list_len, list_mass
        (per selected group) and interactions.  lists_only skips the sums;
        quadrupole adds the second-order terms of cell entries."""
        if self.ngroups is None:
            raise RuntimeError("call groups(n_crit) first")
        tg = None if theta_g is None else _f64(theta_g)
        if tg is not None and tg.shape[0] != self.ngroups:
            raise ValueError("theta_g must have one value per group")
        gs = None if groups is None else np.ascontiguousarray(groups, dtype=np.int64)
        nsel = self.ngroups if gs is None else gs.shape[0]
        acc = pot = aab = None
        if not lists_only:
            acc = np.full((self.n, 3), np.nan)
            pot = np.full(self.n, np.nan)
            aab = np.full(self.n, np.nan)
        ll = np.zeros(nsel, dtype=np.int64)
        lm = np.zeros(nsel)
        inter = C.c_int64()
        rc = lib().oracle_tree_forces2(self._h, float(eps), float(theta), _p(tg), nsel, _p(gs), int(quadrupole),
                                       _p(acc), _p(pot), _p(aab), _p(ll), _p(lm), C.byref(inter))
        if rc != 0:
            raise ValueError("oracle_tree_forces failed")
        return {"acc": acc, "pot": pot, "acc_abs": aab, "list_len": ll, "list_mass": lm,
                "interactions": inter.value}

    def group_list(self, g: int, theta: float):
        """Interaction list of group g: (xyzm [L,4], particle [L], node [L])
        with the Morton index of particle entries (-1 for cells) and the id of
        the node each entry comes from."""
        L = lib().oracle_tree_group_list(self._h, int(g), float(theta), 0, None, None, None)
        if L < 0:
            raise ValueError("bad group")
        xyzm = np.zeros((L, 4))
        part = np.zeros(L, dtype=np.int64)
        node = np.zeros(L, dtype=np.int64)
        lib().oracle_tree_group_list(self._h, int(g), float(theta), L, _p(xyzm), _p(part), _p(node))
        return xyzm, part, node


def hilbert_key(x: int, y: int, z: int) -> int:
    """Peano-Hilbert index of integer cell coordinates (21 bits per axis)."""
    return int(lib().oracle_hilbert_key(int(x), int(y), int(z)))


def sph_kernel(r: float, h: float) -> float:
    """The cubic spline kernel W(r, h) with compact support h."""
    return lib().oracle_sph_kernel(float(r), float(h))


def neighbors(pos, mass, h, lists: bool = False):
    """Brute-force neighbours within each particle's own radius h_i (j != i,
    |x_j - x_i| < h_i): dict with count [n] (int64), rho [n] (SPH density,
    when mass is given) and, with lists, a list of index arrays (increasing)."""
    pos = _f64(pos).reshape(-1, 3)
    n = pos.shape[0]
    h = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (n,)))
    m = None if mass is None else _f64(mass)
    count = np.zeros(n, dtype=np.int64)
    rho = None if m is None else np.zeros(n)
    if lib().oracle_neighbors(n, _p(pos), _p(m), _p(h), _p(count), _p(rho), None, None) != 0:
        raise ValueError("oracle_neighbors failed")
    out = {"count": count, "rho": rho}
    if lists:
        off = np.zeros(n + 1, dtype=np.int64)
        off[1:] = np.cumsum(count)
        nbr = np.zeros(max(int(off[-1]), 1), dtype=np.int64)
        if lib().oracle_neighbors(n, _p(pos), None, _p(h), None, None, _p(off), _p(nbr)) != 0:
            raise ValueError("oracle_neighbors failed")
        out["lists"] = [nbr[off[i]:off[i + 1]] for i in range(n)]
        out["offsets"] = off
        out["flat"] = nbr[:off[-1]]
    return out


def neighbors_sampled(pos, mass, h, sel):
    """Brute-force neighbour counts and SPH density of the particles sel only
    (each against all n): dict with count [k] and rho [k] (or None)."""
    pos = _f64(pos).reshape(-1, 3)
    n = pos.shape[0]
    h = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (n,)))
    m = None if mass is None else _f64(mass)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    count = np.zeros(sel.shape[0], dtype=np.int64)
    rho = None if m is None else np.zeros(sel.shape[0])
    if lib().oracle_neighbors_sel(n, _p(pos), _p(m), _p(h), sel.shape[0], _p(sel), _p(count), _p(rho)) != 0:
        raise ValueError("oracle_neighbors_sel failed")
    return {"count": count, "rho": rho}


def tree_forces(pos, mass, eps: float, theta: float, n_crit: int, theta_g=None):
    """Convenience: build, group and evaluate in one call."""
    t = Tree(pos, mass)
    t.groups(n_crit)
    out = t.forces(eps, theta, theta_g)
    out["tree"] = t
    return out
