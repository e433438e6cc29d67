"""Pins of the oracle's quadrupole extension (second mass moments of each
cell and the second-order term of the softened potential of a cell entry).

The moments are pinned by identities that relate different nodes and by
positivity: every cell's moments equal the sum over its children of their
own moments plus the parallel-axis shift (the children's are computed from
their own particles independently), the tensor is symmetric positive
semi-definite with trace sum m |x - com|^2, and its dipole partner (the mass
weighted mean displacement) vanishes.

The force terms are pinned by their order of accuracy against direct
summation of Eq. (1) (itself pinned elsewhere): a cluster shrunk by a factor
h about a fixed centre of mass and seen as one cell by a distant particle
leaves a monopole error of order h^2 and a quadrupole error of order h^3,
with softening comparable to the distance (a dropped or mis-softened term,
a wrong sign or factor, leaves an h^2 error).  Without softening, the
residual also falls one power of the distance faster than the monopole's.
"""
import numpy as np
import pytest

import oracle
from oracle import KIND_PARTICLE
from paper_0909_0541_amd import inputs


def _moment_tensor(row):
    xx, yy, zz, xy, xz, yz = row
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


@pytest.mark.parametrize("seed", [1, 2])
def test_second_moments_parallel_axis(seed):
    pos, mass = inputs.clustered(3000, seed, n_halos=6)[:2]
    t = oracle.Tree(pos, mass)
    nd = t.nodes()
    S = t.second_moments()
    n = nd["mass"].shape[0]
    checked = 0
    for v in range(n):
        if nd["kind"][v] == KIND_PARTICLE:
            assert np.all(S[v] == 0.0)
            continue
        kids = [c for c in nd["children"][v] if c >= 0]
        if not kids:
            continue
        acc = np.zeros((3, 3))
        for c in kids:
            d = nd["com"][c] - nd["com"][v]
            acc += _moment_tensor(S[c]) + nd["mass"][c] * np.outer(d, d)
        ref = _moment_tensor(S[v])
        scale = max(np.trace(ref), 1e-300)
        assert np.max(np.abs(acc - ref)) <= 1e-12 * scale, v
        checked += 1
    assert checked > 100


def test_second_moments_invariants():
    pos, mass = inputs.plummer(2000, 5, with_vel=False)[:2]
    t = oracle.Tree(pos, mass)
    nd = t.nodes()
    S = t.second_moments()
    keys, perm = t.sorted()
    spos, smass = pos[perm], mass[perm]
    for v in np.flatnonzero(nd["kind"] != KIND_PARTICLE)[:400]:
        a, c = nd["first"][v], nd["count"][v]
        x, m = spos[a:a + c], smass[a:a + c]
        d = x - nd["com"][v]
        # dipole about the centre of mass vanishes; trace is the spread
        assert np.max(np.abs(m @ d)) <= 1e-12 * max(np.sum(m * np.abs(d).sum(1)), 1e-300)
        T = _moment_tensor(S[v])
        assert np.allclose(T, T.T)
        np.testing.assert_allclose(np.trace(T), np.sum(m * np.sum(d * d, axis=1)), rtol=1e-12, atol=1e-300)
        ev = np.linalg.eigvalsh(T)
        assert ev[0] >= -1e-12 * max(ev[-1], 1e-300)


def _probe_setup(h, r, seed=11, k=40):
    """A cluster of k bodies, displacements scaled by h about a fixed centre
    of mass c, and one light probe at distance r from c."""
    rng = np.random.default_rng(seed)
    m = rng.uniform(0.5, 1.5, k)
    y = rng.normal(0.0, 1.0, (k, 3)) * np.array([1.0, 0.6, 0.3])
    y -= (m @ y) / m.sum()
    c = np.array([0.1234, -0.0712, 0.0431])
    u = np.array([0.8, 0.36, 0.48])
    u /= np.linalg.norm(u)
    pos = np.concatenate([c + h * y, (c + r * u)[None]])
    mass = np.concatenate([m, [1e-6]])
    return pos, mass


def _probe_errors(h, r, eps):
    pos, mass = _probe_setup(h, r)
    n = pos.shape[0]
    t = oracle.Tree(pos, mass)
    assert t.groups(1) == n
    # the probe's group (one particle, the last in input order) must see the
    # whole cluster as a single cell entry
    _, perm = t.sorted()
    g = int(np.flatnonzero(perm == n - 1)[0])
    xyzm, part, _ = t.group_list(g, 1.0)
    cells = part < 0
    assert cells.sum() == 1 and np.isclose(xyzm[cells, 3].sum(), mass[:-1].sum(), rtol=1e-14)
    da, dp = oracle.direct(pos, mass, eps, idx=np.array([n - 1]))
    out = {}
    for quad in (False, True):
        f = t.forces(eps, 1.0, groups=np.array([g]), quadrupole=quad)
        out[quad] = (np.linalg.norm(f["acc"][n - 1] - da[0]), abs(f["pot"][n - 1] - dp[0]))
    return out


@pytest.mark.parametrize("eps", [0.0, 0.7])
def test_quadrupole_order_in_cluster_size(eps):
    r = 1.0
    hs = [0.02, 0.01, 0.005]
    errs = [_probe_errors(h, r, eps) for h in hs]
    for a, b in zip(errs, errs[1:]):
        for comp in (0, 1):
            mono = a[False][comp] / b[False][comp]
            quad = a[True][comp] / b[True][comp]
            assert 3.0 < mono < 5.0, (mono, comp)
            assert 6.0 < quad < 10.5, (quad, comp)
    for e in errs:
        for comp in (0, 1):
            assert e[True][comp] < 0.2 * e[False][comp]


def test_quadrupole_order_in_distance():
    h = 0.02
    rs = [0.5, 1.0, 2.0]
    errs = [_probe_errors(h, r, 0.0) for r in rs]
    for a, b in zip(errs, errs[1:]):
        # potential: monopole residual ~ r^-3, quadrupole residual ~ r^-4;
        # acceleration one power more
        mono_p, quad_p = a[False][1] / b[False][1], a[True][1] / b[True][1]
        mono_a, quad_a = a[False][0] / b[False][0], a[True][0] / b[True][0]
        assert 6.0 < mono_p < 10.0 and 12.0 < quad_p < 20.0, (mono_p, quad_p)
        assert 12.0 < mono_a < 20.0 and 24.0 < quad_a < 40.0, (mono_a, quad_a)


def test_quadrupole_two_body_closed_form():
    """Two equal bodies at com -/+ d e_z seen from x = com + r e_x: the exact
    softened potential is -2m / sqrt(r^2 + d^2 + eps^2); its expansion to
    second order in d is -2m/R + m d^2 / R^3 with R^2 = r^2 + eps^2, which the
    quadrupole entry must reproduce to O(d^4)."""
    m, d, r, eps = 0.7, 1e-3, 1.0, 0.4
    pos = np.array([[0.0, 0.0, -d], [0.0, 0.0, d], [r, 0.0, 0.0]])
    mass = np.array([m, m, 1e-9])
    t = oracle.Tree(pos, mass)
    t.groups(1)
    _, perm = t.sorted()
    g = int(np.flatnonzero(perm == 2)[0])
    xyzm, part, _ = t.group_list(g, 1.0)
    assert (part < 0).sum() == 1
    f = t.forces(eps, 1.0, groups=np.array([g]), quadrupole=True)
    R = np.sqrt(r * r + eps * eps)
    want = -2 * m / R + m * d * d / R ** 3
    assert abs(f["pot"][2] - want) <= 1e-10 * abs(want)
    # acceleration: -d/dr of the same expansion, pointing at the pair (-x)
    dpdr = 2 * m * r / R ** 3 - 3 * m * d * d * r / R ** 5
    np.testing.assert_allclose(f["acc"][2], [-dpdr, 0.0, 0.0], rtol=1e-10, atol=1e-14)
