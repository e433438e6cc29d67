"""Pins of the oracle's neighbour search and SPH density (the general
treewalk applied to a short-range interaction).

Neighbour sets are checked against scipy's k-d tree ball query (a library
routine, no shared code), symmetry under a common radius, and exact integer
counts on a lattice (enumerated here from the lattice vectors).  The cubic
spline kernel is pinned by its normalisation (the integral over its support
is 1) and continuity; the density of a uniform unit lattice is 1 to within
the kernel's discretisation error.
"""
import numpy as np
import pytest
from scipy import integrate
from scipy.spatial import cKDTree

import oracle
from paper_0909_0541_amd import inputs


def test_neighbors_match_kdtree():
    pos, mass = inputs.clustered(5000, 3, n_halos=8)[:2]
    rng = np.random.default_rng(7)
    h = 0.02 * rng.uniform(0.5, 2.0, pos.shape[0])
    out = oracle.neighbors(pos, mass, h, lists=True)
    tree = cKDTree(pos)
    for i in range(pos.shape[0]):
        got = tree.query_ball_point(pos[i], h[i], return_sorted=True)
        got = [j for j in got if j != i]
        d = np.linalg.norm(pos[got] - pos[i], axis=1) if got else np.zeros(0)
        # the ball query is closed (<=), the definition strict (<): no ties here
        assert not np.any(np.abs(d - h[i]) <= 1e-9 * h[i])
        assert np.array_equal(out["lists"][i], np.asarray(got, dtype=np.int64)), i
        assert out["count"][i] == len(got)
    assert out["count"].sum() > 20 * pos.shape[0]


def test_neighbors_symmetric_for_common_radius():
    pos = inputs.plummer(3000, 2, with_vel=False)[0]
    out = oracle.neighbors(pos, None, 0.3, lists=True)
    pairs = {(i, int(j)) for i in range(pos.shape[0]) for j in out["lists"][i]}
    assert pairs and all((j, i) in pairs for i, j in pairs)
    assert out["rho"] is None


def _lattice(k):
    g = np.arange(float(k))
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)


@pytest.mark.parametrize("h", [2.0, 2.5, 3.0])
def test_lattice_counts_and_density(h):
    pos = _lattice(12)
    out = oracle.neighbors(pos, np.ones(pos.shape[0]), h)
    r = int(np.ceil(h))
    v = np.arange(-r, r + 1)
    vec = np.stack(np.meshgrid(v, v, v, indexing="ij"), -1).reshape(-1, 3)
    n2 = (vec ** 2).sum(1)
    want = int(np.count_nonzero((n2 > 0) & (n2 < h * h)))
    inner = np.all((pos >= r) & (pos <= 11 - r), axis=1)
    assert np.all(out["count"][inner] == want)
    np.testing.assert_allclose(out["rho"][inner], 1.0, rtol=5e-3)


def test_kernel_normalisation_and_continuity():
    for hh in (0.3, 1.0, 2.5):
        val, _ = integrate.quad(lambda r: 4 * np.pi * r * r * oracle.sph_kernel(r, hh), 0, hh, points=[hh / 2])
        assert abs(val - 1.0) < 1e-10
        for q in (0.5, 1.0):
            lo, hi = oracle.sph_kernel(q * hh * (1 - 1e-12), hh), oracle.sph_kernel(q * hh * (1 + 1e-12), hh)
            assert abs(lo - hi) <= 1e-9 * oracle.sph_kernel(0.0, hh)
        assert oracle.sph_kernel(1.01 * hh, hh) == 0.0


def test_two_particles():
    m = np.array([2.0, 3.0])
    for d, hh, n in ((0.3, 0.5, 1), (0.6, 0.5, 0)):
        pos = np.array([[0.1, 0.2, 0.3], [0.1 + d, 0.2, 0.3]])
        out = oracle.neighbors(pos, m, hh)
        assert list(out["count"]) == [n, n]
        w0, wd = oracle.sph_kernel(0.0, hh), oracle.sph_kernel(d, hh)
        np.testing.assert_allclose(out["rho"], [m[0] * w0 + n * m[1] * wd, m[1] * w0 + n * m[0] * wd], rtol=1e-14)


def test_sampled_equals_full():
    pos, mass = inputs.clustered(3000, 5, n_halos=6)[:2]
    h = 0.03 * np.random.default_rng(1).uniform(0.5, 1.5, 3000)
    full = oracle.neighbors(pos, mass, h)
    sel = np.array([0, 17, 1234, 2999])
    part = oracle.neighbors_sampled(pos, mass, h, sel)
    assert np.array_equal(part["count"], full["count"][sel])
    assert np.array_equal(part["rho"], full["rho"][sel])
