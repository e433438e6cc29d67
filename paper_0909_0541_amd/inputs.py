"""Seeded synthetic particle sets (positions, masses, velocities) for every workload.

This module only draws random numbers; it holds none of the force method's
arithmetic, so the GPU path, the FP64 oracle and the tests can all take their
inputs from it without sharing any of the method.

The paper measures on random particles in a sphere (Sec. 3.5), a random cube
(Sec. 5) and a cosmological box from COSMICS initial conditions (Sec. 4).  The
initial conditions are not available, so a clustered box stands in for them:
a uniform background plus many truncated Plummer halos.  All particles have
equal mass 1/N (total mass 1, G = 1).

Workloads (sizes as used by the tests and the benchmark):
  * ``plummer``   -- Plummer sphere, a = 1, isotropic, speeds below escape
                     (Aarseth-Henon-Wielen rejection sampling).
  * ``clustered`` -- 30% uniform in the unit sphere, 70% in Plummer halos with
                     log-uniform masses 1e-4..1e-2 (renormalised to 0.7),
                     scale radius 0.002*(M/1e-4)^(1/2), centres uniform within
                     r <= 0.8, each halo truncated at 10 scale radii.
  * ``batch``     -- 64 systems with N log-uniform in [1024, 262144]; even
                     systems are Plummer spheres, odd systems clustered boxes
                     with max(1, N/4096) halos.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "plummer", "clustered", "uniform_sphere", "uniform_cube", "batch_systems",
    "Workload", "WORKLOADS", "make_workload",
]


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniformly distributed on the sphere, shape [n, 3]."""
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def _plummer_radii(rng: np.random.Generator, n: int, b: float, xmax: float = 1.0) -> np.ndarray:
    """Radii of a Plummer sphere of scale b by inverting the cumulative mass
    M(<r)/M = r^3 / (r^2 + b^2)^(3/2); xmax < 1 truncates the profile."""
    x = rng.uniform(0.0, xmax, n)
    x = np.maximum(x, 1e-300)
    return b / np.sqrt(np.power(x, -2.0 / 3.0) - 1.0)


def _plummer_speeds(rng: np.random.Generator, r: np.ndarray, b: float, mass: float) -> np.ndarray:
    """Isotropic speeds from the Plummer distribution function by rejection on
    g(q) = q^2 (1 - q^2)^(7/2), q = v / v_esc < 1 (G = 1)."""
    n = r.shape[0]
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x1 = rng.uniform(0.0, 1.0, todo.size)
        x2 = rng.uniform(0.0, 0.1, todo.size)
        ok = x2 < x1 * x1 * np.power(1.0 - x1 * x1, 3.5)
        q[todo[ok]] = x1[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0 * mass) * np.power(r * r + b * b, -0.25)
    return q * vesc


def plummer(n: int, seed: int, a: float = 1.0, with_vel: bool = True):
    """Plummer sphere with total mass 1 and scale a; returns (pos, mass, vel).

    Positions and velocities are recentred on the centre of mass.  The
    profile is not truncated, so the ensemble-mean potential energy is the
    closed form -(1 - 1/N) 3 pi / (32 a) (pairs i != j only)."""
    rng = np.random.default_rng(seed)
    r = _plummer_radii(rng, n, a)
    pos = r[:, None] * _isotropic(rng, n)
    mass = np.full(n, 1.0 / n)
    vel = None
    if with_vel:
        v = _plummer_speeds(rng, r, a, 1.0)
        vel = v[:, None] * _isotropic(rng, n)
        vel -= vel.mean(axis=0)
    pos -= pos.mean(axis=0)
    return np.ascontiguousarray(pos), mass, (None if vel is None else np.ascontiguousarray(vel))


def uniform_sphere(n: int, seed: int, radius: float = 1.0):
    """Random particles in a sphere (the paper's basic test distribution)."""
    rng = np.random.default_rng(seed)
    r = radius * np.cbrt(rng.uniform(0.0, 1.0, n))
    pos = r[:, None] * _isotropic(rng, n)
    return np.ascontiguousarray(pos), np.full(n, 1.0 / n), None


def uniform_cube(n: int, seed: int, side: float = 1.0):
    """Random particles in a cube (the paper's comparison distribution)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, side, (n, 3))
    return np.ascontiguousarray(pos), np.full(n, 1.0 / n), None


def _largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    """Integer counts proportional to weights that sum exactly to total."""
    w = weights / weights.sum() * total
    base = np.floor(w).astype(np.int64)
    rem = total - int(base.sum())
    if rem > 0:
        order = np.argsort(-(w - base), kind="stable")
        base[order[:rem]] += 1
    return base


def clustered(n: int, seed: int, n_halos: int = 512, with_vel: bool = False,
              bg_frac: float = 0.3, r_centres: float = 0.8):
    """Cosmology-like clustered box in the unit sphere; returns (pos, mass, vel).

    30% of the particles are uniform in the unit sphere, 70% sit in n_halos
    Plummer halos (log-uniform masses in [1e-4, 1e-2] renormalised to 0.7,
    scale b = 0.002 (M/1e-4)^(1/2) from the drawn mass, truncated at 10 b).
    With with_vel, halo members get Plummer velocities of their halo (mass =
    halo particle count / n, G = 1) and the background is at rest."""
    rng = np.random.default_rng(seed)
    n_bg = int(round(bg_frac * n))
    n_h = n - n_bg
    m_draw = np.power(10.0, rng.uniform(-4.0, -2.0, n_halos))
    b = 0.002 * np.sqrt(m_draw / 1e-4)
    counts = _largest_remainder(m_draw, n_h)
    rc = r_centres * np.cbrt(rng.uniform(0.0, 1.0, n_halos))
    centres = rc[:, None] * _isotropic(rng, n_halos)
    # truncation at 10 b: enclosed mass fraction 10^3 / (10^2 + 1)^(3/2)
    xmax = 1000.0 / math.pow(101.0, 1.5)

    pos = np.empty((n, 3))
    vel = np.zeros((n, 3)) if with_vel else None
    rb = np.cbrt(rng.uniform(0.0, 1.0, n_bg))
    pos[:n_bg] = rb[:, None] * _isotropic(rng, n_bg)
    off = n_bg
    for h in range(n_halos):
        c = int(counts[h])
        if c == 0:
            continue
        r = _plummer_radii(rng, c, float(b[h]), xmax)
        pos[off:off + c] = centres[h] + r[:, None] * _isotropic(rng, c)
        if with_vel:
            mh = c / n
            v = _plummer_speeds(rng, r, float(b[h]), mh)
            vel[off:off + c] = v[:, None] * _isotropic(rng, c)
        off += c
    mass = np.full(n, 1.0 / n)
    return np.ascontiguousarray(pos), mass, vel


def batch_systems(seed: int = 3, n_systems: int = 64, n_min: int = 1024, n_max: int = 262144):
    """64 independent systems of uneven size; returns (pos, mass, offsets, eps).

    N_k = round(exp(U(ln n_min, ln n_max))) with the given seed; system k is
    drawn with seed 1000 + k: a Plummer sphere for even k, a clustered box
    with max(1, N_k // 4096) halos for odd k.  Softening eps_k = N_k^(-1/3)/20.
    Particles of system k occupy rows offsets[k]:offsets[k+1]."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_systems))).astype(np.int64)
    offsets = np.zeros(n_systems + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    pos = np.empty((int(offsets[-1]), 3))
    mass = np.empty(int(offsets[-1]))
    for k in range(n_systems):
        nk = int(sizes[k])
        if k % 2 == 0:
            p, m, _ = plummer(nk, 1000 + k, with_vel=False)
        else:
            p, m, _ = clustered(nk, 1000 + k, n_halos=max(1, nk // 4096))
        pos[offsets[k]:offsets[k + 1]] = p
        mass[offsets[k]:offsets[k + 1]] = m
    eps = np.power(sizes.astype(np.float64), -1.0 / 3.0) / 20.0
    return pos, mass, offsets, eps


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    seed: int
    eps: float
    theta: float
    n_crit: int
    kind: str
    n_halos: int = 0
    description: str = ""


WORKLOADS = {
    "plummer_8k": Workload("plummer_8k", 8192, 1, 1.0 / 256.0, 0.75, 64, "plummer",
                           description="Plummer sphere N=8192, a=1, eps=1/256, theta=0.75, n_crit=64"),
    "clustered_2m": Workload("clustered_2m", 2097152, 2, 1e-4, 0.6, 256, "clustered", 512,
                             description="clustered box N=2,097,152, 512 halos, eps=1e-4, theta=0.6, n_crit=256"),
    "clustered_4m": Workload("clustered_4m", 4194304, 4, 1e-4, 0.6, 256, "clustered", 2048,
                             description="clustered box N=4,194,304, 2048 halos, eps=1e-4"),
    "clustered_8m": Workload("clustered_8m", 8388608, 5, 1e-4, 0.6, 256, "clustered", 2048,
                             description="clustered box N=8,388,608, 2048 halos, eps=1e-4, with velocities"),
}


def make_workload(name: str, n: int | None = None, with_vel: bool = False):
    """Build (pos, mass, vel, workload) for a named workload; n overrides the size."""
    w = WORKLOADS[name]
    nn = w.n if n is None else n
    if w.kind == "plummer":
        pos, mass, vel = plummer(nn, w.seed, with_vel=with_vel)
    else:
        halos = w.n_halos if n is None else max(1, int(round(w.n_halos * nn / w.n)))
        pos, mass, vel = clustered(nn, w.seed, n_halos=halos, with_vel=with_vel)
    return pos, mass, vel, w
