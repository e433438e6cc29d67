"""FP64 time integration on top of the oracle's tree forces (test infrastructure only).

The paper integrates its cosmological run in time with the tree forces
(Sec. 4) without naming the scheme; the reading taken here is the
kick-drift-kick leapfrog, all in FP64:

    v <- v + dt/2 a(x);  x <- x + dt v;  rebuild the tree;  v <- v + dt/2 a(x)

and the energy E = sum m v^2 / 2 + sum m pot / 2 with the tree potential.
Only the tests may use this module.
"""
from __future__ import annotations

import numpy as np

from . import Tree, direct


def forces(pos, mass, eps: float, theta: float, n_crit: int):
    """Grouped tree forces (theta > 0) or direct summation (theta == 0) in FP64."""
    if theta == 0.0:
        return direct(pos, mass, eps)
    t = Tree(pos, mass)
    t.groups(n_crit)
    out = t.forces(eps, theta)
    return out["acc"], out["pot"]


def leapfrog(pos, vel, mass, eps: float, theta: float, n_crit: int, dt: float, steps: int, acc=None):
    """steps kick-drift-kick steps; returns (pos, vel, acc, pot) at the end.
    acc: the accelerations at pos (computed when None)."""
    x = np.array(pos, dtype=np.float64, copy=True)
    v = np.array(vel, dtype=np.float64, copy=True)
    m = np.asarray(mass, dtype=np.float64)
    if acc is None:
        a, p = forces(x, m, eps, theta, n_crit)
    else:
        a, p = np.asarray(acc, dtype=np.float64), None
    h = 0.5 * dt
    for _ in range(steps):
        v = v + h * a
        x = x + dt * v
        a, p = forces(x, m, eps, theta, n_crit)
        v = v + h * a
    return x, v, a, p


def energy(vel, mass, pot):
    """(kinetic, potential) = (sum m |v|^2 / 2, sum m pot / 2)."""
    v = np.asarray(vel, dtype=np.float64)
    m = np.asarray(mass, dtype=np.float64)
    return 0.5 * float(np.sum(m * np.sum(v * v, axis=1))), 0.5 * float(np.sum(m * np.asarray(pot, np.float64)))
