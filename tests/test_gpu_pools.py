"""List pools that are too small: the walk reports it, the pools grow and the
walk runs again, and the result is the one a context with large enough
pools computes.

A context first used on a small system sizes its list pools for it; a
clustered box of 200,000 particles at theta = 0.3 then needs several times
more list chunks.  The first force call must walk at least twice, a repeated
call once, both must give bit-identical forces, and sampled groups must
match the FP64 oracle (lists exactly, forces to the parity bar).
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import check_forces, to_dev
from paper_0909_0541_amd import inputs

pytestmark = pytest.mark.gpu


def test_pools_grow_and_walk_again(gpu):
    bh = gpu
    ps, ms = inputs.plummer(2000, 3, with_vel=False)[:2]
    pos, mass = inputs.clustered(200000, 21, n_halos=50)[:2]
    eps, theta, n_crit = 1e-4, 0.3, 64
    # (a fixed cap: the automatic one may change with the previous call's lists)
    c = bh.Context(split_visits=-1)
    c.build_tree(to_dev(ps), to_dev(ms))
    c.make_groups(n_crit)
    c.compute_forces(1e-3, 0.5)
    assert c.get_stats().n_walk_attempts == 1

    c.build_tree(to_dev(pos), to_dev(mass))
    G = c.make_groups(n_crit)
    a1, p1 = c.compute_forces(eps, theta)
    st1 = c.get_stats()
    print("walks", st1.n_walk_attempts, "list entries", st1.list_entries, flush=True)
    assert st1.error_flags == 0 and st1.n_walk_attempts >= 2
    a1, p1 = a1.clone(), p1.clone()
    a2, p2 = c.compute_forces(eps, theta)
    st2 = c.get_stats()
    assert st2.error_flags == 0 and st2.n_walk_attempts == 1
    assert torch.equal(a1, a2) and torch.equal(p1, p2)
    assert st2.interactions == st1.interactions

    _, _, ll, lm = c.export_groups(lists=True)
    ll, lm = ll.cpu().numpy(), lm.cpu().numpy()
    t = oracle.Tree(pos, mass)
    assert t.groups(n_crit) == G
    sel = np.sort(np.random.default_rng(5).choice(G, 24, replace=False))
    sel = np.unique(np.concatenate([sel, np.argsort(ll)[-2:]]))
    ref = t.forces(eps, theta, groups=sel)
    assert np.array_equal(ll[sel], ref["list_len"])
    # sums of L positive FP64 terms in two orders: within 2 (L - 1) u of each other
    bound = ref["list_mass"] * ll[sel] * 2.0 ** -52
    assert np.all(np.abs(lm[sel] - ref["list_mass"]) <= bound)
    rows = np.flatnonzero(~np.isnan(ref["pot"]))
    sub = {"acc": ref["acc"][rows], "pot": ref["pot"][rows], "acc_abs": ref["acc_abs"][rows]}
    acc = a1.cpu().numpy().astype(np.float64)
    pot = p1.cpu().numpy().astype(np.float64)
    check_forces(acc[rows], pot[rows], sub)
