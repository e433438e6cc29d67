"""Split walks: a group whose walk reaches the visit cap hands the rest of its
stack to new walk tasks, and its list is summed in segments.  With a tiny cap
(64 node tests) nearly every group splits, several times over; lists must
still equal the oracle's, forces meet the parity bar, and results must not
depend on when the tasks ran."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import check_forces, gpu_run, to_dev
from paper_0909_0541_amd import inputs

pytestmark = pytest.mark.gpu


def _cases():
    p8, m8, _ = inputs.plummer(8192, 1, with_vel=False)
    pc, mc = inputs.clustered(20000, 9, n_halos=40)[:2]
    dup = np.repeat(np.random.default_rng(3).uniform(0, 1, (300, 3)), 3, axis=0)
    return [("plummer_8k", p8, m8, 1 / 256, 0.75, 64), ("clustered_20k", pc, mc, 1e-4, 0.6, 64),
            ("duplicates", dup, np.full(900, 1 / 900), 1e-3, 0.5, 16)]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
@pytest.mark.parametrize("cap", [64, 500, 0])
def test_split_lists_and_forces_match_oracle(gpu, case, cap):
    bh = gpu
    name, pos, mass, eps, theta, n_crit = case
    c = bh.Context(split_visits=cap)
    c, acc, pot, st, G = gpu_run(bh, pos, mass, eps, theta, n_crit, ctx=c)
    assert st.error_flags == 0
    if cap == 64:  # nearly every group splits; on the larger trees tasks hand over again
        assert st.n_split_groups > 0 and st.n_segments > st.n_split_groups
        assert st.n_split_levels >= (1 if name == "duplicates" else 2)
    t = oracle.Tree(pos, mass)
    t.groups(n_crit)
    ref = t.forces(eps, theta)
    _, _, ll, lm = c.export_groups(lists=True)
    assert np.array_equal(ll.cpu().numpy(), ref["list_len"])
    np.testing.assert_allclose(lm.cpu().numpy(), ref["list_mass"], rtol=1e-13)
    assert st.interactions == ref["interactions"]
    check_forces(acc, pot, ref)


def test_split_with_more_segments_than_the_rank_sort_takes(gpu):
    """Enough segments (over 16384) that their order comes from the radix
    sort rather than the small rank sort."""
    bh = gpu
    pos, mass = inputs.clustered(100000, 19, n_halos=100)[:2]
    eps, theta, n_crit = 1e-4, 0.6, 64
    c = bh.Context(split_visits=64)
    c, acc, pot, st, G = gpu_run(bh, pos, mass, eps, theta, n_crit, ctx=c)
    assert st.error_flags == 0 and st.n_segments > 16384
    t = oracle.Tree(pos, mass)
    t.groups(n_crit)
    ref = t.forces(eps, theta)
    _, _, ll, lm = c.export_groups(lists=True)
    ll = ll.cpu().numpy()
    assert np.array_equal(ll, ref["list_len"])
    # list mass: an FP64 sum of L positive masses, here over many segments
    # summed in key order; two orders of the same L terms differ by at most
    # 2 (L - 1) u of the sum (u = 2^-53 each side)
    lm = lm.cpu().numpy()
    assert np.all(np.abs(lm - ref["list_mass"]) <= 2.0 * np.maximum(ll - 1, 0) * 2.0**-53 * ref["list_mass"])
    assert st.interactions == ref["interactions"]
    check_forces(acc, pot, ref)


def test_split_is_deterministic_and_batch_equals_standalone(gpu):
    bh = gpu
    pos, mass, off, eps = inputs.batch_systems(seed=9, n_systems=6, n_min=2000, n_max=20000)
    theta = np.full(6, 0.7)
    dpos, dmass = to_dev(pos), to_dev(mass)
    outs = []
    for _ in range(2):
        c = bh.Context(split_visits=64)
        c.build_batch(off, dpos, dmass)
        c.make_groups(32)
        a, p = c.compute_forces_batch(eps, theta)
        outs.append((a.clone(), p.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    for k in range(6):
        lo, hi = int(off[k]), int(off[k + 1])
        c = bh.Context(split_visits=64)
        c.build_tree(dpos[lo:hi].contiguous(), dmass[lo:hi].contiguous())
        c.make_groups(32)
        a, p = c.compute_forces(float(eps[k]), 0.7)
        assert torch.equal(a, outs[0][0][lo:hi]) and torch.equal(p, outs[0][1][lo:hi]), f"system {k}"


def test_split_graph_replays(gpu):
    bh = gpu
    pos, mass = inputs.clustered(20000, 17, n_halos=20)[:2]
    dpos, dmass = to_dev(pos), to_dev(mass)
    off = np.array([0, 20000])
    c0 = bh.Context(split_visits=64)
    c0.build_tree(dpos, dmass)
    c0.make_groups(64)
    a0, p0 = c0.compute_forces(1e-4, 0.6)
    c = bh.Context(split_visits=64)
    acc, pot = c.graph_capture(off, dpos, dmass, 64, [1e-4], [0.6])
    torch.cuda.synchronize()
    assert torch.equal(acc, a0) and torch.equal(pot, p0)
    for k in range(3):
        acc.zero_()
        c.graph_launch()
        c.sync()
        assert torch.equal(acc, a0) and torch.equal(pot, p0), f"replay {k}"
