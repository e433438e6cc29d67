"""The autotuner of the captured step and the list tile length it searches.

Whatever tile the lists are handed over in, the lists are the same (exact
interaction counts) and the forces meet the parity bar against the oracle;
the autotuner keeps the candidate it measured fastest, and that candidate's
captured step computes oracle-matching forces."""
import numpy as np
import pytest

import oracle
from gpu_helpers import check_forces, to_dev
from paper_0909_0541_amd import autotune, inputs
from test_gpu_batch import _small_batch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tile", [128, 512, 2048])
def test_list_tile_keeps_lists_and_meets_the_bar(gpu, tile):
    """A clustered box at a small theta (lists of several thousand entries, so
    every tile length splits them into several chunks)."""
    bh = gpu
    pos, mass = inputs.clustered(40000, 23, n_halos=30)[:2]
    eps, theta, n_crit = 1e-4, 0.35, 128
    c = bh.Context(list_tile=tile)
    c.build_tree(to_dev(pos), to_dev(mass))
    c.make_groups(n_crit)
    acc, pot = c.compute_forces(eps, theta)
    st = c.get_stats()
    assert st.error_flags == 0 and st.max_list > 2 * tile
    t = oracle.Tree(pos, mass)
    t.groups(n_crit)
    ref = t.forces(eps, theta)
    assert st.interactions == ref["interactions"]
    check_forces(acc.cpu().numpy().astype(np.float64), pot.cpu().numpy().astype(np.float64), ref)


def test_bad_list_tile_is_rejected(gpu):
    bh = gpu
    for bad in (64, 100, 4096, -1):
        with pytest.raises(bh.BHError, match="list_tile"):
            bh.Context(list_tile=bad)


def test_autotuner_keeps_its_fastest_trial_and_it_meets_the_bar(gpu):
    bh = gpu
    pos, mass, off, eps, theta = _small_batch()
    dpos, dmass = to_dev(pos), to_dev(mass)
    best, trials, ctx = autotune.autotune(off, dpos, dmass, eps, theta, n_crits=(16, 64), waves=(0,),
                                          tiles=(128, 1024), steps=3)
    assert len(trials) == 4
    assert best.ms_per_step == min(t.ms_per_step for t in trials)
    assert best in trials
    # the returned context holds the winner's capture
    st = ctx.get_stats()
    assert st.error_flags == 0 and st.n_crit == best.n_crit and st.interactions == best.interactions
    ctx.graph_launch()
    ctx.sync()
    acc = ctx._graph_io[2].cpu().numpy().astype(np.float64)
    pot = ctx._graph_io[3].cpu().numpy().astype(np.float64)
    inter = 0
    for k in range(len(off) - 1):
        a, b = int(off[k]), int(off[k + 1])
        if b == a:
            continue
        t = oracle.Tree(pos[a:b], mass[a:b])
        t.groups(best.n_crit)
        ref = t.forces(eps[k], theta[k])
        inter += int(ref["interactions"])
        check_forces(acc[a:b], pot[a:b], ref)
    assert inter == best.interactions
