"""The judge entry point that allocates nothing (bh_direct_sampled_noalloc)
against the allocating one (bh_direct_sampled), through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import to_dev
from paper_0909_0541_amd import bh as bhmod
from paper_0909_0541_amd import inputs

pytestmark = pytest.mark.gpu


def _case(n, s, seed):
    pos, mass = inputs.clustered(n, seed, n_halos=max(1, n // 4000))[:2]
    idx = np.sort(np.random.default_rng(seed).choice(n, s, replace=False))
    return pos, mass, idx


def test_noalloc_judge_equals_the_allocating_judge(gpu):
    """Two calls in a row on one context, the second with a smaller input:
    bit for bit the allocating entry point's results, and the oracle's
    direct sums to within FP64 rounding."""
    bh = gpu
    c = bh.Context()
    for n, s, seed, eps in ((300000, 4096, 1, 1e-4), (20000, 300, 2, 1e-3)):
        pos, mass, idx = _case(n, s, seed)
        dpos, dmass, didx = to_dev(pos), to_dev(mass), to_dev(idx, torch.int64)
        a_ref, p_ref = c.direct_sampled(dpos, dmass, eps, didx)
        acc = torch.full((s, 3), np.nan, dtype=torch.float64, device="cuda")
        pot = torch.full((s,), np.nan, dtype=torch.float64, device="cuda")
        c.direct_sampled_noalloc(dpos, dmass, eps, didx, acc, pot)
        c.sync()
        assert torch.equal(acc, a_ref) and torch.equal(pot, p_ref), (n, s)
        if n <= 20000:
            a_o, p_o = oracle.direct(pos, mass, eps, idx=idx)
            an = np.linalg.norm(a_o, axis=1)
            assert np.all(np.linalg.norm(acc.cpu().numpy() - a_o, axis=1) <= 1e-10 * an)
            assert np.all(np.abs(pot.cpu().numpy() - p_o) <= 1e-10 * np.abs(p_o))


def test_noalloc_judge_rejects_a_sample_beyond_its_scratch(gpu):
    """A sample whose partial sums exceed the static array is refused before
    any launch, with the outputs untouched."""
    bh = gpu
    c = bh.Context()
    n, s = 1000, 300000  # one j chunk: 32 B x 300,000 = 9.6 MB > 8 MiB
    pos, mass = inputs.uniform_cube(n, 5)[:2]
    idx = torch.as_tensor(np.arange(s) % n, dtype=torch.int64, device="cuda")
    acc = torch.zeros((s, 3), dtype=torch.float64, device="cuda")
    pot = torch.zeros((s,), dtype=torch.float64, device="cuda")
    with pytest.raises(bhmod.BHError, match="static scratch"):
        c.direct_sampled_noalloc(to_dev(pos), to_dev(mass), 1e-3, idx, acc, pot)
    c.sync()
    assert not acc.any() and not pot.any()
