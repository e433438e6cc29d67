"""Autotuner of the captured step: group size n_crit, waves per CU and the
list tile length.

For a given particle set (one system or a batch of many), every candidate
(n_crit, waves per CU, list tile) is captured as a HIP graph
(bh_graph_capture) and its replays are timed with HIP events; the fastest
candidate wins.  The interaction lists, and so the accuracy, depend on n_crit
only through the grouping: a smaller group has a tighter box and a shorter
list, but more walks and more partly filled force blocks.  The list tile is
the number of entries per chunk in which the walk hands a group's list to
the force sum (which folds its FP32 partial sums into FP64 after each): a
longer tile means fewer chunk links and folds, a shorter one less unused
pool space at the end of each list.  The waves per CU cap the persistent
grids (0: as many as fit); 8 per CU was always the slowest on the batched
workload and is not searched.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
import torch

from . import bh

N_CRIT = (64, 128, 256)
WAVES_PER_CU = (0, 16)     # 0: as many as fit
LIST_TILE = (256, 512, 1024)


@dataclass
class Trial:
    n_crit: int
    waves_per_cu: int
    list_tile: int
    ms_per_step: float
    interactions: int
    groups: int


def time_graph(ctx: bh.Context, steps: int, warmup: int = 2) -> float:
    for _ in range(warmup):
        ctx.graph_launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        ctx.graph_launch()
    e1.record()
    torch.cuda.synchronize()
    ctx.sync()
    return e0.elapsed_time(e1) / steps


def autotune(offsets, dpos, dmass, eps_sys, theta_sys, n_crits=N_CRIT, waves=WAVES_PER_CU, tiles=LIST_TILE,
             steps: int = 5, log=None):
    """Time every (n_crit, waves per CU, list tile) candidate; returns (best
    Trial, all trials, the best candidate's context with its captured step)."""
    trials = []
    best = None
    best_ctx = None
    for nc, wv, tl in itertools.product(n_crits, waves, tiles):
        ctx = bh.Context(waves_per_cu=wv if wv > 0 else None, list_tile=tl)
        ctx.graph_capture(offsets, dpos, dmass, nc, eps_sys, theta_sys)
        ms = time_graph(ctx, steps)
        st = ctx.get_stats()
        tr = Trial(nc, wv, tl, ms, st.interactions, st.n_groups)
        trials.append(tr)
        if log:
            log(f"n_crit {nc:4d} waves/CU {wv:3d} tile {tl:5d}: {ms:8.3f} ms  {st.interactions:.4e} interactions")
        if best is None or ms < best.ms_per_step:
            if best_ctx is not None:
                best_ctx.close()
            best, best_ctx = tr, ctx
        else:
            ctx.close()
    return best, trials, best_ctx


def batch_rms(ctx: bh.Context, offsets, pos, mass, eps_sys, acc, sample: int = 4096, seed: int = 12345) -> float:
    """RMS relative force error of a batch on a seeded sample, each sampled
    particle judged by FP64 direct summation over its own system."""
    rng = np.random.default_rng(seed)
    n = int(offsets[-1])
    idx = np.sort(rng.choice(n, min(sample, n), replace=False))
    sys_of = np.searchsorted(offsets, idx, side="right") - 1
    a = acc.double().cpu().numpy()
    rel2 = []
    for s in np.unique(sys_of):
        lo, hi = int(offsets[s]), int(offsets[s + 1])
        local = idx[sys_of == s] - lo
        d, _ = ctx.direct_sampled(pos[lo:hi].contiguous(), mass[lo:hi].contiguous(), float(eps_sys[s]),
                                  torch.as_tensor(local, device="cuda"))
        d = d.cpu().numpy()
        t = a[lo + local]
        rel2.append((np.linalg.norm(t - d, axis=1) / np.linalg.norm(d, axis=1)) ** 2)
    r = np.concatenate(rel2)
    return float(np.sqrt(r.mean()))
