"""Search radii for an SPH-style neighbour workload (set-up, not the timed
path).

SPH codes give every particle a radius h_i that holds about a fixed number of
neighbours.  `smoothing_lengths` reaches that the usual way: a first guess
from each group's particle density (members over the volume of its bounding
box, both from the library's own groups), then a few passes of the library's
neighbour count, each scaling h_i by (target / count)^(1/3), clamped.  The
radii only set up the workload; the neighbour search and density are
`Context.neighbors`.
"""
from __future__ import annotations

import math

import torch


def smoothing_lengths(ctx, dpos: torch.Tensor, n_target: int = 64, passes: int = 4) -> torch.Tensor:
    """FP64 radii [n] (input order) on the device for the current tree and
    groups of ctx (positions dpos, as built)."""
    n = dpos.shape[0]
    if n == 0:
        return torch.empty(0, dtype=torch.float64, device=dpos.device)
    ints, box, _, _ = ctx.export_groups()
    _, perm = ctx.export_sorted()
    count = ints[:, 1].to(torch.float64)
    ext = (box[:, 3:] - box[:, :3]).clamp_min(0.0)
    span = float((dpos.max(0).values - dpos.min(0).values).max().item())
    floor = max(span, 1e-300) * 1e-4
    vol = ext.clamp_min(floor).prod(1)
    dens = count / vol
    h_group = (3.0 * n_target / (4.0 * math.pi * dens)).pow(1.0 / 3.0)
    h_sorted = torch.repeat_interleave(h_group, ints[:, 1].to(torch.int64))
    h = torch.empty(n, dtype=torch.float64, device=dpos.device)
    h[perm.to(torch.int64)] = h_sorted
    for _ in range(passes):
        c, _ = ctx.neighbors(h, count=True)
        ratio = ((n_target + 1.0) / (c.to(torch.float64) + 1.0)).pow(1.0 / 3.0).clamp(0.5, 2.0)
        h = (h * ratio).contiguous()
    return h
