#!/usr/bin/env python3
"""Benchmark of the grouped Barnes-Hut tree force on one MI355X.

One step = the whole hot path over one synthetic particle set already
resident in HBM: root cube, Morton keys, radix sort, tree topology and
moments, groups, the group walk writing the interaction lists, and the FP32
force sum.  Default workload: clustered box, N = 2,097,152 (30% uniform + 70%
in 512 Plummer halos), eps = 1e-4, n_crit = 256.

Before timing, theta is bisected until the RMS relative force error against
FP64 direct summation on a seeded sample of 4096 particles is 1e-3 (+-3%).
Prints one JSON line.  value = tree-force interactions per second of whole
steps at that theta (sum over members of list length - 1, divided by the
step time).  Beside it: particles/s; the learned per-group theta at the same
error (its output shift bisected the same way, features + network in the
step); the quadrupole option and Peano-Hilbert order at the same error; the
neighbour search with SPH densities at 64 neighbours per particle; the
per-particle walk at the same error; the workload's own theta of 0.6; the
roofline of the dominant kernel (the force sum, FP32 VALU); and the FP64 CPU
oracle's throughput.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "tree-force interactions/s and particles/s at 1e-3 RMS force error, learned vs fixed θ"
FP32_VALU_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
FLOPS_PER_INTERACTION = 20      # 3 sub, 3 FMA (r^2), rsqrt, 3 mul, 3 FMA (acc), 1 add (pot)


# HBM traffic of the force kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# of this script (bytes per interaction, scaled by the counters' reading of a
# device copy of known size), valid only for the kernel source it was taken on.
TRAFFIC = {
    # clustered box, 2,097,152 particles, theta 0.4203125 (the 1e-3 RMS theta):
    # FETCH_SIZE 2830548.1 KiB x 1.99987 (a 512 MiB device copy reads as
    # 262160.69 KiB) + WRITE_SIZE 145878.8 KiB x 1.0 (the copy writes 524288 KiB)
    "clustered_2m": {"theta": 0.4203125, "bytes_per_launch": 5945973442,
                     "k_force_sha256": "62fa39ed51d4b632e2aa53196c44a7abed544f7f661602e52b7600e59dfb1141"},
}


def traffic_for(workload, theta):
    rec = TRAFFIC.get(workload)
    if rec is None or abs(rec["theta"] - theta) > 1e-12:
        return None
    src = os.path.join(ROOT, "paper_0909_0541_amd", "csrc", "k_force.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["k_force_sha256"]:
            return None
    return rec["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered_2m")
    ap.add_argument("--n", type=int, default=None, help="override the particle count")
    ap.add_argument("--judge-sample", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--waves-per-cu", type=int, default=None)
    ap.add_argument("--theta", type=float, default=None,
                    help="time this fixed theta (no calibration, no learned leg)")
    ap.add_argument("--target-rms", type=float, default=1e-3,
                    help="calibrate theta by bisection to this RMS force error before timing "
                         "(0: time the workload's own theta)")
    ap.add_argument("--theta-lo", type=float, default=0.3,
                    help="lower end of the theta bisections (tighter targets need smaller theta)")
    ap.add_argument("--theta-net", default=os.path.join(ROOT, "paper_0909_0541_amd", "theta_net.npz"),
                    help="trained per-group theta network (the learned leg is skipped when missing)")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-particle", action="store_true", help="skip the per-particle walk A/B leg")
    ap.add_argument("--no-quadrupole", action="store_true", help="skip the quadrupole A/B leg")
    ap.add_argument("--no-neighbors", action="store_true", help="skip the neighbour-search leg")
    ap.add_argument("--no-hilbert", action="store_true", help="skip the Peano-Hilbert order A/B leg")
    ap.add_argument("--curve", type=int, default=0, choices=(0, 1),
                    help="key order of the headline step: 0 Morton (default), 1 Peano-Hilbert (for counter runs)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-systems leg")
    ap.add_argument("--copy-check-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB before the timed steps, "
                         "as the reference kernel that scales HBM byte counters")
    return ap.parse_args()


def cpu_baseline(pos, mass, w, total_interactions, target_s):
    """The FP64 oracle on the host: full tree build and grouping, then the
    walk + force sum for a seeded random sample of groups sized to about
    target_s seconds; whole-job throughput is extrapolated from the sample."""
    import numpy as np

    import oracle

    t0 = time.perf_counter()
    tree = oracle.Tree(pos, mass)
    G = tree.groups(w.n_crit)
    t_build = time.perf_counter() - t0
    order = np.random.default_rng(0).permutation(G)
    k = max(8, G // 500)
    t0 = time.perf_counter()
    pilot = tree.forces(w.eps, w.theta, groups=order[:k])
    dt = time.perf_counter() - t0
    rate = max(pilot["interactions"], 1) / max(dt, 1e-6)
    want = max(1.0, target_s - dt) * rate
    # extend the sample until it holds about `want` interactions
    frac = min(1.0, want / max(total_interactions, 1))
    k2 = int(min(G, max(k, round(frac * G))))
    t0 = time.perf_counter()
    out = tree.forces(w.eps, w.theta, groups=order[:k2])
    t_force = time.perf_counter() - t0
    sample_inter = max(out["interactions"], 1)
    t_job = t_build + t_force * total_interactions / sample_inter
    return {
        "value": total_interactions / t_job,
        "unit": "interactions/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"FP64 oracle: full tree build + grouping of all {pos.shape[0]} particles "
                   f"({t_build:.2f} s), walk + force for {k2} of {G} groups chosen at random "
                   f"({sample_inter} interactions, {t_force:.2f} s); whole job extrapolated by "
                   f"interaction count"),
        "cpu_model": _cpu_model(),
    }


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def batch_leg(args):
    """64 independent systems of uneven size (Plummer spheres and clustered
    boxes, N log-uniform in [1024, 262144], theta = 0.7, eps = N^(-1/3)/20) as
    one captured HIP graph per step, n_crit and waves per CU autotuned."""
    import torch

    from paper_0909_0541_amd import autotune, inputs

    pos, mass, off, eps = inputs.batch_systems()
    dpos = torch.as_tensor(pos, device="cuda")
    dmass = torch.as_tensor(mass, device="cuda")
    theta = 0.7
    best, trials, ctx = autotune.autotune(off, dpos, dmass, eps, theta)
    ms = autotune.time_graph(ctx, args.steps, args.warmup)
    st = ctx.get_stats()
    acc = ctx._graph_io[2]
    n = int(off[-1])
    return {"workload": "batch_64", "systems": int(len(off) - 1), "n": n, "theta": theta,
            "n_crit": best.n_crit, "waves_per_cu": best.waves_per_cu, "ms_per_step": ms,
            "interactions_per_step": st.interactions, "interactions_per_s": st.interactions / (ms * 1e-3),
            "particles_per_s": n / (ms * 1e-3),
            "rms_force_error": autotune.batch_rms(ctx, off, dpos, dmass, eps, acc, sample=args.judge_sample),
            "step": "one HIP graph replay: build of all 64 trees, groups, list walk, force sum",
            "autotune": [{"n_crit": t.n_crit, "waves_per_cu": t.waves_per_cu, "ms": t.ms_per_step}
                         for t in trials]}


def particle_leg(args, ctx, judge, dpos, dmass, w, line):
    """The paper's own GPU form as an A/B: every particle walks the tree by
    itself and sums on the way (no groups, no lists); theta bisected to the
    same RMS error; the step is the tree build plus that walk."""
    import torch

    from paper_0909_0541_amd import learned

    n = dpos.shape[0]

    def step(th):
        ctx.build_tree(dpos, dmass)
        return ctx.compute_forces_particle(w.eps, th)

    def rms_of(th):
        acc, _ = step(th)
        return judge.rms(acc)

    theta, r = learned.bisect(rms_of, 0.2, 1.0, args.target_rms)
    for _ in range(max(args.warmup, 1)):
        step(theta)
    torch.cuda.synchronize()
    ctx.get_stats()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    steps = max(1, min(args.steps, 5))
    e0.record()
    for _ in range(steps):
        step(theta)
    e1.record()
    torch.cuda.synchronize()
    st = ctx.get_stats()
    if st.error_flags:
        raise RuntimeError(f"device error flags {st.error_flags}")
    ms = e0.elapsed_time(e1) / steps
    return {"theta": theta, "rms_force_error": r, "ms_per_step": ms, "interactions_per_step": st.interactions,
            "interactions_per_s": st.interactions / (ms * 1e-3), "particles_per_s": n / (ms * 1e-3),
            "walk_ms": st.t_particle_ms / max(st.n_particle_calls, 1), "max_list": st.max_list,
            "grouped_speedup": ms / line["ms_per_step"],
            "interactions_vs_grouped": st.interactions / line["interactions_per_step"],
            "step": "tree build + per-particle walk and sum (the paper's threaded-tree kernel form)"}


def variant_leg(args, judge, dpos, dmass, w, line, inter_ref, step, **opts):
    """An option of the same step as an A/B at the same RMS force error:
    theta bisected to the target error with the option set, timed as a graph
    replay checked bit for bit against its eager step."""
    import numpy as np
    import torch

    from paper_0909_0541_amd import autotune, bh, learned

    n = dpos.shape[0]
    vctx = bh.Context(timing=True, waves_per_cu=args.waves_per_cu, **opts)
    v = learned.Stepper(vctx, dpos, dmass, w.eps, w.n_crit)

    def rms_of(th):
        v(theta=th)
        return judge.rms(v.acc)

    theta, r = learned.bisect(rms_of, args.theta_lo, 1.0, args.target_rms)
    ms_eager, st = learned.timed_steps(v, args.steps, args.warmup, theta=theta)
    per = lambda t, k: t / max(k, 1)
    stage = {"build": per(st.t_build_ms, st.n_build_calls), "groups": per(st.t_groups_ms, st.n_groups_calls),
             "walk": per(st.t_walk_ms, st.n_walk_calls), "force": per(st.t_force_ms, st.n_force_calls)}
    ms, mode = ms_eager, "eager"
    try:
        g = bh.Context(waves_per_cu=args.waves_per_cu, **opts)
        g.graph_capture(np.array([0, n], dtype=np.int64), dpos, dmass, w.n_crit, [w.eps], [theta])
        ms_g = autotune.time_graph(g, args.steps, args.warmup)
        gst = g.get_stats()
        if not gst.error_flags and gst.interactions == st.interactions and torch.equal(g._graph_io[2], v.acc):
            ms, mode = ms_g, "graph"
        del g
    except (RuntimeError, bh.BHError):
        pass
    return {"options": opts, "theta": theta, "rms_force_error": judge.rms(v.acc), "ms_per_step": ms,
            "step_mode": mode, "eager_ms_per_step": ms_eager, "interactions_per_step": st.interactions,
            "interactions_per_s": st.interactions / (ms * 1e-3), "particles_per_s": n / (ms * 1e-3),
            "stage_ms": stage, "max_list": st.max_list, "groups": st.n_groups,
            "interactions_vs_default": st.interactions / inter_ref,
            "particles_per_s_vs_default": (n / (ms * 1e-3)) / line["particles_per_s"],
            "step": step}


FP64_VALU_PEAK_TFLOPS = 78.6    # MI355X published FP64 vector peak
NEIGHBOR_NCRIT = 64             # group size of the neighbour search
FLOPS_PER_NEIGHBOR_TEST = 8      # FP64: 3 sub, 3 mul, 2 add for r^2 (the compare is not counted)


def neighbor_leg(args, dpos, dmass, w):
    """Neighbour search and SPH density (the general treewalk for a short-
    range interaction) on the same particles: radii for 64 neighbours (set-up,
    a few count passes), then the search with counts and densities timed."""
    import torch

    from paper_0909_0541_amd import bh, sph

    n = dpos.shape[0]
    c = bh.Context(timing=True, waves_per_cu=args.waves_per_cu)
    c.build_tree(dpos, dmass)
    c.make_groups(w.n_crit)
    h = sph.smoothing_lengths(c, dpos, n_target=64)
    # the search's own groups: smaller groups test fewer candidate pairs per
    # member (64 measured best on this machine; 256 tests 2.2x as many pairs)
    c.make_groups(NEIGHBOR_NCRIT)
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    rho = torch.empty(n, dtype=torch.float64, device="cuda")
    for _ in range(max(args.warmup, 1)):
        c.neighbors(h, count=True, rho=True)
    torch.cuda.synchronize()
    c.get_stats()
    steps = max(1, args.steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        c.neighbors(h, count=True, rho=True)
    e1.record()
    torch.cuda.synchronize()
    st = c.get_stats()
    if st.error_flags:
        raise RuntimeError(f"device error flags {st.error_flags}")
    ms = e0.elapsed_time(e1) / steps
    kms = st.t_neighbor_ms / max(st.n_neighbor_calls, 1)
    achieved = FLOPS_PER_NEIGHBOR_TEST * st.neighbor_tests / (kms * 1e-3) / 1e12
    cn = c.neighbors(h, count=True)[0].cpu()
    return {"workload": w.name, "n": n, "n_target": 64, "n_crit": NEIGHBOR_NCRIT, "ms_per_call": ms, "kernel_ms": kms,
            "neighbor_pairs": st.neighbor_pairs, "pair_tests": st.neighbor_tests,
            "pairs_per_s": st.neighbor_pairs / (ms * 1e-3), "tests_per_s": st.neighbor_tests / (ms * 1e-3),
            "particles_per_s": n / (ms * 1e-3),
            "median_neighbors": float(cn.median().item()), "max_neighbors": int(cn.max().item()),
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP64_VALU_PEAK_TFLOPS, "kernel": "k_neighbors",
                         "flops_per_test": FLOPS_PER_NEIGHBOR_TEST},
            "step": "neighbour counts and SPH densities of every particle on a built tree and groups"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              f"(the method runs on a single MI355X here)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_0909_0541_amd import bh, inputs, learned

    torch.cuda.set_device(0)
    pos, mass, _, w = inputs.make_workload(args.workload, n=args.n)
    n = pos.shape[0]
    dpos = torch.as_tensor(pos, device="cuda")
    dmass = torch.as_tensor(mass, device="cuda")
    ctx = bh.Context(timing=True, waves_per_cu=args.waves_per_cu, curve=args.curve)
    judge = learned.Judge(ctx, dpos, dmass, w.eps, args.judge_sample)
    fixed = learned.Stepper(ctx, dpos, dmass, w.eps, w.n_crit)

    calib = None
    theta = w.theta if args.theta is None else args.theta
    if args.target_rms > 0 and args.theta is None:
        def rms_of(th):
            fixed(theta=th)
            return judge.rms(fixed.acc)
        theta, r = learned.bisect(rms_of, args.theta_lo, 1.0, args.target_rms)
        calib = {"target_rms": args.target_rms, "theta": theta, "rms": r, "band": 0.03,
                 "search": f"bisection over theta in [{args.theta_lo}, 1.0]"}

    if args.copy_check_mib > 0:
        nb = args.copy_check_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def stages(st):
        per = lambda t, k: t / max(k, 1)
        return {"build": per(st.t_build_ms, st.n_build_calls), "groups": per(st.t_groups_ms, st.n_groups_calls),
                "walk": per(st.t_walk_ms, st.n_walk_calls), "force": per(st.t_force_ms, st.n_force_calls)}

    ms_eager, st = learned.timed_steps(fixed, args.steps, args.warmup, theta=theta)
    stage = stages(st)
    rms = judge.rms(fixed.acc)
    inter = st.interactions
    # The timed step: the same whole step (build, groups, list walk, force
    # sum) captured once as a HIP graph and replayed, which takes the host's
    # launch work and the force call's list-pool check off the GPU's path.
    # (A replay that does not reproduce the eager step's forces bit for bit
    # is not reported: the eager time is then the step time.)
    from paper_0909_0541_amd import autotune
    step_mode, graph_error = "graph", None
    try:
        gctx = bh.Context(waves_per_cu=args.waves_per_cu, curve=args.curve)
        gctx.graph_capture(np.array([0, n], dtype=np.int64), dpos, dmass, w.n_crit, [w.eps], [theta])
        ms_per_step = autotune.time_graph(gctx, args.steps, args.warmup)
        gst = gctx.get_stats()
        if gst.error_flags or gst.interactions != inter or not torch.equal(gctx._graph_io[2], fixed.acc):
            raise RuntimeError(f"replay differs from the eager step (flags {gst.error_flags}, "
                               f"interactions {gst.interactions} vs {inter})")
        del gctx
    except (RuntimeError, bh.BHError) as e:
        step_mode, graph_error, ms_per_step = "eager", str(e), ms_eager
    value = inter / (ms_per_step * 1e-3)
    t_force = stage["force"]
    achieved = FLOPS_PER_INTERACTION * inter / (t_force * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "description": w.description, "n": n, "eps": w.eps, "theta": theta,
                   "workload_theta": w.theta, "n_crit": w.n_crit,
                   "theta_mode": "fixed" if calib is None else "fixed, bisected to the target RMS force error",
                   "key_order": "Peano-Hilbert" if args.curve else "Morton"},
        "particles_per_s": n / (ms_per_step * 1e-3),
        "step": ("one HIP graph replay: tree build, groups, list walk, force sum" if step_mode == "graph"
                 else f"eager calls (graph replay not used: {graph_error})"),
        "eager": {"ms_per_step": ms_eager, "interactions_per_s": inter / (ms_eager * 1e-3),
                  "step": "the same calls issued one by one (the force call waits for the walk to check its "
                          "list pools)"},
        "interactions_per_step": inter,
        "interactions_per_particle": inter / n,
        "rms_force_error": rms,
        "judge_sample": int(judge.idx.shape[0]),
        "theta_calibration": calib,
        "groups": st.n_groups,
        "cells": st.n_cells,
        "max_list": st.max_list,
        "stage_ms": stage,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": traffic_for(w.name, theta),
                     "kernel": "k_force_lists", "flops_per_interaction": FLOPS_PER_INTERACTION},
        "force_kernel_interactions_per_s": inter / (t_force * 1e-3),
        "walk_plus_force_interactions_per_s": inter / ((stage["walk"] + t_force) * 1e-3),
    }
    if calib is not None and not args.no_learned and os.path.exists(args.theta_net):
        net = learned.ThetaNet.load(args.theta_net)
        lstep = learned.Stepper(ctx, dpos, dmass, w.eps, w.n_crit, net)

        def rms_shift(sh):
            lstep(shift=sh)
            return judge.rms(lstep.acc)
        sh, r = learned.bisect(rms_shift, -8.0, 8.0, args.target_rms)
        if abs(r / args.target_rms - 1) <= 0.03 or r <= args.target_rms:
            ms_l, st_l = learned.timed_steps(lstep, args.steps, args.warmup, shift=sh)
            tg = lstep.theta_g[:st_l.n_groups].cpu().numpy()
            line["learned"] = {
                "shift": sh, "rms_force_error": judge.rms(lstep.acc), "ms_per_step": ms_l,
                "interactions_per_step": st_l.interactions, "interactions_per_s": st_l.interactions / (ms_l * 1e-3),
                "particles_per_s": n / (ms_l * 1e-3), "stage_ms": stages(st_l),
                "theta_mean": float(tg.mean()), "theta_min": float(tg.min()), "theta_max": float(tg.max()),
                "interactions_saved": 1.0 - st_l.interactions / inter,
                "particles_per_s_vs_fixed": (n / (ms_l * 1e-3)) / line["particles_per_s"]}
        else:
            line["learned"] = {"fallback_to_fixed": True, "shift": sh, "rms_force_error": r}
    if calib is not None and abs(theta - w.theta) > 1e-12:
        ms2, st2 = learned.timed_steps(fixed, args.steps, args.warmup, theta=w.theta)
        s2 = stages(st2)
        line["at_workload_theta"] = {
            "theta": w.theta, "rms_force_error": judge.rms(fixed.acc), "ms_per_step": ms2,
            "interactions_per_s": st2.interactions / (ms2 * 1e-3), "particles_per_s": n / (ms2 * 1e-3),
            "interactions_per_step": st2.interactions, "stage_ms": s2,
            "force_kernel_tflops": FLOPS_PER_INTERACTION * st2.interactions / (s2["force"] * 1e-3) / 1e12}
    if calib is not None and not args.no_quadrupole:
        line["quadrupole"] = variant_leg(
            args, judge, dpos, dmass, w, line, inter,
            "tree build with second moments, groups, list walk, force sum with quadrupole terms", quadrupole=True)
    if calib is not None and not args.no_hilbert:
        line["hilbert"] = variant_leg(
            args, judge, dpos, dmass, w, line, inter,
            "the same step with Peano-Hilbert keys (particles, children and groups in curve order)", curve=1)
    if not args.no_neighbors:
        line["neighbors"] = neighbor_leg(args, dpos, dmass, w)
    if calib is not None and not args.no_particle:
        line["per_particle"] = particle_leg(args, ctx, judge, dpos, dmass, w, line)
    if not args.no_batch:
        line["batch"] = batch_leg(args)
    if not args.no_cpu_baseline:
        w_cpu = dataclasses.replace(w, theta=theta)
        line["cpu_baseline"] = cpu_baseline(pos, mass, w_cpu, inter, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
