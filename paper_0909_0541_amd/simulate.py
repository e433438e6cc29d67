"""Leapfrog time integration of a workload with the tree forces (GPU).

    python -m paper_0909_0541_amd.simulate --workload clustered_8m --steps 100 --dt 1e-4

Kick-drift-kick with FP64 positions and velocities and FP32 accelerations;
the tree and groups are rebuilt every step (the time integration of the
paper's cosmological run, Sec. 4, with the scheme as the reading).  theta is
either fixed or chosen per group by the trained network; in both cases it is
first calibrated on the initial state to the target RMS force error against
FP64 direct summation on a seeded sample (bisection of theta, or of the
network's output shift), then held for the run.  Prints one JSON line with
the energy at every checkpoint, the relative energy drift, the step time and
the throughput.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from . import bh, inputs, learned


def energy(ctx, vel, mass, pot):
    e = ctx.energy(vel, mass, pot).cpu().numpy()
    return float(e[0]), float(e[1])


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="clustered_8m")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--dt", type=float, default=1e-4)
    ap.add_argument("--target-rms", type=float, default=1e-3)
    ap.add_argument("--theta", type=float, default=None, help="fixed theta (skips calibration)")
    ap.add_argument("--learned", action="store_true", help="per-group theta from the trained network")
    ap.add_argument("--theta-net", default=learned.DEFAULT_NET)
    ap.add_argument("--judge-sample", type=int, default=4096)
    ap.add_argument("--every", type=int, default=10, help="energy checkpoint interval")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    pos, mass, vel, w = inputs.make_workload(args.workload, n=args.n, with_vel=True)
    n = pos.shape[0]
    x = torch.as_tensor(pos, device="cuda")
    v = torch.as_tensor(vel, device="cuda")
    m = torch.as_tensor(mass, device="cuda")
    ctx = bh.Context()
    net = learned.ThetaNet.load(args.theta_net) if args.learned else None
    step = learned.Stepper(ctx, x, m, w.eps, w.n_crit, net)
    theta, shift, calib_rms = (w.theta if args.theta is None else args.theta), 0.0, None
    if args.theta is None and args.target_rms > 0:
        judge = learned.Judge(ctx, x, m, w.eps, args.judge_sample)
        if net is None:
            def f(th):
                step(theta=th)
                return judge.rms(step.acc)
            theta, calib_rms = learned.bisect(f, 0.3, 1.0, args.target_rms)
        else:
            def f(sh):
                step(shift=sh)
                return judge.rms(step.acc)
            shift, calib_rms = learned.bisect(f, -8.0, 8.0, args.target_rms)
    step(theta=theta, shift=shift)  # forces at the initial positions
    acc, pot = step.acc, step.pot
    k0, u0 = energy(ctx, v, m, pot)
    log = [{"step": 0, "kinetic": k0, "potential": u0, "total": k0 + u0}]
    h = 0.5 * args.dt
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    inter = 0
    for s in range(1, args.steps + 1):
        if net is None:
            ctx.leapfrog(x, v, m, w.eps, theta, w.n_crit, args.dt, 1, acc, pot)
        else:
            ctx.kick(v, acc, h)
            ctx.drift(x, v, args.dt)
            step(shift=shift)
            ctx.kick(v, acc, h)
        if s % args.every == 0 or s == args.steps:
            st = ctx.get_stats()  # synchronises; counts the last force call
            inter += st.interactions
            k, u = energy(ctx, v, m, pot)
            log.append({"step": s, "kinetic": k, "potential": u, "total": k + u})
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    st = ctx.get_stats()
    etot = [r["total"] for r in log]
    out = {"workload": w.name, "n": n, "steps": args.steps, "dt": args.dt, "eps": w.eps, "n_crit": w.n_crit,
           "theta_mode": "learned" if net is not None else "fixed", "theta": theta, "shift": shift,
           "calibration_rms": calib_rms, "ms_per_step": ms, "particles_per_s": n / (ms * 1e-3),
           "interactions_last_step": st.interactions,
           "energy_drift": (etot[-1] - etot[0]) / abs(etot[0]),
           "max_energy_error": max(abs(e - etot[0]) for e in etot) / abs(etot[0]),
           "energy": log, "error_flags": st.error_flags,
           "note": "step time includes the energy checkpoints every --every steps"}
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
    sys.exit(0)
