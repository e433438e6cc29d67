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

import torch

from . import bh, inputs, learned


def energy(ctx, vel, mass, pot):
    e = ctx.energy(vel, mass, pot).cpu().numpy()
    return float(e[0]), float(e[1])


def run(workload: str = "clustered_8m", n: int | None = None, steps: int = 100, dt: float = 1e-4,
        target_rms: float = 1e-3, theta: float | None = None, learned_theta: bool = False,
        theta_net: str = learned.DEFAULT_NET, judge_sample: int = 4096, every: int = 10):
    """Calibrate theta (or the network's shift) on the initial state, then run
    `steps` kick-drift-kick steps; returns the summary as a dict."""
    pos, mass, vel, w = inputs.make_workload(workload, n=n, with_vel=True)
    n = pos.shape[0]
    x = torch.as_tensor(pos, device="cuda")
    v = torch.as_tensor(vel, device="cuda")
    m = torch.as_tensor(mass, device="cuda")
    del pos, mass, vel
    ctx = bh.Context()
    net = learned.ThetaNet.load(theta_net) if learned_theta else None
    th, shift, calib_rms, mode, reason = (w.theta if theta is None else theta), 0.0, None, "fixed", ""
    if theta is None and target_rms > 0:
        judge = learned.Judge(ctx, x, m, w.eps, judge_sample)
        cal = learned.calibrate(ctx, x, m, w.eps, w.n_crit, net, judge, target_rms)
        th, mode, reason = cal.theta, cal.mode, cal.reason
        shift = cal.shift if cal.mode == "learned" else 0.0
        calib_rms = cal.learned_rms if cal.mode == "learned" else cal.fixed_rms
    elif net is not None:
        mode = "learned"
    step = learned.Stepper(ctx, x, m, w.eps, w.n_crit, net if mode == "learned" else None)
    step(theta=th, shift=shift)  # forces at the initial positions
    acc, pot = step.acc, step.pot
    k0, u0 = energy(ctx, v, m, pot)
    log = [{"step": 0, "kinetic": k0, "potential": u0, "total": k0 + u0}]
    h = 0.5 * dt
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for s in range(1, steps + 1):
        if mode == "fixed":
            ctx.leapfrog(x, v, m, w.eps, th, w.n_crit, dt, 1, acc, pot)
        else:
            ctx.kick(v, acc, h)
            ctx.drift(x, v, dt)
            step(theta=th, shift=shift)
            ctx.kick(v, acc, h)
        if s % every == 0 or s == steps:
            st = ctx.get_stats()  # synchronises; counts the last force call
            k, u = energy(ctx, v, m, pot)
            log.append({"step": s, "kinetic": k, "potential": u, "total": k + u})
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = ctx.get_stats()
    etot = [r["total"] for r in log]
    out = {"workload": w.name, "n": n, "steps": steps, "dt": dt, "eps": w.eps, "n_crit": w.n_crit,
           "theta_mode": mode, "fallback_reason": reason, "theta": th, "shift": shift,
           "calibration_rms": calib_rms, "ms_per_step": ms, "particles_per_s": n / (ms * 1e-3),
           "interactions_last_step": st.interactions, "theta_fallback_groups": st.n_theta_fallback,
           "energy_drift": (etot[-1] - etot[0]) / abs(etot[0]),
           "max_energy_error": max(abs(e - etot[0]) for e in etot) / abs(etot[0]),
           "energy": log, "error_flags": st.error_flags,
           "note": f"step time includes the energy checkpoints every {every} steps"}
    ctx.close()
    return out


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
    out = run(args.workload, args.n, args.steps, args.dt, args.target_rms, args.theta, args.learned,
              args.theta_net, args.judge_sample, args.every)
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
    sys.exit(0)
