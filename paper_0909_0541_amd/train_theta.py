"""Train the per-group theta network on seeded clustered snapshots (GPU).

    python -m paper_0909_0541_amd.train_theta --out paper_0909_0541_amd/theta_net.npz

Labels come from the snapshots' own tree-versus-direct errors over a theta
ladder (see learned.py); the evaluation snapshots (clustered boxes of 2 and 4
million particles, seeds 2 and 4) are never used for training.  Prints one
JSON line per stage and a final summary with the equal-error comparison.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import bh, inputs, learned


def log(msg):
    print(msg, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=learned.DEFAULT_NET)
    ap.add_argument("--target-rms", type=float, default=1e-3)
    ap.add_argument("--snapshots", default="4194304:2048:101,4194304:2048:102,4194304:2048:103,"
                                           "4194304:2048:104,2097152:512:201,2097152:512:202,"
                                           "2097152:512:203,1048576:256:301",
                    help="comma-separated N:halos:seed")
    ap.add_argument("--groups-per-snapshot", type=int, default=1500)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--labels-only", action="store_true")
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--n-crit", type=int, default=256)
    ap.add_argument("--eval", default="clustered_2m,clustered_4m")
    ap.add_argument("--judge-sample", type=int, default=4096)
    ap.add_argument("--save-tables", default=None, help="write the label tables to this .npz")
    ap.add_argument("--walk-weight", type=float, default=learned.WALK_WEIGHT,
                    help="walk time per list entry in force-sum lane passes (the label cost model)")
    ap.add_argument("--baseline-net", default=None,
                    help="also evaluate this network on the same workloads, for comparison")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    ctx = bh.Context()
    tables = []
    t0 = time.time()
    for spec in args.snapshots.split(","):
        n, halos, seed = (int(v) for v in spec.split(":"))
        pos, mass, _ = inputs.clustered(n, seed, n_halos=halos)
        dpos, dmass = learned._dev(pos, torch.float64), learned._dev(mass, torch.float64)
        tb = learned.group_tables(ctx, dpos, dmass, args.eps, args.n_crit, args.groups_per_snapshot, seed,
                                  walk_weight=args.walk_weight)
        tables.append(tb)
        log(json.dumps({"stage": "labels", "snapshot": spec, "groups": int(len(tb["count"])),
                        "seconds": round(time.time() - t0, 1)}))
        del dpos, dmass
    pooled = {k: np.concatenate([t[k] for t in tables]) for k in ("feat", "count", "cost", "err")}
    pooled["ladder"] = tables[0]["ladder"]
    if args.save_tables:
        np.savez(args.save_tables, **{f"{k}_{i}": v for i, tb in enumerate(tables) for k, v in tb.items()})
    theta_lab, lam = learned.allocate(pooled, args.target_rms)
    # what the labels would save on the training groups if predicted exactly
    lab_cost, lab_err = learned._interp(pooled, theta_lab)
    budget = args.target_rms ** 2 * pooled["count"].sum()
    lo, hi = float(pooled["ladder"][0]), float(pooled["ladder"][-1])
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if learned._interp(pooled, np.full(len(theta_lab), mid))[1].sum() > budget:
            hi = mid
        else:
            lo = mid
    fix_cost = learned._interp(pooled, np.full(len(theta_lab), lo))[0].sum()
    log(json.dumps({"stage": "allocation", "lambda": lam, "theta_label_mean": float(theta_lab.mean()),
                    "label_gain_on_training_groups": float(fix_cost / lab_cost.sum()),
                    "fixed_theta_meeting_budget": lo}))
    if args.labels_only:
        return {}
    net = learned.train(ctx, pooled["feat"], theta_lab, pooled["count"].astype(np.float64), steps=args.steps,
                        batch=args.batch, lr=args.lr, log=lambda m: log(json.dumps({"stage": "train", "msg": m})))
    net.save(args.out)
    log(json.dumps({"stage": "saved", "path": args.out}))
    summary = {}
    for name in [s for s in args.eval.split(",") if s]:
        pos, mass, _, w = inputs.make_workload(name)
        dpos, dmass = learned._dev(pos, torch.float64), learned._dev(mass, torch.float64)
        judge = learned.Judge(ctx, dpos, dmass, w.eps, args.judge_sample)
        res = learned.equal_error(ctx, dpos, dmass, w.eps, w.n_crit, net, args.target_rms, judge)
        summary[name] = res
        log(json.dumps({"stage": "eval", "workload": name, **res}))
        if args.baseline_net:
            base = learned.ThetaNet.load(args.baseline_net)
            rb = learned.equal_error(ctx, dpos, dmass, w.eps, w.n_crit, base, args.target_rms, judge)
            log(json.dumps({"stage": "eval_baseline", "workload": name, **rb}))
        del dpos, dmass
    return summary


if __name__ == "__main__":
    main()
    sys.exit(0)
