"""Shared helpers of the GPU parity tests (imported by tests, not collected)."""
import numpy as np
import torch

import oracle

# Parity bar for FP32 forces against the FP64 oracle on the same lists:
# |a_gpu - a_oracle| per component <= TOL * |a_oracle| for at least 99.9% of
# particles, and <= TOL * max(|a_oracle|, A) for all, where A is the sum of the
# magnitudes of the individual terms (the bound of FP32 rounding when the
# resultant cancels).  Potentials (sums of same-sign terms) within TOL.
TOL = 1e-5


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def gpu_run(bh, pos, mass, eps, theta, n_crit, theta_group=None, ctx=None):
    c = ctx or bh.Context()
    c.build_tree(to_dev(pos), to_dev(mass))
    G = c.make_groups(n_crit)
    tg = None if theta_group is None else to_dev(theta_group, torch.float32)
    acc, pot = c.compute_forces(eps, theta, theta_group=tg)
    st = c.get_stats()
    return c, acc.cpu().numpy().astype(np.float64), pot.cpu().numpy().astype(np.float64), st, G


def check_forces(acc_g, pot_g, ref, tol=TOL, frac=0.999):
    acc_o, pot_o, aab = ref["acc"], ref["pot"], ref["acc_abs"]
    an = np.linalg.norm(acc_o, axis=1)
    err = np.abs(acc_g - acc_o).max(axis=1)
    zero = an == 0
    assert np.all(acc_g[zero] == 0.0), "exactly cancelling forces must come back as 0"
    nz = ~zero
    rel = err[nz] / an[nz]
    ok = (rel <= tol).mean() if nz.any() else 1.0
    assert ok >= frac, f"only {ok:.5f} of particles within {tol} (worst {rel.max():.3e})"
    bound = tol * np.maximum(an, aab)
    worst = np.max(err - bound)
    assert np.all(err <= bound), f"error above the conditioning bound by {worst:.3e}"
    prel = np.abs(pot_g - pot_o) / np.maximum(np.abs(pot_o), 1e-300)
    pz = pot_o == 0
    assert np.all(pot_g[pz] == 0.0)
    assert np.all(prel[~pz] <= tol), f"potential error {prel[~pz].max():.3e}"
    return {"rel_max": float(rel.max()) if nz.any() else 0.0,
            "rel_999": float(np.quantile(rel, 0.999)) if nz.any() else 0.0,
            "pot_rel_max": float(prel[~pz].max()) if (~pz).any() else 0.0}


def oracle_nonchain_nodes(tree):
    """Oracle nodes without single-child chain cells, keyed by (first, count, level)."""
    nd = tree.nodes()
    chain = (nd["kind"] == oracle.KIND_CELL) & (nd["nchild"] == 1)
    keep = ~chain
    out = {}
    for k in np.flatnonzero(keep):
        level = -1 if nd["kind"][k] == oracle.KIND_PARTICLE else int(nd["level"][k])
        geo = k
        if nd["kind"][k] == oracle.KIND_BUCKET and nd["parent"][k] >= 0 and chain[nd["parent"][k]]:
            # accepted as one cell iff the deepest chain cell above it is (level 20)
            geo = nd["parent"][k]
        out[(int(nd["first"][k]), int(nd["count"][k]), level)] = (
            int(nd["kind"][k]), float(nd["mass"][k]), tuple(float(v) for v in nd["com"][k]), float(nd["l"][geo]),
            float(nd["s"][geo]))
    # the members of a bucket are particle leaves (its children) on the GPU
    keys, perm = tree.sorted()
    spos = tree.pos[perm]
    smass = tree.mass[perm]
    for k in np.flatnonzero(nd["kind"] == oracle.KIND_BUCKET):
        for i in range(int(nd["first"][k]), int(nd["first"][k] + nd["count"][k])):
            out[(i, 1, -1)] = (oracle.KIND_PARTICLE, float(smass[i]), tuple(float(v) for v in spos[i]), 0.0, 0.0)
    return out


def gpu_nodes(ctx):
    ints, reals = ctx.export_nodes()
    ints = ints.cpu().numpy()
    reals = reals.cpu().numpy()
    out = {}
    for k in range(ints.shape[0]):
        level, kind, first, count = (int(v) for v in ints[k, :4])
        if kind == 3:  # empty system root
            continue
        if kind == 1:
            level = -1
        out[(first, count, level)] = (kind, float(reals[k, 0]), tuple(float(v) for v in reals[k, 1:4]),
                                      float(reals[k, 4]), float(reals[k, 5]))
    return out, ints, reals
