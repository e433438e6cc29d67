"""Learned per-group opening angle: labels, training and calibration.

The paper fixes one theta for all particles and measures how run time and
accuracy move with it (Sec. 3.5, Table "theta").  With groups the error a
given theta makes differs a lot from group to group: where the pull of the
surrounding mass nearly cancels, the relative force error is large and a
small theta is needed; elsewhere a large theta is accurate enough.  This
module trains the network of ``k_mlp.hip`` to pick theta per group:

1. *Labels.*  For a snapshot, a seeded sample of groups is evaluated at every
   theta of a ladder (0.3 ... 1.0) on the GPU, together with FP64 direct
   forces for their members.  Per group and theta this gives the cost
   c_g(theta) = list length x (walk weight + member-block passes), a model of
   the group's walk and force-sum time, and the error
   e_g(theta) = sum over members of |a - a_direct|^2 / |a_direct|^2.
   The theta per group that minimises total cost under a total error budget
   (RMS over the sampled particles equal to the target) follows from the
   Lagrangian min c_g(theta) + lambda e_g(theta), with each group's curves
   smoothed by power laws over the ladder and lambda bisected until the
   budget is met (`allocate`).
2. *Training.*  The network is fitted to these labels (weighted by member
   count) with the library's FP32 forward/backward and Adam kernels.
3. *Calibration.*  At use, a shift of the network's output is bisected until
   the RMS error on the judge sample meets the target, exactly as a fixed
   theta is bisected; fixed theta stays the fallback when no shift meets it.

All heavy work runs in the library's kernels; this file marshals arrays and
does the per-group bookkeeping on the host.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import bh

LADDER = np.round(np.arange(0.30, 1.0001, 0.05), 4)


@dataclass
class ThetaNet:
    params: torch.Tensor  # FP32 [5057] on the device
    mu: torch.Tensor      # FP32 [12]
    sigma: torch.Tensor   # FP32 [12]

    def save(self, path):
        np.savez(path, params=self.params.cpu().numpy(), mu=self.mu.cpu().numpy(), sigma=self.sigma.cpu().numpy())

    @staticmethod
    def load(path, device="cuda"):
        z = np.load(path, allow_pickle=False)
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)
        return ThetaNet(f(z["params"]), f(z["mu"]), f(z["sigma"]))


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


WALK_WEIGHT = 2.0  # walk time per list entry / force time per entry and lane pass (measured)


def group_passes(c: int, walk_weight: float = WALK_WEIGHT) -> float:
    """Time of a group per list entry, in force-kernel lane passes: the walk
    (walk_weight) plus one pass per member block of at most 64, divided by
    the lane partitions a small block uses (as the force kernel splits them)."""
    nb = (c + 63) // 64
    total = walk_weight
    for b in range(nb):
        m = c * (b + 1) // nb - c * b // nb
        R = 1
        while R < 64 and m * 2 * R <= 64:
            R *= 2
        total += 1.0 / R
    return total


def group_tables(ctx: bh.Context, dpos, dmass, eps: float, n_crit: int, n_sample: int, seed: int,
                 ladder=LADDER, walk_weight: float = WALK_WEIGHT):
    """Features, costs and errors of a seeded sample of groups over a theta ladder.

    Returns dict: feat [S,12], count [S], cost [S,K], err [S,K] (sum of squared
    relative errors of the members), ladder [K]."""
    ctx.build_tree(dpos, dmass)
    G = ctx.make_groups(n_crit)
    feat = ctx.group_features(eps, G).cpu().numpy()
    ints, _, _, _ = ctx.export_groups()
    ints = ints.cpu().numpy()
    _, perm = ctx.export_sorted()
    perm = perm.cpu().numpy().astype(np.int64)
    rng = np.random.default_rng(seed)
    S = min(n_sample, G)
    sel = np.sort(rng.choice(G, S, replace=False))
    first, count = ints[sel, 0].astype(np.int64), ints[sel, 1].astype(np.int64)
    members = np.concatenate([perm[f:f + c] for f, c in zip(first, count)])
    owner = np.repeat(np.arange(S), count)
    didx = _dev(members, torch.int64)
    a_dir, _ = ctx.direct_sampled(dpos, dmass, eps, didx)
    a_dir = a_dir.cpu().numpy()
    nd = np.linalg.norm(a_dir, axis=1)
    nd = np.where(nd > 0, nd, np.inf)
    passes = np.array([group_passes(int(c), walk_weight) for c in count])
    K = len(ladder)
    cost = np.zeros((S, K))
    err = np.zeros((S, K))
    amag = np.zeros((S, K))
    for k, th in enumerate(ladder):
        acc, _ = ctx.compute_forces(eps, float(th))
        a = acc[didx].double().cpu().numpy()
        rel2 = (np.linalg.norm(a - a_dir, axis=1) / nd) ** 2
        err[:, k] = np.bincount(owner, weights=rel2, minlength=S)
        amag[:, k] = np.bincount(owner, weights=np.linalg.norm(a, axis=1), minlength=S) / count
        _, _, ll, _ = ctx.export_groups(lists=True)
        ll = ll.cpu().numpy()[sel].astype(np.float64)
        cost[:, k] = ll * passes
    adir = np.bincount(owner, weights=np.linalg.norm(a_dir, axis=1), minlength=S) / count
    return {"feat": feat[sel], "count": count, "cost": cost, "err": err, "ladder": np.asarray(ladder),
            "amag": amag, "adir": adir}


def _interp(tables, theta):
    """Per-group cost and error at continuous theta, linear between ladder points."""
    lad = tables["ladder"]
    K = len(lad)
    x = np.clip((theta - lad[0]) / (lad[1] - lad[0]), 0.0, K - 1 - 1e-9)
    k = np.floor(x).astype(np.int64)
    f = x - k
    r = np.arange(len(theta))
    k1 = np.minimum(k + 1, K - 1)
    c = tables["cost"][r, k] * (1 - f) + tables["cost"][r, k1] * f
    e = tables["err"][r, k] * (1 - f) + tables["err"][r, k1] * f
    return c, e


def allocate(tables, target_rms: float):
    """Per-group theta minimising the total cost under the error budget
    sum err = target^2 * members.  Each group's curves are smoothed by a
    power law over the ladder, err ~ A theta^p and cost ~ C theta^-q (least
    squares in log space), whose Lagrangian optimum is
    theta = (q C / (lambda p A))^(1/(p+q)); lambda is bisected (log scale)
    until the interpolated tables meet the budget.  Returns (theta [S], lambda)."""
    lad = np.asarray(tables["ladder"], dtype=np.float64)
    lt = np.log(lad)
    A = np.stack([np.ones_like(lt), lt], axis=1)
    ce = np.linalg.lstsq(A, np.log(tables["err"] + 1e-30).T, rcond=None)[0]
    cc = np.linalg.lstsq(A, np.log(tables["cost"] + 1.0).T, rcond=None)[0]
    a, p = ce
    b, q = cc[0], -cc[1]
    p = np.maximum(p, 0.1)
    q = np.maximum(q, 0.1)
    budget = target_rms ** 2 * float(tables["count"].sum())

    def theta_of(log_lam):
        return np.clip(np.exp((np.log(q) + b - np.log(p) - log_lam - a) / (p + q)), lad[0], lad[-1])

    lo, hi = -60.0, 80.0  # natural log of lambda
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        _, e = _interp(tables, theta_of(mid))
        if e.sum() > budget:
            lo = mid
        else:
            hi = mid
    return theta_of(hi), float(np.exp(hi))


def _glorot(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = np.zeros(bh.MLP_PARAMS, dtype=np.float32)
    o = 0
    for fan_in, fan_out, has_bias in ((12, 64, True), (64, 64, True), (64, 1, True)):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        p[o:o + fan_in * fan_out] = rng.uniform(-lim, lim, fan_in * fan_out)
        o += fan_in * fan_out + fan_out
    return p


def train(ctx: bh.Context, feat, target, weight, steps: int = 3000, batch: int = 1024, lr: float = 2e-3,
          seed: int = 0, log=None) -> ThetaNet:
    """Fit the network to (feat, target) with per-row weights, on the GPU."""
    feat = np.asarray(feat, dtype=np.float64)
    mu = feat.mean(axis=0)
    sigma = feat.std(axis=0)
    sigma = np.where(sigma > 1e-6, sigma, 1.0)
    net = ThetaNet(_dev(_glorot(seed)), _dev(mu), _dev(sigma))
    m = torch.zeros_like(net.params)
    v = torch.zeros_like(net.params)
    X, T, W = _dev(feat), _dev(target), _dev(weight)
    n = X.shape[0]
    rng = np.random.default_rng(seed + 1)
    for step in range(1, steps + 1):
        idx = _dev(rng.choice(n, min(batch, n), replace=False), torch.int64)
        g, loss = ctx.mlp_grad(net.params, net.mu, net.sigma, X[idx].contiguous(), T[idx].contiguous(),
                               W[idx].contiguous())
        ctx.mlp_adam(net.params, g, m, v, step, lr)
        if log is not None and (step % 500 == 0 or step == 1):
            log(f"step {step}: loss {float(loss.cpu()[0]):.5f}")
    return net


def rms_error(acc, didx, a_dir, a_dir_norm) -> float:
    a = acc[didx].double().cpu().numpy()
    rel = np.linalg.norm(a - a_dir, axis=1) / a_dir_norm
    return float(math.sqrt(np.mean(rel * rel)))


def bisect(f, lo: float, hi: float, target: float, increasing: bool = True, rel_tol: float = 0.003,
           iters: int = 24):
    """x in [lo, hi] with f(x) within rel_tol of target (f monotone on
    average); returns (x, f(x)) of the closest evaluation."""
    best = None
    flo, fhi = f(lo), f(hi)
    for x, y in ((lo, flo), (hi, fhi)):
        if best is None or abs(y / target - 1) < abs(best[1] / target - 1):
            best = (x, y)
    if not increasing:
        lo, hi, flo, fhi = hi, lo, fhi, flo
    if fhi <= target:
        return hi, fhi
    if flo >= target:
        return lo, flo
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        y = f(mid)
        if abs(y / target - 1) < abs(best[1] / target - 1):
            best = (mid, y)
        if abs(y / target - 1) <= rel_tol:
            break
        if y > target:
            hi = mid
        else:
            lo = mid
    return best


DEFAULT_NET = os.path.join(os.path.dirname(os.path.abspath(__file__)), "theta_net.npz")


class Judge:
    """RMS relative force error on a seeded sample against FP64 direct summation
    (computed once per particle set by the library's FP64 kernel)."""

    def __init__(self, ctx: bh.Context, dpos, dmass, eps: float, sample: int, seed: int = 12345):
        n = dpos.shape[0]
        rng = np.random.default_rng(seed)
        s = min(sample, n)
        self.idx = np.sort(rng.choice(n, s, replace=False))
        self.didx = _dev(self.idx, torch.int64)
        a, _ = ctx.direct_sampled(dpos, dmass, eps, self.didx)
        self.a = a.cpu().numpy()
        self.norm = np.linalg.norm(self.a, axis=1)
        self.norm = np.where(self.norm > 0, self.norm, np.inf)

    def rms(self, acc) -> float:
        return rms_error(acc, self.didx, self.a, self.norm)


class Stepper:
    """One force evaluation with a fixed theta or with the network's theta."""

    def __init__(self, ctx: bh.Context, dpos, dmass, eps: float, n_crit: int, net: ThetaNet | None = None):
        self.ctx, self.dpos, self.dmass, self.eps, self.n_crit, self.net = ctx, dpos, dmass, eps, n_crit, net
        n = dpos.shape[0]
        self.acc = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        self.pot = torch.empty(n, dtype=torch.float32, device="cuda")
        self.theta_g = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")

    def __call__(self, theta: float = 0.6, shift: float = 0.0):
        c = self.ctx
        c.build_tree(self.dpos, self.dmass)
        c.make_groups(self.n_crit, sync=False)
        tg = None
        if self.net is not None:
            c.group_theta(self.net.params, self.net.mu, self.net.sigma, self.eps, shift, theta=self.theta_g)
            tg = self.theta_g
        c.compute_forces(self.eps, theta, theta_group=tg, acc=self.acc, pot=self.pot)


def timed_steps(stepper, steps: int, warmup: int, **kw):
    """Mean ms per step (HIP events on the current stream) and the stats."""
    for _ in range(warmup):
        stepper(**kw)
    torch.cuda.synchronize()
    stepper.ctx.get_stats()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        stepper(**kw)
    e1.record()
    torch.cuda.synchronize()
    st = stepper.ctx.get_stats()
    if st.error_flags:
        raise RuntimeError(f"device error flags {st.error_flags}")
    return e0.elapsed_time(e1) / steps, st


def equal_error(ctx: bh.Context, dpos, dmass, eps: float, n_crit: int, net: ThetaNet | None, target: float,
                judge: Judge, steps: int = 10, warmup: int = 2):
    """Fixed theta and (when net is given) learned theta, each calibrated to
    the target RMS error on the judge sample, then timed."""
    n = dpos.shape[0]
    out = {}
    fixed = Stepper(ctx, dpos, dmass, eps, n_crit)

    def err_fixed(th):
        fixed(theta=th)
        return judge.rms(fixed.acc)

    th, r = bisect(err_fixed, 0.3, 1.0, target)
    ms, st = timed_steps(fixed, steps, warmup, theta=th)
    out["fixed"] = {"theta": th, "rms": judge.rms(fixed.acc), "calibration_rms": r, "ms_per_step": ms,
                    "interactions": st.interactions, "interactions_per_s": st.interactions / (ms * 1e-3),
                    "particles_per_s": n / (ms * 1e-3)}
    if net is None:
        return out
    learned = Stepper(ctx, dpos, dmass, eps, n_crit, net)

    def err_learned(sh):
        learned(shift=sh)
        return judge.rms(learned.acc)

    sh, r = bisect(err_learned, -8.0, 8.0, target)
    fallback = abs(r / target - 1) > 0.03 and r > target
    ms, st = timed_steps(learned, steps, warmup, shift=sh)
    G = st.n_groups
    tg = learned.theta_g[:G].cpu().numpy()
    out["learned"] = {"shift": sh, "rms": judge.rms(learned.acc), "calibration_rms": r, "ms_per_step": ms,
                      "interactions": st.interactions, "interactions_per_s": st.interactions / (ms * 1e-3),
                      "particles_per_s": n / (ms * 1e-3), "theta_mean": float(tg.mean()),
                      "theta_min": float(tg.min()), "theta_max": float(tg.max()),
                      "fallback_to_fixed": bool(fallback)}
    out["gain"] = {"interactions_fixed_over_learned": out["fixed"]["interactions"] / st.interactions,
                   "particles_per_s_learned_over_fixed": out["learned"]["particles_per_s"] /
                   out["fixed"]["particles_per_s"]}
    return out


class Recorder:
    """Wraps a step and a judge: every evaluation records (parameter, judge
    RMS, interactions) so that a calibration can also be read at exactly the
    target error by interpolation between the evaluations that bracket it."""

    def __init__(self, step, judge, key: str):
        self.step, self.judge, self.key = step, judge, key
        self.history = []

    def __call__(self, x):
        self.step(**{self.key: x})
        r = self.judge.rms(self.step.acc)
        self.history.append((float(x), r, int(self.step.ctx.get_stats().interactions)))
        return r


def at_target(history, target: float):
    """Interactions at exactly the target RMS: log-linear interpolation
    between the closest evaluations below and above the target (None when
    the evaluations do not bracket it)."""
    below = [h for h in history if h[1] <= target]
    above = [h for h in history if h[1] > target]
    if not below or not above:
        return None
    b = max(below, key=lambda h: h[1])
    a = min(above, key=lambda h: h[1])
    if a[1] == b[1] or b[2] <= 0 or a[2] <= 0:
        return float(b[2])
    t = (math.log(target) - math.log(b[1])) / (math.log(a[1]) - math.log(b[1]))
    return float(math.exp(math.log(b[2]) + t * (math.log(a[2]) - math.log(b[2]))))


@dataclass
class Calibration:
    """Outcome of calibrating both modes to one RMS target on a judge sample."""
    mode: str                 # "learned", or "fixed" when the learned mode is not used
    theta: float              # fixed theta at the target (also the theta of NaN groups)
    shift: float | None       # network output shift at the target (learned mode)
    fixed_rms: float
    learned_rms: float | None
    reason: str               # why the fixed path was taken ("" for learned)
    fixed_history: list
    learned_history: list


def calibrate(ctx: bh.Context, dpos, dmass, eps: float, n_crit: int, net: ThetaNet | None, judge: Judge,
              target: float, theta_lo: float = 0.3, rel_tol: float = 0.003) -> Calibration:
    """Fixed theta, then the network's shift, bisected to the target RMS.
    The learned mode is taken only when the network gives a finite theta for
    every group and its calibrated error meets the target (within rel_tol);
    otherwise fixed theta is the fallback."""
    fixed = Stepper(ctx, dpos, dmass, eps, n_crit)
    fr = Recorder(fixed, judge, "theta")
    theta, r_fixed = bisect(fr, theta_lo, 1.0, target, rel_tol=rel_tol)
    base = dict(theta=theta, fixed_rms=r_fixed, fixed_history=fr.history)
    if net is None:
        return Calibration("fixed", shift=None, learned_rms=None, reason="no network", learned_history=[], **base)
    lstep = Stepper(ctx, dpos, dmass, eps, n_crit, net)
    lstep(theta=theta, shift=0.0)
    G = ctx.get_stats().n_groups
    if not bool(torch.isfinite(lstep.theta_g[:G]).all()):
        return Calibration("fixed", shift=None, learned_rms=None, reason="network output not finite",
                           learned_history=[], **base)
    lr = Recorder(_Fixed(lstep, theta), judge, "shift")
    sh, r = bisect(lr, -8.0, 8.0, target, rel_tol=rel_tol)
    if r > target * (1.0 + rel_tol):
        return Calibration("fixed", shift=sh, learned_rms=r, reason="the network misses the error target",
                           learned_history=lr.history, **base)
    return Calibration("learned", shift=sh, learned_rms=r, reason="", learned_history=lr.history, **base)


class _Fixed:
    """A learned Stepper called with its fallback theta held fixed."""

    def __init__(self, step: Stepper, theta: float):
        self.step, self.theta = step, theta
        self.ctx = step.ctx

    @property
    def acc(self):
        return self.step.acc

    def __call__(self, shift: float = 0.0):
        self.step(theta=self.theta, shift=shift)
