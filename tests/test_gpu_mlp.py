"""Learned per-group theta on the GPU against the FP64 oracle: features,
bfloat16 matrix-core inference, FP32 gradients and Adam, and forces with the
learned theta."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import check_forces, to_dev
from oracle import mlp
from oracle.features import all_features
from paper_0909_0541_amd import inputs
from test_oracle_features import _cluster

pytestmark = pytest.mark.gpu


def _f32(a):
    return to_dev(np.asarray(a, dtype=np.float32), torch.float32)


def _net(seed):
    p = mlp.init(seed) + np.random.default_rng(seed + 1).normal(size=mlp.N_PARAMS) * 0.05
    rng = np.random.default_rng(seed + 2)
    mu = rng.normal(size=12).astype(np.float32)
    sigma = rng.uniform(0.5, 3.0, 12).astype(np.float32)
    return p.astype(np.float32).astype(np.float64), mu, sigma


def _feature_cases():
    rng = np.random.default_rng(1)
    two = np.concatenate([_cluster([0, 0, 0], rng), _cluster([1, 1, 1], rng)])
    nested = np.concatenate([_cluster([0.02, 0.02, 0.02], rng), _cluster([0.095, 0.02, 0.02], rng),
                             _cluster([0.98, 0.98, 0.98], rng), _cluster([0.905, 0.98, 0.98], rng)])
    coinc = np.concatenate([np.zeros((6, 3)), np.ones((2, 3))])
    p8, m8, _ = inputs.plummer(8192, 1, with_vel=False)
    pc, mc = inputs.clustered(20000, 9, n_halos=40)[:2]
    return [("two_clusters", two, rng.uniform(0.5, 1.5, 8), 4, 1e-3),
            ("nested", nested, rng.uniform(0.5, 1.5, 16), 4, 1e-4),
            ("coincident", coinc, np.ones(8), 4, 0.1),
            ("plummer_8k", p8, m8, 64, 1 / 256),
            ("clustered_20k", pc, mc, 64, 1e-4),
            ("whole_system", p8[:50], m8[:50], 64, 1e-2)]


@pytest.mark.parametrize("case", _feature_cases(), ids=lambda c: c[0])
def test_features_match_oracle(gpu, case):
    bh = gpu
    name, pos, mass, n_crit, eps = case
    c = bh.Context()
    c.build_tree(to_dev(pos), to_dev(mass))
    G = c.make_groups(n_crit)
    f_gpu = c.group_features(eps, G).cpu().numpy().astype(np.float64)
    t = oracle.Tree(pos, mass)
    assert t.groups(n_crit) == G
    f_orc = all_features(t, eps)
    # FP64 on both sides, one FP32 rounding on the GPU (relative 2^-24)
    err = np.abs(f_gpu - f_orc)
    assert np.all(err <= 1e-6 * np.maximum(1.0, np.abs(f_orc))), (name, err.max())


def _bf16_bound(p, x, mu, sigma, lam=6.0):
    """Bound on |theta_bf16 - theta_fp64| per row, derived from the layer
    widths and the bfloat16 unit roundoff u_b = 2^-8 (8 significant bits).

    Layer 1 rounds both operands of each of its 12 products (x' and W1) to
    bfloat16, layer 2 both operands of its 64 products (h1 and W2); the
    products are accumulated in FP32 (unit roundoff 2^-24, at most n
    roundings for n terms).  Round-to-nearest errors are bounded by
    u_b |v| and, in the probabilistic model of rounding errors (Higham and
    Mary, SIAM J. Sci. Comput. 41, 2019), independent with mean zero, so by
    Hoeffding's inequality a sum of such errors exceeds lam times the root of
    the sum of their squared bounds with probability at most
    2 exp(-lam^2 / 2) (3e-8 for lam = 6).  The error is carried through tanh
    (Lipschitz 1; FP32 tanh within 4 ulps), the output layer (FP32) and the
    sigmoid (Lipschitz 1/4), scaled by the theta span 0.7."""
    w = mlp.unpack(np.asarray(p, dtype=np.float64))
    ub, u = 2.0 ** -8, 2.0 ** -24
    xn = (np.asarray(x, np.float64) - mu) / sigma
    W1, W2, w3 = w["W1"], w["W2"], w["w3"]
    e1 = ub * np.sqrt(2.0 * ((xn[:, None, :] * W1[None, :, :]) ** 2).sum(-1)) \
        + 13 * u * (np.abs(xn) @ np.abs(W1).T + np.abs(w["b1"]))
    h1 = np.tanh(xn @ W1.T + w["b1"])
    d1 = np.sqrt(e1 ** 2 + (ub * np.abs(h1)) ** 2) + 4 * u
    e2 = np.sqrt((d1 ** 2) @ (W2 ** 2).T + ub ** 2 * ((h1 ** 2) @ (W2 ** 2).T)) \
        + 65 * u * (np.abs(h1) @ np.abs(W2).T + np.abs(w["b2"]))
    h2 = np.tanh(h1 @ W2.T + w["b2"])
    d2 = e2 + 4 * u
    ey = np.sqrt((d2 ** 2) @ (w3 ** 2)) + 65 * u * (np.abs(h2) @ np.abs(w3) + abs(w["b3"][0]))
    return mlp.THETA_SPAN * (0.25 * lam * ey + 4 * u)


def _check_inference(th, p, x, mu, sigma, shift):
    """Acceptance: the plain FP64 network within the derived bfloat16 bound,
    and never more than 1e-2 in theta."""
    full, _ = mlp.forward(p, x, mu.astype(np.float64), sigma.astype(np.float64), shift)
    tol = np.minimum(_bf16_bound(p, x, mu.astype(np.float64), sigma.astype(np.float64)), 1e-2)
    err = np.abs(th - full)
    assert np.all(err <= tol), (err.max(), float(tol[np.argmax(err - tol)]))
    return err


@pytest.mark.parametrize("rows", [0, 1, 17, 1003, 4096])
def test_inference_matches_fp64_network(gpu, rows):
    bh = gpu
    p, mu, sigma = _net(3)
    x = np.random.default_rng(rows).normal(size=(rows, 12)).astype(np.float32) * 3.0
    c = bh.Context()
    th = c.mlp_infer(_f32(p), _f32(mu), _f32(sigma), _f32(x.reshape(rows, 12)), shift=0.25)
    th = th.cpu().numpy().astype(np.float64)
    if rows == 0:
        return
    _check_inference(th, p, x, mu, sigma, 0.25)
    # Diagnostic only (not the acceptance check): the same rounding points
    # written out in FP64 agree far more closely, which says the kernel rounds
    # where it is meant to.
    assert np.quantile(np.abs(th - mlp.forward_bf16(p, x, mu, sigma, 0.25)), 0.99) <= 1e-5


def test_trained_network_on_real_features_matches_fp64(gpu):
    """The shipped network on the features of a clustered box (computed by
    the oracle on the CPU), against the FP64 network."""
    bh = gpu
    from paper_0909_0541_amd import learned
    net = learned.ThetaNet.load(learned.DEFAULT_NET)
    p = net.params.cpu().numpy().astype(np.float64)
    mu, sigma = net.mu.cpu().numpy(), net.sigma.cpu().numpy()
    pos, mass = inputs.clustered(30000, 21, n_halos=40)[:2]
    t = oracle.Tree(pos, mass)
    t.groups(64)
    x = all_features(t, 1e-4).astype(np.float32)
    c = bh.Context()
    for shift in (-1.0, 0.0, 0.5):
        th = c.mlp_infer(net.params, net.mu, net.sigma, _f32(x), shift=shift).cpu().numpy().astype(np.float64)
        _check_inference(th, p, x, mu, sigma, shift)


@pytest.mark.parametrize("batch", [1, 333, 2048])
def test_gradient_matches_oracle(gpu, batch):
    bh = gpu
    p, mu, sigma = _net(5)
    rng = np.random.default_rng(batch)
    x = (rng.normal(size=(batch, 12)) * 2.0).astype(np.float32)
    t = rng.uniform(0.3, 1.0, batch).astype(np.float32)
    w = rng.uniform(0.5, 50.0, batch).astype(np.float32)
    c = bh.Context()
    g, loss = c.mlp_grad(_f32(p), _f32(mu), _f32(sigma), _f32(x), _f32(t), _f32(w))
    g = g.cpu().numpy().astype(np.float64)
    loss = float(loss.cpu().numpy()[0])
    l_ref, g_ref = mlp.loss_and_grad(p, x.astype(np.float64), mu.astype(np.float64), sigma.astype(np.float64),
                                     t.astype(np.float64), w.astype(np.float64))
    assert abs(loss - l_ref) <= 1e-5 * l_ref
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
    assert np.abs(g - g_ref).max() <= 1e-4 * np.abs(g_ref).max()


def test_adam_matches_oracle(gpu):
    bh = gpu
    n = mlp.N_PARAMS
    rng = np.random.default_rng(7)
    p0 = rng.normal(size=n).astype(np.float32)
    c = bh.Context()
    P, M, V = _f32(p0), torch.zeros(n, dtype=torch.float32, device="cuda"), torch.zeros(n, dtype=torch.float32,
                                                                                          device="cuda")
    opt = mlp.Adam(n, lr=1e-2)
    pr = p0.astype(np.float64)
    for step in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        c.mlp_adam(P, _f32(g), M, V, step, 1e-2)
        pr = opt.step(pr, g.astype(np.float64))
    assert np.abs(P.cpu().numpy() - pr).max() <= 1e-6 * max(1.0, np.abs(pr).max())


def test_training_on_gpu_fits_a_learnable_target(gpu):
    bh = gpu
    rng = np.random.default_rng(5)
    x = rng.normal(size=(512, 12))
    t = 0.3 + 0.7 / (1.0 + np.exp(-(1.5 * x[:, 0] - x[:, 1])))
    mu, sigma = x.mean(axis=0), x.std(axis=0)
    p = mlp.init(6)
    c = bh.Context()
    P = _f32(p)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    X, T, W, MU, SG = _f32(x), _f32(t), _f32(np.ones(512)), _f32(mu), _f32(sigma)
    _, l0 = c.mlp_grad(P, MU, SG, X, T, W)
    l0 = float(l0.cpu()[0])
    for step in range(1, 301):
        g, _ = c.mlp_grad(P, MU, SG, X, T, W)
        c.mlp_adam(P, g, M, V, step, 3e-3)
    _, l1 = c.mlp_grad(P, MU, SG, X, T, W)
    assert float(l1.cpu()[0]) < 0.05 * l0
    # the FP64 oracle trained the same way ends at a comparable loss
    opt = mlp.Adam(mlp.N_PARAMS, lr=3e-3)
    for _ in range(300):
        _, gr = mlp.loss_and_grad(p, x, mu, sigma, t, np.ones(512))
        p = opt.step(p, gr)
    l_ref, _ = mlp.loss_and_grad(p, x, mu, sigma, t, np.ones(512))
    assert float(l1.cpu()[0]) < 3.0 * l_ref + 1e-6


def test_group_theta_and_forces_with_learned_theta(gpu):
    bh = gpu
    pos, mass = inputs.clustered(20000, 12, n_halos=40)[:2]
    eps, n_crit = 1e-4, 64
    p, mu, sigma = _net(11)
    c = bh.Context()
    c.build_tree(to_dev(pos), to_dev(mass))
    G = c.make_groups(n_crit)
    P, MU, SG = _f32(p), _f32(mu), _f32(sigma)
    th = c.group_theta(P, MU, SG, eps, shift=-0.3)
    feat = c.group_features(eps, G)
    th2 = c.mlp_infer(P, MU, SG, feat.contiguous(), shift=-0.3)
    assert torch.equal(th[:G], th2)
    thv = th[:G].cpu().numpy().astype(np.float64)
    assert np.all((thv >= 0.3) & (thv <= 1.0)) and thv.std() > 0.01
    acc, pot = c.compute_forces(eps, 0.6, theta_group=th[:G].contiguous())
    assert c.get_stats().error_flags == 0
    t = oracle.Tree(pos, mass)
    t.groups(n_crit)
    ref = t.forces(eps, 0.6, theta_g=thv)
    check_forces(acc.cpu().numpy().astype(np.float64), pot.cpu().numpy().astype(np.float64), ref)


def test_walk_order_changes_no_result(gpu):
    """group_theta also orders the list walk (each eighth of the groups by
    predicted walk time, longest first); a new make_groups on the same tree
    drops that order, so the second walk takes the groups in Morton order.
    Both walks must build the same lists: the same forces bit for bit."""
    bh = gpu
    from paper_0909_0541_amd import learned
    net = learned.ThetaNet.load(learned.DEFAULT_NET)
    pos, mass = inputs.clustered(60000, 21, n_halos=50)[:2]
    eps, n_crit = 1e-4, 64
    c = bh.Context()
    c.build_tree(to_dev(pos), to_dev(mass))
    G = c.make_groups(n_crit)
    assert G >= 64
    th = c.group_theta(net.params, net.mu, net.sigma, eps)
    tg = th[:G].contiguous()
    acc1, pot1 = c.compute_forces(eps, 0.6, theta_group=tg)
    s1 = c.get_stats()
    assert s1.error_flags == 0
    assert c.make_groups(n_crit) == G
    acc2, pot2 = c.compute_forces(eps, 0.6, theta_group=tg)
    s2 = c.get_stats()
    assert s2.error_flags == 0
    assert s1.interactions == s2.interactions and s1.list_entries == s2.list_entries
    assert torch.equal(acc1, acc2) and torch.equal(pot1, pot2)


def test_walk_order_in_batched_split_walks(gpu):
    """The same with several systems and split walks: with a fixed visit cap
    both walks split the same groups into the same keyed segments, so the
    ordered walk's forces equal the Morton-order walk's bit for bit."""
    bh = gpu
    from paper_0909_0541_amd import learned
    net = learned.ThetaNet.load(learned.DEFAULT_NET)
    sizes = [30000, 5000, 1, 20000, 12000]
    parts = [inputs.clustered(k, 40 + i, n_halos=max(1, k // 1000))[:2] for i, k in enumerate(sizes)]
    pos = np.concatenate([p for p, _ in parts])
    mass = np.concatenate([m for _, m in parts])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    eps = [1e-4] * len(sizes)
    c = bh.Context(split_visits=256)
    c.build_batch(off, to_dev(pos), to_dev(mass))
    G = c.make_groups(32)
    th = c.group_theta(net.params, net.mu, net.sigma, eps)
    tg = th[:G].contiguous()
    acc1, pot1 = c.compute_forces_batch(eps, [0.6] * len(sizes), theta_group=tg)
    s1 = c.get_stats()
    assert s1.error_flags == 0 and s1.n_split_groups > 0
    assert c.make_groups(32) == G
    acc2, pot2 = c.compute_forces_batch(eps, [0.6] * len(sizes), theta_group=tg)
    s2 = c.get_stats()
    assert s2.error_flags == 0 and s2.n_split_groups == s1.n_split_groups
    assert s1.interactions == s2.interactions
    assert torch.equal(acc1, acc2) and torch.equal(pot1, pot2)
