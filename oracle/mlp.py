"""FP64 reference of the per-group opening-angle network (test infrastructure only).

The paper fixes one opening angle for all particles and shows that it trades
accuracy for work (Sec. 3.5, the run-time and error study over theta in Table "theta").  The
learned part chooses theta per group instead: a multilayer perceptron maps 12
features of a group (`features`) to theta in [0.3, 1.0].  This module is the
plain FP64 definition the GPU kernels are checked against:

    z1 = W1 x' + b1,  h1 = tanh(z1)          x' = (x - mu) / sigma, 12 -> 64
    z2 = W2 h1 + b2,  h2 = tanh(z2)          64 -> 64
    y  = w3 . h2 + b3                        64 -> 1
    theta = 0.3 + 0.7 sigmoid(y + shift)

Training minimises the weighted mean squared error of theta against labels,
sum_b w_b (theta_b - t_b)^2 / sum_b w_b, with Adam (Kingma & Ba, 2015).

Parameters are one flat FP64 vector in the order W1 [64][12], b1 [64],
W2 [64][64], b2 [64], w3 [64], b3 [1] (5057 values).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID = 12, 64
THETA_MIN, THETA_SPAN = 0.3, 0.7
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("w3", (N_HID,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    """Views of the flat parameter vector: dict name -> array."""
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def init(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAMS)
    w = unpack(p)
    for name, fan_in, fan_out in (("W1", N_IN, N_HID), ("W2", N_HID, N_HID), ("w3", N_HID, 1)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        w[name][...] = rng.uniform(-lim, lim, w[name].shape)
    return p


def forward(p, x, mu, sigma, shift: float = 0.0):
    """theta [B] and the cache of activations for `backward`."""
    w = unpack(np.asarray(p, dtype=np.float64))
    xn = (np.asarray(x, dtype=np.float64) - mu) / sigma
    h1 = np.tanh(xn @ w["W1"].T + w["b1"])
    h2 = np.tanh(h1 @ w["W2"].T + w["b2"])
    y = h2 @ w["w3"] + w["b3"][0]
    sg = 1.0 / (1.0 + np.exp(-(y + shift)))
    theta = THETA_MIN + THETA_SPAN * sg
    return theta, {"xn": xn, "h1": h1, "h2": h2, "sg": sg}


def loss_and_grad(p, x, mu, sigma, target, weight):
    """Weighted MSE of theta and its gradient with respect to p (FP64)."""
    w = unpack(np.asarray(p, dtype=np.float64))
    theta, c = forward(p, x, mu, sigma)
    wt = np.asarray(weight, dtype=np.float64)
    W = wt.sum()
    r = theta - target
    loss = float(np.sum(wt * r * r) / W)
    dtheta = 2.0 * wt * r / W
    dy = dtheta * THETA_SPAN * c["sg"] * (1.0 - c["sg"])
    g = np.zeros(N_PARAMS)
    gw = unpack(g)
    gw["w3"][...] = c["h2"].T @ dy
    gw["b3"][0] = dy.sum()
    dz2 = np.outer(dy, w["w3"]) * (1.0 - c["h2"] ** 2)
    gw["W2"][...] = dz2.T @ c["h1"]
    gw["b2"][...] = dz2.sum(axis=0)
    dz1 = (dz2 @ w["W2"]) * (1.0 - c["h1"] ** 2)
    gw["W1"][...] = dz1.T @ c["xn"]
    gw["b1"][...] = dz1.sum(axis=0)
    return loss, g


class Adam:
    """Adam with bias correction: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, p, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        return p - self.lr * mh / (np.sqrt(vh) + self.eps)


def bf16(a):
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(p, x, mu, sigma, shift: float = 0.0):
    """The inference arithmetic of the GPU path written out in FP64: the
    normalised features, the weights of the two hidden layers and the first
    hidden activations are rounded to bfloat16 (the matrix-core operands),
    products and sums are then exact-in-FP64 stand-ins for the FP32
    accumulation; the output layer stays FP32/FP64."""
    w = unpack(np.asarray(p, dtype=np.float64))
    xn = bf16(((np.asarray(x, dtype=np.float32) - np.float32(mu)) / np.float32(sigma)))
    h1 = np.tanh(xn @ bf16(w["W1"]).T + w["b1"].astype(np.float32))
    h2 = np.tanh(bf16(h1) @ bf16(w["W2"]).T + w["b2"].astype(np.float32))
    y = h2 @ w["w3"].astype(np.float32) + np.float32(w["b3"][0])
    return THETA_MIN + THETA_SPAN / (1.0 + np.exp(-(y + shift)))
