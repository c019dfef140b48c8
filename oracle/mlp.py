"""FP64 reference of the learned acceptance criterion's network.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Network: 10 features -> 32 (ReLU) -> 32 (ReLU) -> 1, trained with Adam on
either the mean-squared error or, for a quantile q in (0, 1), the pinball
loss mean(max(q r, (q - 1) r)) with r = label - prediction, whose minimiser
is the q-quantile of the label (Koenker and Bassett, 1978).  Parameters are a
flat vector in the order W1 (32x10, row-major), b1 (32), W2 (32x32), b2 (32),
w3 (32), b3 (1): 1441 values.

Also the bf16 view used to check the GPU's MFMA inference: weights of the two
hidden layers and the layer inputs rounded to bf16 (round to nearest even),
everything accumulated in FP64, the output layer in full precision.
"""
from __future__ import annotations

import numpy as np

NF, NH = 10, 32
SIZES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("w3", (NH,)),
         ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def init(seed: int) -> np.ndarray:
    """He-uniform hidden layers, small output layer, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {
        "W1": rng.uniform(-1, 1, (NH, NF)) * np.sqrt(6.0 / NF),
        "b1": np.zeros(NH),
        "W2": rng.uniform(-1, 1, (NH, NH)) * np.sqrt(6.0 / NH),
        "b2": np.zeros(NH),
        "w3": rng.uniform(-1, 1, NH) * np.sqrt(6.0 / NH) * 0.1,
        "b3": np.zeros(1),
    }
    return pack(p)


def forward(theta, X):
    """Predictions for rows of X (n x 10), with the hidden activations."""
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    out = h2 @ p["w3"] + p["b3"][0]
    return out, (z1, h1, z2, h2)


def loss(theta, X, y, q=None) -> float:
    """Mean-squared error, or the pinball loss of quantile q."""
    out, _ = forward(theta, X)
    if q is None:
        return float(np.mean((out - y) ** 2))
    r = y - out
    return float(np.mean(np.maximum(q * r, (q - 1.0) * r)))


def grad(theta, X, y, q=None):
    """Analytic gradient of the loss (backpropagation); for the pinball loss
    the derivative in the prediction is 1 - q where it exceeds the label,
    else -q."""
    p = unpack(theta)
    out, (z1, h1, z2, h2) = forward(theta, X)
    n = X.shape[0]
    if q is None:
        d_out = 2.0 * (out - y) / n             # (n,)
    else:
        d_out = np.where(out > y, 1.0 - q, -q) / n
    g = {"w3": h2.T @ d_out, "b3": np.array([d_out.sum()])}
    d_h2 = np.outer(d_out, p["w3"]) * (z2 > 0)   # (n, 32)
    g["W2"] = d_h2.T @ h1
    g["b2"] = d_h2.sum(0)
    d_h1 = (d_h2 @ p["W2"]) * (z1 > 0)
    g["W1"] = d_h1.T @ X
    g["b1"] = d_h1.sum(0)
    return pack(g)


class Adam:
    """Adam (Kingma & Ba) with bias correction."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def bf16(x):
    """Round to bfloat16 (nearest even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def f16(x):
    """Round FP32 values to IEEE binary16 (numpy's conversion: nearest even,
    subnormals kept, overflow to infinity), returned as float64."""
    with np.errstate(over="ignore"):  # overflow to infinity is the format's rule
        return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


def forward_bf16(theta, X, rnd=None):
    """The network as the MFMA inference evaluates it: features, W1 (with b1)
    and W2 rounded to bf16 (or by ``rnd``, e.g. ``f16``), first hidden layer
    rounded the same way after ReLU, b2, w3, b3 and all accumulation in full
    precision."""
    rnd = bf16 if rnd is None else rnd
    p = unpack(theta)
    W1 = rnd(p["W1"])
    b1 = rnd(p["b1"])
    W2 = rnd(p["W2"])
    b2 = np.asarray(p["b2"], dtype=np.float32).astype(np.float64)
    w3 = np.asarray(p["w3"], dtype=np.float32).astype(np.float64)
    b3 = float(np.float32(p["b3"][0]))
    h1 = rnd(np.maximum(rnd(X) @ W1.T + b1, 0.0))
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ w3 + b3
