"""Oracle for the warm-start network: an MLP 12 -> 64 -> 64 -> 1 with GELU.

TEST INFRASTRUCTURE: CPU oracle, imported only by tests, the smoke check and
the benchmark's CPU-baseline leg.

The network maps node v's 12 inputs (oracle.features) to s_v, its estimate
of the remaining PageRank correction at a warm restart (oracle.restart).
Its defined arithmetic, which the device kernels follow:
  - parameters: W1 (64 x 12), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3;
    the weights W1, W2, w3 are BF16 values (round-to-nearest-even copies of
    FP32 master weights), the biases FP32;
  - every operand entering a matrix product (a layer's input activations and
    its weights) is a BF16 value; products and sums are exact up to the
    accumulation's own rounding; biases and GELU apply to the sums;
  - z1 = W1 bf(x) + b1, h1 = gelu(z1); z2 = W2 bf(h1) + b2, h2 = gelu(z2);
    s = w3 . h2 + b3 (the last layer takes h2 unrounded);
  - gelu(z) = z sigma(1.702 z), sigma the logistic function: the sigmoid form
    of GELU (Hendrycks & Gimpel), within 0.021 of z Phi(z) everywhere and one
    exponential and one reciprocal on the device;
  - loss: mean squared error over the batch; backward by the chain rule with
    the same BF16 rounding of the operands of each product (bf(dz2) with
    bf(h1) and W2; bf(dz1) with bf(x));
  - Adam (Kingma & Ba) on FP32 master parameters.
Here every sum is taken in float64, so the oracle differs from the device
only by accumulation order and FP32 rounding.  With `quantize=False` it is
the plain float64 network, which the finite-difference pins use.

Parameter vector order (also the device's): W1 row-major (out, in), b1, W2
row-major (out, in), b2, w3, b3: 768 + 64 + 4096 + 64 + 64 + 1 = 5057 values.
"""
from __future__ import annotations

import math

import numpy as np

NIN, NH = 12, 64
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("w3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
WEIGHTS = ("W1", "W2", "w3")


def bf16(a):
    """Round to the nearest BF16 value (ties to even) from the FP32 value of
    `a`: keep the top 16 bits of the float32 pattern after adding 0x7FFF plus
    the lowest kept bit."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


GELU_A = 1.702


def _sigma(u):
    """Logistic function 1 / (1 + exp(-u)), written through tanh so that it
    does not overflow."""
    return 0.5 * (1.0 + np.tanh(0.5 * np.asarray(u, dtype=np.float64)))


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return z * _sigma(GELU_A * z)


def gelu_grad(z):
    """d/dz z s(a z) = s + a z s (1 - s), s = sigma(a z)."""
    z = np.asarray(z, dtype=np.float64)
    s = _sigma(GELU_A * z)
    return s + GELU_A * z * s * (1.0 - s)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == NPARAM
    out, k = {}, 0
    for name, shape in SIZES:
        c = int(np.prod(shape))
        out[name] = theta[k:k + c].reshape(shape)
        k += c
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def weights_bf16(theta):
    """The parameters the network uses: BF16 weights, biases as given."""
    p = unpack(theta)
    return {k: (bf16(v) if k in WEIGHTS else np.array(v)) for k, v in p.items()}


def init_params(seed):
    """Uniform Glorot initialisation of the weights from numpy's default_rng(seed), zero biases.
    The tests' own copy of the recipe: the benchmark draws its starting
    parameters from the seeded inputs module, and a pin checks that both
    give the same values."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SIZES:
        if name.startswith("b"):
            p[name] = np.zeros(shape)
        else:
            fan_out, fan_in = (shape if len(shape) == 2 else (1, shape[0]))
            a = math.sqrt(6.0 / (fan_in + fan_out))
            p[name] = rng.uniform(-a, a, size=shape)
    return pack(p).astype(np.float32).astype(np.float64)


def forward(theta, X, quantize=True):
    """s (n,) and the intermediates, for features X (n, 12)."""
    p = weights_bf16(theta) if quantize else unpack(theta)
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    xq = q(X)
    z1 = xq @ p["W1"].T + p["b1"]
    h1 = gelu(z1)
    h1q = q(h1)
    z2 = h1q @ p["W2"].T + p["b2"]
    h2 = gelu(z2)
    s = h2 @ p["w3"] + p["b3"][0]
    return s, dict(p=p, xq=xq, z1=z1, h1q=h1q, z2=z2, h2=h2, q=q)


def loss(theta, X, t, quantize=True):
    s, _ = forward(theta, X, quantize)
    return float(np.mean((s - np.asarray(t, dtype=np.float64)) ** 2))


def grad(theta, X, t, quantize=True):
    """(loss, gradient vector in parameter order) of the mean squared error."""
    s, c = forward(theta, X, quantize)
    p, q = c["p"], c["q"]
    t = np.asarray(t, dtype=np.float64)
    nb = len(s)
    gs = 2.0 * (s - t) / nb
    g = {}
    g["w3"] = c["h2"].T @ gs
    g["b3"] = np.array([gs.sum()])
    dz2 = np.outer(gs, p["w3"]) * gelu_grad(c["z2"])
    dz2q = q(dz2)
    g["W2"] = dz2q.T @ c["h1q"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2q @ p["W2"]
    dz1 = dh1 * gelu_grad(c["z1"])
    dz1q = q(dz1)
    g["W1"] = dz1q.T @ c["xq"]
    g["b1"] = dz1.sum(axis=0)
    return float(np.mean((s - t) ** 2)), pack(g)


class Adam:
    """theta_t = theta_{t-1} - lr * mhat / (sqrt(vhat) + eps), with
    m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, mhat = m/(1-b1^t),
    vhat = v/(1-b2^t)."""

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
