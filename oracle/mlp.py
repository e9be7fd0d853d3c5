"""FP64 reference of the learned proposal's network (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The network maps the 64 features of a candidate pair
site to one logit s: three hidden layers of 128 units with the GELU of
Hendrycks & Gimpel (2016) in its tanh form, then a linear output.

Parameter vector theta (41,473 values) in this order:
    W1[64][128], b1[128], W2[128][128], b2[128], W3[128][128], b3[128],
    w4[128], b4
(W[i][o] multiplies input i into output o).  Training fits s with a
mean-squared loss and Adam; the benchmark's target for a pilot insertion is
its clipped log ratio clip(beta mu + I - beta dH, -100, 10) at the operating
beta mu, I = 2 ln(V / (N + 1)).
"""
from __future__ import annotations

import math

import numpy as np

SHAPES = [(64, 128), (128, 128), (128, 128), (128, 1)]
N_PARAMS = sum(i * o + o for i, o in SHAPES)
GELU_C = math.sqrt(2.0 / math.pi)


def unpack(theta):
    """Views (W, b) of each layer."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, q = [], 0
    for i, o in SHAPES:
        W = theta[q:q + i * o].reshape(i, o)
        q += i * o
        b = theta[q:q + o]
        q += o
        out.append((W, b))
    return out


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(GELU_C * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    t = np.tanh(GELU_C * (x + 0.044715 * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * 0.044715 * x * x)


def forward(theta, X, keep=False):
    """Logits of the rows of X (n x 64)."""
    layers = unpack(theta)
    a = np.asarray(X, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        z = a @ W + b
        cache.append((a, z))
        a = gelu(z) if li < len(layers) - 1 else z
    s = a[:, 0]
    return (s, cache) if keep else s


def loss_and_grad(theta, X, t):
    """Mean-squared loss of the logits against targets t and its gradient
    with respect to theta (backpropagation through the four layers)."""
    s, cache = forward(theta, X, keep=True)
    t = np.asarray(t, dtype=np.float64)
    n = len(t)
    r = s - t
    loss = float(np.mean(r * r))
    layers = unpack(theta)
    grads = [None] * len(layers)
    delta = (2.0 / n) * r[:, None]                    # dL/dz of the output layer
    for li in range(len(layers) - 1, -1, -1):
        a, z = cache[li]
        W, _ = layers[li]
        grads[li] = (a.T @ delta, delta.sum(axis=0))
        if li > 0:
            _, zp = cache[li - 1]
            delta = (delta @ W.T) * gelu_grad(zp)
    g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, g


def adam_step(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One Adam update (Kingma & Ba 2015) with bias correction and decoupled
    weight decay wd (Loshchilov & Hutter 2019); step counts from 1.  Returns
    the new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * (mh / (np.sqrt(vh) + eps) + wd * theta), m, v


def target_of(dH, kT):
    """Training target of a pilot insertion: -beta dH clipped to [-50, 10]."""
    return np.clip(-np.asarray(dH, dtype=np.float64) / kT, -50.0, 10.0)


def random_theta(seed: int, scale: float = 1.0):
    """Seeded Glorot-uniform weights and zero biases (an input generator for
    tests: any weights are valid for the exactness of the proposal)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in SHAPES:
        a = scale * math.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-a, a, size=i * o))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def standardization(X):
    """Per-column mean and standard deviation of the data (columns with
    deviation below 1e-6 keep a scale of 1)."""
    X = np.asarray(X, dtype=np.float64)
    mean = X.mean(axis=0)
    sd = X.std(axis=0)
    sd[~(sd > 1e-6)] = 1.0
    return mean, sd


def to_standard(theta, mean, sd):
    """The same network in standardized input coordinates x' = (x - mean) / sd:
    W1' = sd W1 (row-wise), b1' = b1 + mean W1."""
    th = np.array(theta, dtype=np.float64)
    W1 = th[:64 * 128].reshape(64, 128)
    b1 = th[64 * 128:64 * 128 + 128]
    b1 += mean @ W1
    W1 *= sd[:, None]
    return th


def from_standard(theta, mean, sd):
    """Inverse of to_standard: W1 = W1' / sd, b1 = b1' - (mean / sd) W1'."""
    th = np.array(theta, dtype=np.float64)
    W1 = th[:64 * 128].reshape(64, 128)
    b1 = th[64 * 128:64 * 128 + 128]
    b1 -= (mean / sd) @ W1
    W1 /= sd[:, None]
    return th
