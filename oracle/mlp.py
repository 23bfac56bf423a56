"""Reference MLP for the learned flow-map surrogate -- TEST INFRASTRUCTURE ONLY.

The surrogate (not in the paper; it is a learned stand-in for a fixed number of
RK4 steps of the method of Sect. 2.1.1) is a fully connected network
    64 inputs -> 256 -> 256 -> 256 -> 256 -> 2 outputs,
with the tanh form of GELU (Hendrycks & Gimpel, 2016),
    g(x) = 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))),
after each hidden layer and a linear output.  Loss: L = (1 / 2B) sum (y - t)^2 over
the batch and the two outputs.  Optimiser: Adam (Kingma & Ba, 2015).

Two forward/backward modes:
  * exact: everything in float64 (checked against central differences);
  * mirror: float64 arithmetic, but values rounded to bfloat16 exactly where the GPU
    stores them in bfloat16 (weights, inputs, hidden activations and the
    pre-activation gradients fed to the products), so that the GPU, which only
    differs by accumulating in float32, can be compared closely.
Parameters: W[l] has shape (fan_in, fan_out), b[l] has shape (fan_out,).
"""

from __future__ import annotations

import numpy as np

from .quantize import bf16_round

SIZES = (64, 256, 256, 256, 256, 2)
C0 = np.sqrt(2.0 / np.pi)
C1 = 0.044715


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(C0 * (x + C1 * x ** 3)))


def gelu_grad(x):
    u = C0 * (x + C1 * x ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * C0 * (1.0 + 3.0 * C1 * x * x)


def init_params(rng: np.random.Generator, sizes=SIZES):
    """He-style normal init (std sqrt(2 / fan_in)), zero biases."""
    W, b = [], []
    for i in range(len(sizes) - 1):
        W.append(rng.standard_normal((sizes[i], sizes[i + 1])) * np.sqrt(2.0 / sizes[i]))
        b.append(np.zeros(sizes[i + 1]))
    return W, b


def _q(a, mirror):
    return bf16_round(np.asarray(a, np.float32)).astype(np.float64) if mirror else a


def forward(W, b, x, mirror=False):
    """Returns the output and the cache (inputs of each layer, pre-activations)."""
    h = _q(x, mirror)
    hs, zs = [h], []
    L = len(W)
    for l in range(L):
        z = h @ _q(W[l], mirror) + b[l]
        zs.append(z)
        if l < L - 1:
            h = _q(gelu(z), mirror)
            hs.append(h)
        else:
            h = z
    return h, (hs, zs)


def loss(y, t):
    return 0.5 * np.sum((y - t) ** 2) / y.shape[0]


def backward(W, b, cache, y, t, mirror=False):
    """Gradients of the loss with respect to every W[l] and b[l]."""
    hs, zs = cache
    B = y.shape[0]
    L = len(W)
    dW = [None] * L
    db = [None] * L
    dz = (y - t) / B
    for l in range(L - 1, -1, -1):
        dzq = _q(dz, mirror)
        dW[l] = hs[l].T @ dzq
        db[l] = dz.sum(axis=0)
        if l > 0:
            dh = dzq @ _q(W[l], mirror).T
            dz = dh * gelu_grad(zs[l - 1])
    return dW, db


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1) of lists of arrays, in place."""
    for p, g, mm, vv in zip(params, grads, m, v):
        mm *= b1
        mm += (1 - b1) * g
        vv *= b2
        vv += (1 - b2) * g * g
        mh = mm / (1 - b1 ** t)
        vh = vv / (1 - b2 ** t)
        p -= lr * mh / (np.sqrt(vh) + eps)
