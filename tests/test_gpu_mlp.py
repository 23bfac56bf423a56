"""The surrogate's BF16-MFMA forward, backward and Adam kernels against the FP64
oracle that mirrors the bfloat16 rounding points (only FP32 accumulation differs)."""

import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _net(seed=0):
    from paper_1707_05163_amd import Surrogate
    s = Surrogate(seed)
    rng = np.random.default_rng(seed + 1)
    layers = s.get_params()
    # nonzero biases so their gradients and the epilogue are exercised
    layers = [(W, (rng.standard_normal(b.shape) * 0.05).astype(np.float32)) for W, b in layers]
    s.set_params(layers)
    return s, [W.astype(np.float64) for W, _ in layers], [b.astype(np.float64) for _, b in layers]


def _batch(B, seed=5):
    rng = np.random.default_rng(seed)
    X = np.zeros((B, 64), np.float32)
    X[:, :54] = rng.standard_normal((B, 54)) * 0.5
    T = (rng.standard_normal((B, 2)) * 0.3).astype(np.float32)
    return X, T


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def test_init_statistics_and_roundtrip():
    s, W, b = _net(1)
    for (w, _), fan in zip(s.get_params(), (64, 256, 256, 256, 256)):
        assert abs(w.std() / np.sqrt(2.0 / fan) - 1) < 0.05


@pytest.mark.parametrize("B", [128, 384, 1000])
def test_forward_matches_mirror_oracle(B):
    s, W, b = _net()
    X, _ = _batch(B)
    y = s.forward(X)
    yo, _ = M.forward(W, b, X.astype(np.float64), mirror=True)
    assert _rel(y, yo) < 2e-3


def test_gradients_match_mirror_oracle():
    s, W, b = _net()
    X, T = _batch(512)
    g, loss = s.gradients(X, T)
    yo, cache = M.forward(W, b, X.astype(np.float64), mirror=True)
    dW, db = M.backward(W, b, cache, yo, T.astype(np.float64), mirror=True)
    assert loss == pytest.approx(M.loss(yo, T), rel=2e-3)
    for l in range(5):
        assert _rel(g[l][0], dW[l]) < 5e-3, l
        assert _rel(g[l][1], db[l]) < 5e-3, l


def test_adam_step_matches_oracle_update():
    s, W, b = _net()
    X, T = _batch(256)
    g, _ = s.gradients(X, T)
    before = s.get_params()
    s.train_step(X, T, lr=1e-3)
    after = s.get_params()
    for l in range(5):
        p = [before[l][0].astype(np.float64)]
        M.adam_step(p, [g[l][0].astype(np.float64)], [np.zeros_like(p[0])],
                    [np.zeros_like(p[0])], 1, lr=1e-3)
        assert np.abs(after[l][0] - p[0]).max() < 2e-5


def test_training_reduces_loss_on_a_fixed_batch():
    s, W, b = _net(7)
    X, T = _batch(1024, seed=11)
    losses = [s.train_step(X, T, lr=3e-3) for _ in range(60)]
    assert losses[-1] < 0.2 * losses[0]


def test_fused_inference_matches_layerwise_forward():
    """The inference kernel (all layers fused, activations in registers) against the
    training forward (layer-by-layer GEMMs) through the loss both report, on a
    batch spanning many 256-row tiles (several per block)."""
    s, W, b = _net()
    B = 100_096
    X, T = _batch(B)
    y = s.forward(X).astype(np.float64)
    loss_fused = 0.5 * np.mean(np.sum((y - T) ** 2, axis=1))
    _, loss_layerwise = s.gradients(X, T)
    assert abs(loss_fused - loss_layerwise) <= 2e-3 * loss_layerwise
    yo, _ = M.forward(W, b, X[:2048].astype(np.float64), mirror=True)
    assert _rel(y[:2048], yo) < 2e-3
