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


def _ulp_bf16(v):
    a = np.abs(v)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    return np.where(a > 0, np.exp2(e - 7), 0.0)


def _output_bound(W, b, X):
    """Per output element: how far the GPU's output may lie from the bf16-mirror
    oracle's.  Two sources, to first order through the network's Jacobian
    dy/dz (pre-activations) and dy/dh (bf16 activations), from the mirror forward:
      * FP32 arithmetic: each pre-activation of fan-in K accumulates K bf16 products
        (exact in FP32) plus the bias, so it errs by at most (K + 2) 2^-24 sum|h w|;
        the GELU of the fused kernel (hardware exp2 and reciprocal) by 2^-20 |h|;
      * bfloat16 flips: an activation whose FP32 value sits at a rounding boundary can
        round to the neighbouring bf16 value on one side only, one ulp; the bound
        allows three such flips per row, each as large as the largest single one."""
    yo, (hs, zs) = M.forward(W, b, X, mirror=True)
    Wq = [M._q(w, True) for w in W]
    B = X.shape[0]
    out = np.zeros((B, 2))
    for i in range(2):
        acc = (256 + 2) * 2.0 ** -24 * (np.abs(hs[4]) @ np.abs(Wq[4]))[:, i]
        gz = np.zeros((B, 2))
        gz[:, i] = 1.0
        flip = np.zeros(B)
        for l in range(4, 0, -1):
            gh = gz @ Wq[l].T                       # dy_i / dh^l
            flip = np.maximum(flip, np.max(np.abs(gh) * _ulp_bf16(hs[l]), axis=1))
            acc += np.sum(np.abs(gh) * 2.0 ** -20 * np.abs(hs[l]), axis=1)
            gz = gh * M.gelu_grad(zs[l - 1])        # dy_i / dz^(l-1)
            K = Wq[l - 1].shape[0]
            acc += np.sum(np.abs(gz) * (K + 2) * 2.0 ** -24
                          * (np.abs(hs[l - 1]) @ np.abs(Wq[l - 1])), axis=1)
        out[:, i] = acc + 3.0 * flip
    return yo, out


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
    # element by element, within the bound derived in _output_bound
    yb, bound = _output_bound(W, b, X.astype(np.float64))
    err = np.abs(y.astype(np.float64) - yb)
    assert (err <= bound).all(), (float((err / bound).max()), np.argwhere(err > bound)[:5])


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
    # element by element: dW[l][a, c] = sum_n h[n, a] dzq[n, c] and db = sum_n dz[n, c];
    # each product's two bf16 factors may each sit one rounding flip (2^-7 relative)
    # away on the GPU, which bounds every term by 2^-6 of its size (FP32 accumulation
    # over 512 rows, 3e-5, is inside that)
    hs, _ = cache
    dz = (yo - T.astype(np.float64)) / X.shape[0]
    for l in range(4, -1, -1):
        dzq = M._q(dz, True)
        termsW = np.abs(hs[l]).T @ np.abs(dzq)
        assert (np.abs(g[l][0] - dW[l]) <= 2.0 ** -6 * termsW + 1e-30).all(), l
        assert (np.abs(g[l][1] - db[l]) <= 2.0 ** -6 * np.abs(dz).sum(axis=0) + 1e-30).all(), l
        if l > 0:
            dz = (dzq @ M._q(W[l], True).T) * M.gelu_grad(cache[1][l - 1])


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
