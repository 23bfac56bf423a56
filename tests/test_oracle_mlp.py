"""Pin of the FP64 MLP oracle: its backward pass against central differences."""

import numpy as np

from oracle import mlp as M


def test_gelu_closed_forms():
    assert M.gelu(0.0) == 0.0
    x = np.linspace(-6, 6, 101)
    # large |x|: identity / zero; derivative against central differences
    assert abs(M.gelu(8.0) - 8.0) < 1e-12 and abs(M.gelu(-8.0)) < 1e-12
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.allclose(M.gelu_grad(x), fd, rtol=1e-7, atol=1e-9)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(3)
    sizes = (64, 256, 256, 256, 256, 2)
    W, b = M.init_params(rng, sizes)
    for l in range(len(b)):
        b[l] = rng.standard_normal(b[l].shape) * 0.1
    X = rng.standard_normal((16, 64)) * 0.5
    T = rng.standard_normal((16, 2)) * 0.3
    y, cache = M.forward(W, b, X)
    dW, db = M.backward(W, b, cache, y, T)
    h = 1e-6
    for l in range(len(W)):
        for _ in range(12):
            i, j = rng.integers(0, W[l].shape[0]), rng.integers(0, W[l].shape[1])
            W[l][i, j] += h
            lp = M.loss(M.forward(W, b, X)[0], T)
            W[l][i, j] -= 2 * h
            lm = M.loss(M.forward(W, b, X)[0], T)
            W[l][i, j] += h
            fd = (lp - lm) / (2 * h)
            assert abs(fd - dW[l][i, j]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(dW[l]).max())
        j = rng.integers(0, b[l].shape[0])
        b[l][j] += h
        lp = M.loss(M.forward(W, b, X)[0], T)
        b[l][j] -= 2 * h
        lm = M.loss(M.forward(W, b, X)[0], T)
        b[l][j] += h
        fd = (lp - lm) / (2 * h)
        assert abs(fd - db[l][j]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(db[l]).max())


def test_adam_first_step_is_lr_times_sign():
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    M.adam_step(p, g, m, v, 1, lr=0.01)
    # first bias-corrected step is lr * g / (|g| + eps)
    assert np.allclose(p[0], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], atol=1e-6)
