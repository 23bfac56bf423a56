"""Pins of the reference quantisers against their definitions and library routines."""

import numpy as np
import torch

from oracle import quantize as Q


def test_bf16_round_to_nearest_even_known_values():
    one = np.float32(1.0)
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -2.5 - 2 ** -9,
                     3.0e38, 1e-40, 0.0, -0.0], np.float32)
    exp = np.array([1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -2.5, None, None, 0.0, -0.0],
                   dtype=object)
    got = Q.bf16_round(vals)
    for g, e in zip(got[:6], exp[:6]):
        if e is not None:
            assert g == np.float32(e)
    assert one == Q.bf16_round(np.array([one]))[0]


def test_bf16_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(100000).astype(np.float32) * 10,
                        (rng.integers(0, 2 ** 16, 20000).astype(np.uint32) << 16 | 0x8000)
                        .view(np.float32)])  # exact ties
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(Q.bf16_round(x), ref)


def test_f16_scale_power_of_two_and_bound():
    rng = np.random.default_rng(1)
    for m in (1.0, 3.0, 0.75, 1e-4, 2.0 ** -20, 123.456):
        lev = rng.uniform(-m, m, (40, 50)).astype(np.float32)
        lev[3, 7] = np.float32(m)
        s = Q.f16_scale(lev)
        assert np.log2(s) == int(np.log2(s))
        assert np.abs(lev / s).max() <= 2 ** 14
        assert np.abs(lev / s).max() > 2 ** 13
    assert Q.f16_scale(np.zeros((3, 3), np.float32)) == 1.0
    assert Q.f16_scale(np.array([[1.0]], np.float32)) == 2.0 ** -14
    assert Q.f16_scale(np.array([[1.5]], np.float32)) == 2.0 ** -13


def test_f16_scaled_relative_error_bound():
    rng = np.random.default_rng(2)
    F = (rng.standard_normal((5, 30, 40)) * np.logspace(-4, 0, 5)[:, None, None]).astype(np.float32)
    G = Q.f16_scaled_round(F)
    for k in range(5):
        s = Q.f16_scale(F[k])
        # float16 has 11 significant bits: error <= half an ulp of |F/s| <= 2^14 -> s * 2^3
        assert np.abs(G[k] - F[k]).max() <= s * 2 ** 3
        # the scale keeps values out of the float16 subnormal range at the level's top
        ref = (F[k] / np.float32(s)).astype(np.float16).astype(np.float32) * np.float32(s)
        assert np.array_equal(G[k], ref)
