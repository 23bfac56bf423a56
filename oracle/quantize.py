"""Reference quantisers for reduced-precision field storage -- TEST INFRASTRUCTURE ONLY.

Two storage forms of a float32 snapshot (not in the paper, which stores fields at
the precision of its input files; these are the reduced-precision forms whose error
is reported against the FP64 oracle):
  * bfloat16: the upper 16 bits of the float32 pattern after rounding to nearest,
    ties to even;
  * float16 with a power-of-two scale per (variable, level): s = 2^(e - 14) with
    e = ceil(log2 max|F_level|) (s = 1 for an all-zero level), stored value
    float16(F / s) (round to nearest even), read back as float16 * s.
Both return the values the storage represents, as float32 (exactly).
"""

from __future__ import annotations

import numpy as np


def bf16_round(F: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even) -> float32."""
    b = np.ascontiguousarray(F, np.float32).view(np.uint32).astype(np.uint64)
    nan = (b & 0x7F800000) == 0x7F800000
    nan &= (b & 0x007FFFFF) != 0
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) & 0xFFFF
    r = np.where(nan, (b >> 16) | 0x40, r)
    return (r.astype(np.uint32) << 16).view(np.float32).reshape(np.shape(F))


def f16_scale(level: np.ndarray) -> float:
    """Power-of-two scale of one level: 2^(ceil(log2 max|F|) - 14), or 1 for zeros."""
    m = float(np.max(np.abs(level))) if level.size else 0.0
    if not m > 0.0:
        return 1.0
    fr, e = np.frexp(np.float32(m))  # m = fr * 2^e, fr in [0.5, 1)
    c = int(e) - 1 if fr == 0.5 else int(e)
    return float(2.0 ** (c - 14))


def f16_scaled_round(F: np.ndarray) -> np.ndarray:
    """Per level (leading axis of a 3D array, or the whole 2D array): float16(F/s)*s."""
    F = np.asarray(F, np.float32)
    levels = F[None] if F.ndim == 2 else F
    out = np.empty_like(levels)
    for k in range(levels.shape[0]):
        s = np.float32(f16_scale(levels[k]))
        out[k] = (levels[k] / s).astype(np.float16).astype(np.float32) * s
    return out[0] if F.ndim == 2 else out
