"""Pins of the oracle for the surrogate's feature assembly and residual check
(oracle/surrogate.py) against closed forms.

* A field linear in space and time is reproduced exactly by linear interpolation,
  so every patch value is the formula at that node and time, and U, V at the
  particle is the formula at the particle: the patch order (rows outer, columns
  inner, U then V), the time weight, the clamping at the border and the bilinear
  value are all fixed.
* The nearest node and the offset come from a brute-force nearest-node search;
  the cell widths from the axis itself, times M cos(lat) on a sphere.
* The residual check accepts a network displacement equal to the coarse one,
  rejects it just beyond the threshold, and rejects a coarse estimate that left the
  grid, an end point off the grid and an end point in a land cell.
"""

from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from oracle import surrogate as S

M = 1852.0 * 60.0


def _axis(rng, n, lo, hi):
    w = rng.uniform(0.5, 1.5, n - 1)
    x = np.concatenate([[0.0], np.cumsum(w)])
    return lo + (hi - lo) * x / x[-1]


def _linear_fs(spherical=False, periodic=False):
    rng = np.random.default_rng(4)
    X = _axis(rng, 12, 10.0, 40.0) if spherical else _axis(rng, 12, 0.0, 3e5)
    Y = _axis(rng, 9, -30.0, -5.0) if spherical else _axis(rng, 9, 0.0, 2e5)
    T = np.array([0.0, 86400.0, 2 * 86400.0])
    cu = np.array([0.3, 2e-3, -1e-3, 1e-6]) if spherical else np.array([0.3, 2e-6, -1e-6, 1e-6])
    cv = np.array([-0.1, -1e-3, 3e-3, -2e-6]) if spherical else np.array([-0.1, -1e-6, 3e-6, -2e-6])
    TT, YY, XX = np.meshgrid(T, Y, X, indexing="ij")

    def f(c, x, y, t):
        return c[0] + c[1] * x + c[2] * y + c[3] * t

    U, V = f(cu, XX, YY, TT), f(cv, XX, YY, TT)
    P = 3 * 86400.0 if periodic else 0.0
    fs = O.OracleFieldSet(X, Y, None, T, U, V, spherical=spherical, period=P)
    return fs, (lambda x, y, t: f(cu, x, y, t)), (lambda x, y, t: f(cv, x, y, t)), P


def _nearest(x, X):
    """Brute force: the node closest to x (clamped), the upper one on a tie."""
    xc = min(max(x, X[0]), X[-1])
    d = np.abs(X - xc)
    k = int(np.argmin(d - 1e-12 * (X >= xc) * (d == d.min())))
    return k, xc


@pytest.mark.parametrize("spherical", [False, True])
def test_features_of_a_linear_field(spherical):
    fs, fu, fv, _ = _linear_fs(spherical)
    X, Y = fs.lon, fs.lat
    rng = np.random.default_rng(8)
    n = 60
    xs = np.concatenate([rng.uniform(X[0], X[-1], n - 4), [X[0], X[-1], X[1], X[-2]]])
    ys = np.concatenate([rng.uniform(Y[0], Y[-1], n - 4), [Y[0], Y[-1], Y[-2], Y[1]]])
    t = 1.3 * 86400.0
    F = S.features(fs, xs, ys, t, 0.0, 2 * 86400.0)
    for r in range(n):
        x, y = xs[r], ys[r]
        i0, _ = _nearest(x, X)
        j0, _ = _nearest(y, Y)
        q = 4
        for dj in range(-2, 3):
            jj = min(max(j0 + dj, 0), Y.size - 1)
            for di in range(-2, 3):
                ii = min(max(i0 + di, 0), X.size - 1)
                assert F[r, q] == pytest.approx(fu(X[ii], Y[jj], t), abs=1e-13)
                assert F[r, q + 1] == pytest.approx(fv(X[ii], Y[jj], t), abs=1e-13)
                q += 2
        assert F[r, 56] == pytest.approx(fu(x, y, t), abs=1e-13)
        assert F[r, 57] == pytest.approx(fv(x, y, t), abs=1e-13)
        # offset from the nearest node in cell widths
        ci = min(max(np.searchsorted(X, x, side="right") - 1, 0), X.size - 2)
        cj = min(max(np.searchsorted(Y, y, side="right") - 1, 0), Y.size - 2)
        assert F[r, 54] == pytest.approx((x - X[i0]) / (X[ci + 1] - X[ci]), abs=1e-13)
        assert F[r, 55] == pytest.approx((y - Y[j0]) / (Y[cj + 1] - Y[cj]), abs=1e-13)
        hx, hy = X[ci + 1] - X[ci], Y[cj + 1] - Y[cj]
        if spherical:
            hx, hy = hx * M * np.cos(np.deg2rad(y)), hy * M
        assert F[r, 58] == pytest.approx(hx / 3e4, rel=1e-14)
        assert F[r, 59] == pytest.approx(hy / 3e4, rel=1e-14)
        assert F[r, 0] == x / 180.0 and F[r, 1] == y / 90.0
        ph = 2 * np.pi * 1.3 / 2.0
        assert F[r, 2] == pytest.approx(np.sin(ph), abs=1e-15)
        assert F[r, 3] == pytest.approx(np.cos(ph), abs=1e-15)
        assert (F[r, 60:] == 0).all()


def test_features_clamp_positions_outside_the_grid():
    fs, fu, fv, _ = _linear_fs()
    X, Y = fs.lon, fs.lat
    F = S.features(fs, [X[0] - 5e3, X[-1] + 5e3], [Y[-1] + 1e3, Y[0] - 1e3], 0.5 * 86400.0,
                   0.0, 2 * 86400.0)
    assert F[0, 56] == pytest.approx(fu(X[0], Y[-1], 0.5 * 86400.0), abs=1e-13)
    assert F[1, 57] == pytest.approx(fv(X[-1], Y[0], 0.5 * 86400.0), abs=1e-13)
    assert F[0, 54] == 0.0 and F[1, 54] == 0.0


def _check_case(fs, spherical):
    X, Y = fs.lon, fs.lat
    x0 = np.array([0.5 * (X[3] + X[4])] * 6)
    y0 = np.array([0.5 * (Y[3] + Y[4])] * 6)
    dx = np.array([0.4, 0.4, 0.4, 0.4, 0.4, 50.0]) * (X[4] - X[3])
    dy = np.array([-0.3, -0.3, -0.3, -0.3, -0.3, 0.0]) * (Y[4] - Y[3])
    xc, yc = x0 + dx, y0 + dy
    m = M * np.cos(np.deg2rad(y0)) if spherical else 1.0
    mm = M if spherical else 1.0
    ex, ey = dx * m, dy * mm  # the coarse displacement in metres
    Yn = np.stack([ex / S.OUT_SCALE, ey / S.OUT_SCALE], axis=1)
    thr = 40.0
    # 1: equal -> accept; 2: 41 m east -> reject; 3: 39 m east -> accept;
    # 4: the coarse run failed -> reject; 5: the same, status 0, accepted; 6: end off grid
    Yn[1, 0] += 41.0 / S.OUT_SCALE
    Yn[2, 0] += 39.0 / S.OUT_SCALE
    st = np.array([0, 0, 0, 1, 0, 0], np.uint8)
    return x0, y0, xc, yc, st, Yn, thr


@pytest.mark.parametrize("spherical", [False, True])
def test_residual_check_decisions(spherical):
    fs, _, _, _ = _linear_fs(spherical)
    x0, y0, xc, yc, st, Yn, thr = _check_case(fs, spherical)
    acc, x1, y1, r = S.check(fs, x0, y0, xc, yc, st, Yn, thr)
    assert list(acc) == [True, False, True, False, True, False]
    assert r[0] < 1e-9 and r[1] == pytest.approx(41.0, abs=1e-6)
    assert r[2] == pytest.approx(39.0, abs=1e-6)
    # accepted end points are the network's: here the coarse end point (to rounding)
    assert x1[0] == pytest.approx(xc[0], abs=1e-9 * abs(xc[0]))
    assert y1[0] == pytest.approx(yc[0], abs=1e-9 * max(abs(yc[0]), 1))
    # rejected ones keep the start
    assert x1[1] == x0[1] and y1[3] == y0[3] and x1[5] == x0[5]


def test_residual_check_rejects_an_end_point_in_a_land_cell():
    fs, _, _, _ = _linear_fs()
    X, Y = fs.lon, fs.lat
    land = np.zeros((Y.size, X.size), np.uint8)
    land[5:7, 6:8] = 1  # the cell (j=5, i=6) has four land corners
    fsl = O.OracleFieldSet(X, Y, None, fs.times, fs.U, fs.V, land=land)
    x0 = np.array([0.5 * (X[5] + X[6])])
    y0 = np.array([0.5 * (Y[5] + Y[6])])
    xe, ye = 0.5 * (X[6] + X[7]), y0[0]
    Yn = np.array([[(xe - x0[0]) / S.OUT_SCALE, 0.0]])
    acc, x1, _, _ = S.check(fsl, x0, y0, np.array([xe]), np.array([ye]),
                            np.zeros(1, np.uint8), Yn, 40.0)
    assert not acc[0] and x1[0] == x0[0]
    acc, _, _, _ = S.check(fs, x0, y0, np.array([xe]), np.array([ye]), np.zeros(1, np.uint8),
                           Yn, 40.0)
    assert acc[0]
