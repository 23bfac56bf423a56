"""Reference for the two steps around the learned flow-map surrogate -- TEST
INFRASTRUCTURE ONLY (the tests import it; the product library never does).

The surrogate is not in the paper: it is a learned stand-in for a fixed number of
RK4 steps of the method (Sect. 2.1.1, Eq. 1), with plain RK4 as the fallback and
the arbiter.  This module restates, in FP64 with numpy, what its two steps around the
network compute, from their definitions:

features(fs, x, y, t) -- the network's 64 input values per position (before the
  network's bfloat16 rounding):
    [0..3]   lon / 180, lat / 90, sin(phi), cos(phi) with phi = 2 pi (t - T0) / P
             (T0 the first snapshot time; P the period, or the snapshot span);
    [4..53]  U, V (m/s) at the 5 x 5 nodes around the nearest node (rows j0 - 2 ..
             j0 + 2 outer, columns i0 - 2 .. i0 + 2 inner, U then V), indices clamped
             to the grid, each linear in time between the bracketing snapshots
             (the oracle's time bracket, O3);
    [54..55] the position's offset from the nearest node in cell widths;
    [56..57] U, V bilinear at the position (O2) and linear in time;
    [58..59] the cell's width and height in metres over 30 km (width at the
             position's latitude on a sphere);
    [60..63] zero.
  The nearest node on an axis is the lower node of the position's cell (the cell
  search O1, with positions clamped to the axis) when the cell fraction is below
  one half, else the upper one.

check(...) -- the residual check of the inference: the network's displacement
  (Y times 7200 m) is accepted when the coarse RK4 estimate (two steps over the
  segment) stayed in the grid, the distance between the two displacements in
  metres (the coarse one converted with the metric at the start latitude on a
  sphere, M = 1852 * 60 m per degree) is at most the threshold, and the end point
  lies in the grid and not in a land cell (four land corners); otherwise the
  particle keeps its start and is re-integrated with fine RK4.
"""

from __future__ import annotations

import numpy as np

from . import oracle as O

M = 1852.0 * 60.0
D = np.pi / 180.0
OUT_SCALE = 7200.0  # metres per unit of network output: 1 m/s over 2 h


def _cell(x, X):
    """Cell index and fraction of x clamped into [X0, X(n-1)] (the O1 rule)."""
    xc = min(max(x, X[0]), X[-1])
    i, f = O.locate(xc, X)
    return i, f


def features(fs: O.OracleFieldSet, x, y, t, t_first, period):
    """Rows [n x 64] of the network's input in FP64 (see the module docstring).
    `fs` is a 2D OracleFieldSet (U, V [nt, ny, nx]); `t_first` and `period` give the
    phase."""
    X, Y = fs.lon, fs.lat
    nx, ny = X.size, Y.size
    rc, s0, s1, tau = fs.time_bracket(t)
    assert rc == 0, "time not covered"
    U = fs.U.astype(np.float64)
    V = fs.V.astype(np.float64)
    steady = fs.times.size == 1

    def at(F, j, i):
        if steady:
            return F[0, j, i]
        return (1.0 - tau) * F[s0, j, i] + tau * F[s1, j, i]

    ph = 2.0 * np.pi * np.fmod(t - t_first, period) / period if period > 0 else 0.0
    out = np.zeros((len(x), 64))
    for r, (px, py) in enumerate(zip(x, y)):
        ci, fx = _cell(px, X)
        cj, fy = _cell(py, Y)
        i0 = ci if fx < 0.5 else ci + 1
        j0 = cj if fy < 0.5 else cj + 1
        row = out[r]
        row[0], row[1] = px / 180.0, py / 90.0
        row[2], row[3] = np.sin(ph), np.cos(ph)
        q = 4
        for dj in range(-2, 3):
            jj = min(max(j0 + dj, 0), ny - 1)
            for di in range(-2, 3):
                ii = min(max(i0 + di, 0), nx - 1)
                row[q] = at(U, jj, ii)
                row[q + 1] = at(V, jj, ii)
                q += 2
        row[54] = fx if fx < 0.5 else fx - 1.0
        row[55] = fy if fy < 0.5 else fy - 1.0
        w = ((1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy)
        corners = ((cj, ci), (cj, ci + 1), (cj + 1, ci), (cj + 1, ci + 1))
        row[56] = sum(wk * at(U, j, i) for wk, (j, i) in zip(w, corners))
        row[57] = sum(wk * at(V, j, i) for wk, (j, i) in zip(w, corners))
        hx, hy = X[ci + 1] - X[ci], Y[cj + 1] - Y[cj]
        if fs.s.spherical:
            hx *= M * np.cos(py * D)
            hy *= M
        row[58], row[59] = hx / 30000.0, hy / 30000.0
    return out


def check(fs: O.OracleFieldSet, x0, y0, xc, yc, coarse_status, Y, thr):
    """(accept, x1, y1, r): the residual decision per candidate and the distance r in
    metres between the network's and the coarse displacement."""
    X, Yax = fs.lon, fs.lat
    land = fs.land
    n = len(x0)
    acc = np.zeros(n, bool)
    x1 = np.array(x0, np.float64, copy=True)
    y1 = np.array(y0, np.float64, copy=True)
    r = np.zeros(n)
    for k in range(n):
        mx = float(Y[k][0]) * OUT_SCALE
        my = float(Y[k][1]) * OUT_SCALE
        ex, ey = xc[k] - x0[k], yc[k] - y0[k]
        nx1, ny1 = x0[k] + mx, y0[k] + my
        if fs.s.spherical:
            m = M * np.cos(y0[k] * D)
            ex, ey = ex * m, ey * M
            nx1, ny1 = x0[k] + mx / m, y0[k] + my / M
        r[k] = np.sqrt((mx - ex) ** 2 + (my - ey) ** 2)
        ok = coarse_status[k] == 0 and r[k] <= thr
        if ok:
            i, _ = O.locate(nx1, X)
            j, _ = O.locate(ny1, Yax)
            ok = i is not None and j is not None
            if ok and land is not None:
                ok = not (land[j, i] and land[j, i + 1] and land[j + 1, i] and land[j + 1, i + 1])
        if ok:
            acc[k] = True
            x1[k], y1[k] = nx1, ny1
    return acc, x1, y1, r
