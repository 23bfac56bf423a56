"""Brute-force check for tiny grids, in pure Python with 40-digit decimals.

TEST INFRASTRUCTURE ONLY.  This is a second, independent formulation used to
pin the C oracle (it does not call it):
  * the cell is found by scanning every cell of the axis (the definition of the
    rectilinear cell search, Sect. 2.4), not by bisection;
  * the interpolant inside a cell is written as the polynomial
    a + b dx + c dy + d dx dy (times (1, dz) in 3D) whose coefficients are solved
    from the corner values, instead of the corner-weight form;
  * the time interpolant, the metric and the RK4 stages are written out directly
    from Sect. 2.1.1 and Sect. 2.3, in decimal arithmetic, so rounding plays no
    part at FP64 level.
Only flat meshes are supported (no cosine).
"""

from __future__ import annotations

from decimal import Decimal, getcontext

getcontext().prec = 40


def D(v) -> Decimal:
    return Decimal(float(v)) if not isinstance(v, Decimal) else v


def scan_cell(x: Decimal, X):
    """Largest i with X[i] <= x among cells 0..n-2, or None outside [X0, Xn-1]."""
    Xd = [D(v) for v in X]
    if x < Xd[0] or x > Xd[-1]:
        return None
    found = None
    for i in range(len(Xd) - 1):
        if Xd[i] <= x:
            found = i
    return found


def _poly2(F, i, j, X, Y, x, y):
    """Bilinear polynomial through the four corners, evaluated at (x, y)."""
    hx = D(X[i + 1]) - D(X[i])
    hy = D(Y[j + 1]) - D(Y[j])
    f00 = D(F[j][i])
    f10 = D(F[j][i + 1])
    f01 = D(F[j + 1][i])
    f11 = D(F[j + 1][i + 1])
    a = f00
    b = (f10 - f00) / hx
    c = (f01 - f00) / hy
    d = (f11 - f10 - f01 + f00) / (hx * hy)
    dx = x - D(X[i])
    dy = y - D(Y[j])
    return a + b * dx + c * dy + d * dx * dy


def sample(grid, snaps, times, x, y, z, t, period=0.0):
    """Velocity (u, v, w) at a point, or None if outside.  ``snaps`` is a list over
    time of (U, V[, W]) arrays [ny][nx] or [nz][ny][nx]."""
    X, Y, Z = grid
    i = scan_cell(x, X)
    j = scan_cell(y, Y)
    if i is None or j is None:
        return None
    k = None
    if Z is not None:
        k = scan_cell(z, Z)
        if k is None:
            return None

    def spatial(F):
        if Z is None:
            return _poly2(F, i, j, X, Y, x, y)
        lo = _poly2(F[k], i, j, X, Y, x, y)
        hi = _poly2(F[k + 1], i, j, X, Y, x, y)
        hz = D(Z[k + 1]) - D(Z[k])
        return lo + (hi - lo) * (z - D(Z[k])) / hz

    nvar = 2 if Z is None else 3
    if len(times) == 1:
        return tuple(spatial(snaps[0][q]) for q in range(nvar)) + ((Decimal(0),) if Z is None else ())
    T = [D(v) for v in times]
    if period > 0:
        P = D(period)
        r = (t - T[0]) % P
        if r < 0:
            r += P
        tp = T[0] + r
        s = max(q for q in range(len(T)) if T[q] <= tp)
        t1 = T[s + 1] if s + 1 < len(T) else T[0] + P
        s1 = (s + 1) % len(T)
    else:
        if t < T[0] or t > T[-1]:
            raise ValueError("time outside snapshots")
        tp = t
        s = max(q for q in range(len(T) - 1) if T[q] <= tp)
        t1 = T[s + 1]
        s1 = s + 1
    out = []
    for q in range(nvar):
        f0 = spatial(snaps[s][q])
        f1 = spatial(snaps[s1][q])
        out.append(f0 + (f1 - f0) * (tp - T[s]) / (t1 - T[s]))
    if Z is None:
        out.append(Decimal(0))
    return tuple(out)


def rk4(grid, snaps, times, x0, y0, z0, t0, dt, nsteps, period=0.0):
    """Classical RK4 from (x0, y0, z0) at t0; returns the list of positions after
    each step, stopping (and returning 'OOB') if a stage or end point leaves."""
    x, y = D(x0), D(y0)
    z = D(z0) if z0 is not None else Decimal(0)
    dtd = D(dt)
    path = []
    for n in range(nsteps):
        tn = D(t0) + n * dtd
        k1 = sample(grid, snaps, times, x, y, z, tn, period)
        if k1 is None:
            return path, "OOB"
        h = dtd / 2
        k2 = sample(grid, snaps, times, x + k1[0] * h, y + k1[1] * h, z + k1[2] * h, tn + h, period)
        if k2 is None:
            return path, "OOB"
        k3 = sample(grid, snaps, times, x + k2[0] * h, y + k2[1] * h, z + k2[2] * h, tn + h, period)
        if k3 is None:
            return path, "OOB"
        k4 = sample(grid, snaps, times, x + k3[0] * dtd, y + k3[1] * dtd, z + k3[2] * dtd,
                    tn + dtd, period)
        if k4 is None:
            return path, "OOB"
        nx_ = x + dtd * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0]) / 6
        ny_ = y + dtd * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1]) / 6
        nz_ = z + dtd * (k1[2] + 2 * k2[2] + 2 * k3[2] + k4[2]) / 6
        X, Y, Z = grid
        if (scan_cell(nx_, X) is None or scan_cell(ny_, Y) is None
                or (Z is not None and scan_cell(nz_, Z) is None)):
            return path, "OOB"
        x, y, z = nx_, ny_, nz_
        path.append((x, y, z))
    return path, "OK"
