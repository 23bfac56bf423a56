"""Pins of the oracle's spherical metric where particles move in latitude.

The conversion of m/s to degrees/s on a spherical mesh (Sect. 4.2.2) divides the
eastward velocity by M cos(lat); the library's reading takes cos(lat) at every
stage point, because it is part of the right-hand side of the trajectory equation
(Eq. 1).  Paper test 2 (zonal flow) keeps the latitude constant, so it cannot tell
where the cosine is taken.  A uniform field with a northward component can: the
interpolant reproduces it exactly, the latitude then moves linearly in time, and
classical RK4 on the longitude equation is Simpson's rule over one step,

    lat_n     = lat_0 + n dt V / M
    lon_(n+1) = lon_n + dt/6 (f(lat_n) + 4 f(lat_n + dt V / 2M) + f(lat_(n+1))),
    f(phi)    = U / (M cos(phi pi / 180)),

evaluated here in 40-digit arithmetic.

The Brownian displacement sqrt(2 Kh |dt|) N(0, 1) per component (Sect. 4.2.7) is
metres; on a sphere it is converted with the same metric at the latitude of the
RK4 end point X*, before the kick.  The normals are recomputed here with numpy
from the Philox words (those are pinned to published known answers elsewhere),
so the kick's size, sign, component order and metric latitude are all fixed.
"""

from __future__ import annotations

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O

M = 1852.0 * 60.0


def _sphere(U, V, lat_lo=-89.0, lat_hi=89.0):
    lon = np.arange(-180.0, 181.0, 1.0)
    lat = np.arange(lat_lo, lat_hi + 0.5, 1.0)
    Uf = np.full((1, lat.size, lon.size), U)
    Vf = np.full((1, lat.size, lon.size), V)
    return O.OracleFieldSet(lon, lat, None, [0.0], Uf, Vf, spherical=True)


def _rk4_uniform_sphere(lon0, lat0, U, V, dt, n):
    """RK4 positions after n steps of the uniform flow (U, V) m/s, 40 digits."""
    mp.mp.dps = 40
    Mm = mp.mpf(M)
    D = mp.pi / 180
    u, v, h = mp.mpf(U), mp.mpf(V), mp.mpf(dt)

    def f(phi):
        return u / (Mm * mp.cos(phi * D))

    lon, lat = mp.mpf(float(lon0)), mp.mpf(float(lat0))
    dlat = h * v / Mm
    for _ in range(n):
        lon = lon + h / 6 * (f(lat) + 4 * f(lat + dlat / 2) + f(lat + dlat))
        lat = lat + dlat
    return lon, lat


def _numpy_normals(run_id, pid, step):
    """Box-Muller on the Philox words with numpy's own log, sqrt, cos and sin."""
    w = [int(x) for x in O.philox4x32_10([pid, step, 0, 0], [run_id, O.SEED])]

    def unit(a, b):
        m = ((a << 32) | b) >> 11
        return np.float64(m) * 2.0 ** -53 + 2.0 ** -54

    u1, u2 = unit(w[0], w[1]), unit(w[2], w[3])
    r = np.sqrt(-2.0 * np.log(u1))
    a = 2.0 * np.pi * u2
    return r * np.cos(a), r * np.sin(a)


LAT0 = np.array([-70.0, -45.5, -12.25, 0.0, 3.75, 33.3, 47.0, 61.9])


@pytest.mark.parametrize("U,V,dt,n", [(0.7, 0.9, 3600.0, 48), (-0.4, -1.1, 1800.0, 60),
                                      (0.0, 0.8, 600.0, 30)])
def test_stage_metric_with_meridional_motion(U, V, dt, n):
    fs = _sphere(U, V)
    lon0 = np.linspace(-40.0, 40.0, LAT0.size)
    st = O.make_state(lon0, LAT0)
    assert O.advance(fs, st, dt, n) == 0
    assert (st.status == 0).all()
    for p in range(LAT0.size):
        lon, lat = _rk4_uniform_sphere(lon0[p], LAT0[p], U, V, dt, n)
        assert abs(st.y[p] - float(lat)) < 1e-11
        assert abs(st.x[p] - float(lon)) < 1e-11
    if U != 0.0:
        # the same run with cos(lat) frozen at the step start differs by far more than
        # the tolerance (the size a mistake in the stage latitude would show)
        alt = lon0.copy()
        lat = LAT0.copy()
        for _ in range(n):
            alt = alt + dt * U / (M * np.cos(np.deg2rad(lat)))
            lat = lat + dt * V / M
        assert np.abs(alt - st.x).max() > 1e-6


def _one_step_kick(lon0, lat0, U, V, dt, Kh, pid, step, run_id):
    lon_s, lat_s = _rk4_uniform_sphere(lon0, lat0, U, V, dt, 1)
    n1, n2 = _numpy_normals(run_id, pid, step)
    sig = np.sqrt(2.0 * Kh * abs(dt))
    lat1 = float(lat_s) + sig * n2 / M
    lon1 = float(lon_s) + sig * n1 / (M * np.cos(np.deg2rad(float(lat_s))))
    return lon1, lat1


@pytest.mark.parametrize("dt", [3600.0, -3600.0])
def test_brownian_kick_metric_at_the_rk4_end_point(dt):
    U, V, Kh, run_id = 0.3, 1.0, 25.0, 3
    fs = _sphere(U, V)
    lon0 = np.linspace(-20.0, 20.0, LAT0.size)
    st = O.make_state(lon0, LAT0, t_org=0.0 if dt > 0 else 0.0)
    assert O.advance(fs, st, dt, 1, Kh=Kh, run_id=run_id) == 0
    assert (st.status == 0).all()
    for p in range(LAT0.size):
        lon1, lat1 = _one_step_kick(lon0[p], LAT0[p], U, V, dt, Kh, p, 0, run_id)
        assert abs(st.y[p] - lat1) < 1e-11
        assert abs(st.x[p] - lon1) < 1e-11
    # a metric taken at the start latitude, or after the kick, would be this far off
    sig = np.sqrt(2.0 * Kh * abs(dt))
    n1 = np.array([_numpy_normals(run_id, p, 0)[0] for p in range(LAT0.size)])
    lat_s = LAT0 + dt * V / M
    at_end = sig * n1 / (M * np.cos(np.deg2rad(lat_s)))
    at_start = sig * n1 / (M * np.cos(np.deg2rad(LAT0)))
    assert np.abs(at_end - at_start).max() > 1e-7


def test_brownian_kick_keys_later_steps_by_absolute_step():
    """Several steps: each step's kick uses that step's normals, the metric at that
    step's RK4 end point, and every step starts where the last one ended."""
    U, V, Kh, dt, run_id = -0.5, 0.6, 10.0, 1800.0, 9
    fs = _sphere(U, V)
    lon0 = np.array([5.0, -100.0, 150.0])
    lat0 = np.array([-30.0, 10.0, 55.0])
    st = O.make_state(lon0, lat0, step=17)
    assert O.advance(fs, st, dt, 5, Kh=Kh, run_id=run_id) == 0
    for p in range(3):
        lon, lat = lon0[p], lat0[p]
        for s in range(17, 22):
            lon, lat = _one_step_kick(lon, lat, U, V, dt, Kh, p, s, run_id)
        assert abs(st.x[p] - lon) < 1e-11
        assert abs(st.y[p] - lat) < 1e-11


def test_backward_brownian_spread_matches_forward():
    """Zero flow on a flat mesh: a backward run's spread is that of a forward run,
    variance 2 Kh t per component (sigma uses the duration |dt|)."""
    n = 20000
    X = np.linspace(-1e6, 1e6, 21)
    Z = np.zeros((1, X.size, X.size))
    fs = O.OracleFieldSet(X, X, None, [0.0], Z, Z)
    Kh, dt, nsteps = 10.0, 300.0, 288
    var = 2.0 * Kh * abs(dt) * nsteps
    fw = O.make_state(np.zeros(n), np.zeros(n))
    bw = O.make_state(np.zeros(n), np.zeros(n))
    assert O.advance(fs, fw, dt, nsteps, Kh=Kh) == 0
    assert O.advance(fs, bw, -dt, nsteps, Kh=Kh) == 0
    assert (bw.status == 0).all() and np.isfinite(bw.x).all()
    # the same normals key both runs (particle id, step), so the paths are identical
    assert np.array_equal(fw.x, bw.x) and np.array_equal(fw.y, bw.y)
    for comp in (bw.x, bw.y):
        assert abs(comp.mean()) < 4 * np.sqrt(var / n)
        assert abs(comp.var() / var - 1) < 4 * np.sqrt(2.0 / n)
