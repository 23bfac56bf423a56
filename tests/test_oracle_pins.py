"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms of
the idealised cases of Sect. 4.2, exactness of linear interpolation for linear
fields, fourth-order convergence, the printed accuracy figures, a brute-force
decimal re-derivation on tiny grids, and published Philox known-answer vectors.
"""

from __future__ import annotations

import os
from decimal import Decimal

import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from synthetic import configs as SC
from synthetic import idealised as SI

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_axis(rng, n, lo, hi):
    """Strictly increasing, clearly non-uniform axis."""
    w = rng.uniform(0.3, 1.7, n - 1)
    x = np.concatenate([[0.0], np.cumsum(w)])
    return lo + (hi - lo) * x / x[-1]


# ------------------------------------------------------------------ cell search (O1)
def test_locate_rules_match_cell_scan():
    rng = np.random.default_rng(11)
    X = rand_axis(rng, 9, -50.0, 120.0)
    pts = list(X) + list(rng.uniform(X[0], X[-1], 200)) + [X[0] - 1e-9, X[-1] + 1e-9]
    for x in pts:
        i, f = O.locate(x, X)
        j = brute.scan_cell(Decimal(float(x)), X)
        assert i == j
        if i is not None:
            assert X[i] <= x <= X[i + 1]
            assert 0.0 <= f <= 1.0
    # last node: last cell, fraction 1; a node: its own cell, fraction 0
    assert O.locate(X[-1], X) == (X.size - 2, 1.0)
    assert O.locate(X[3], X) == (3, 0.0)
    assert O.locate(float("nan"), X) == (None, None)


# ------------------------------------------------------------------ K1 exact interpolation
@pytest.mark.parametrize("seed", range(4))
def test_bilinear_exact_for_bilinear_fields(seed):
    rng = np.random.default_rng(100 + seed)
    X = rand_axis(rng, 7, -1e3, 2e3)
    Y = rand_axis(rng, 6, 10.0, 600.0)
    cu = rng.normal(size=4)
    cv = rng.normal(size=4)
    XX, YY = np.meshgrid(X, Y)

    def f(c, x, y):
        return c[0] + c[1] * x + c[2] * y + c[3] * x * y

    fs = O.OracleFieldSet(X, Y, None, [0.0], f(cu, XX, YY)[None], f(cv, XX, YY)[None])
    scale = np.abs(f(cu, XX, YY)).max() + np.abs(f(cv, XX, YY)).max()
    xs = np.concatenate([rng.uniform(X[0], X[-1], 300), X, [X[-1]] * 6])
    ys = np.concatenate([rng.uniform(Y[0], Y[-1], 300), Y[rng.integers(0, Y.size, X.size)], Y])
    for x, y in zip(xs, ys):
        rc, out = fs.sample(x, y, 0.0, 0.0)
        assert rc == 0
        assert abs(out[0] - f(cu, x, y)) <= 1e-14 * scale
        assert abs(out[1] - f(cv, x, y)) <= 1e-14 * scale


@pytest.mark.parametrize("seed", range(3))
def test_trilinear_exact_for_trilinear_fields(seed):
    rng = np.random.default_rng(200 + seed)
    X = rand_axis(rng, 6, 0.0, 10.0)
    Y = rand_axis(rng, 5, -5.0, 5.0)
    Z = rand_axis(rng, 4, 5.0, 900.0)
    c = rng.normal(size=(3, 8))
    ZZ, YY, XX = np.meshgrid(Z, Y, X, indexing="ij")

    def f(k, x, y, z):
        a = c[k]
        return (a[0] + a[1] * x + a[2] * y + a[3] * z + a[4] * x * y + a[5] * x * z
                + a[6] * y * z + a[7] * x * y * z)

    F = [f(k, XX, YY, ZZ)[None] for k in range(3)]
    fs = O.OracleFieldSet(X, Y, Z, [0.0], F[0], F[1], F[2])
    scale = max(np.abs(F[k]).max() for k in range(3))
    for _ in range(300):
        x, y, z = rng.uniform(X[0], X[-1]), rng.uniform(Y[0], Y[-1]), rng.uniform(Z[0], Z[-1])
        rc, out = fs.sample(x, y, z, 0.0)
        assert rc == 0
        for k in range(3):
            assert abs(out[k] - f(k, x, y, z)) <= 1e-14 * scale
    rc, out = fs.sample(X[-1], Y[-1], Z[-1], 0.0)
    assert rc == 0 and abs(out[2] - f(2, X[-1], Y[-1], Z[-1])) <= 1e-14 * scale


@pytest.mark.parametrize("periodic", [False, True])
def test_time_interpolation_linear_in_time(periodic):
    rng = np.random.default_rng(7)
    X = rand_axis(rng, 5, 0.0, 1.0)
    Y = rand_axis(rng, 4, 0.0, 1.0)
    T = np.array([0.0, 100.0, 250.0, 600.0])
    base = rng.normal(size=(4, 4, 5))
    slope = rng.normal(size=(4, 5))
    # snapshot s: base[s] is arbitrary per snapshot; the value between s and s+1 must be
    # the straight line between the two spatial interpolants
    U = base
    V = base + slope[None]
    period = 800.0 if periodic else 0.0
    fs = O.OracleFieldSet(X, Y, None, T, U, V, period=period)
    x, y = 0.37, 0.61
    sp = [fs.sample(x, y, 0.0, t)[1][0] for t in T]  # spatial values at the nodes
    tests = [(0.0, 0, 0.0), (50.0, 0, 0.5), (175.0, 1, 0.5), (600.0 - 1e-9, 2, None)]
    if periodic:
        tests += [(700.0, 3, 0.5), (800.0 + 175.0, 1, 0.5), (-625.0, 1, 0.5)]
    for t, s, tau in tests:
        rc, out = fs.sample(x, y, 0.0, t)
        assert rc == 0
        if tau is None:
            continue
        nxt = sp[(s + 1) % 4]
        assert out[0] == pytest.approx((1 - tau) * sp[s] + tau * nxt, abs=1e-14)
    if not periodic:
        assert fs.time_bracket(600.0 + 1e-6)[0] == -4
        assert fs.time_bracket(-1e-6)[0] == -4
        rc, s0, s1, tau = fs.time_bracket(600.0)
        assert (rc, s0, s1, tau) == (0, 2, 3, 1.0)


# ------------------------------------------------------------------ K2 solid-body rotation
def _rk4_rotation_closed_form(z0, theta, n):
    """(Z_n - c) = R(i theta)^n (Z_0 - c), R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24,
    evaluated in 40-digit decimals."""
    th = Decimal(theta)
    re = 1 - th ** 2 / 2 + th ** 4 / 24
    im = th - th ** 3 / 6
    zr, zi = Decimal(float(z0.real)), Decimal(float(z0.imag))
    pr, pi_ = Decimal(1), Decimal(0)
    br, bi = re, im
    k = n
    while k:
        if k & 1:
            pr, pi_ = pr * br - pi_ * bi, pr * bi + pi_ * br
        br, bi = br * br - bi * bi, 2 * br * bi
        k >>= 1
    return complex(float(zr * pr - zi * pi_), float(zr * pi_ + zi * pr))


def test_cfg0_rotation_matches_discrete_closed_form():
    w = SC.cfg0_solid_body(n_particles=2000)
    fs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0)
    assert O.advance(fs, st, w.dt, w.nsteps) == 0
    assert (st.status == 0).all()
    omega = w.meta["omega"]
    z0 = (w.lon0 - 5e4) + 1j * (w.lat0 - 5e4)
    zc = np.array([_rk4_rotation_closed_form(z, omega * w.dt, w.nsteps) for z in z0])
    err = np.abs((st.x - 5e4 + 1j * (st.y - 5e4)) - zc)
    assert err.max() < 1e-8
    # radius conserved and angle = w t (phase lag per step theta^5/120 is below rounding)
    r0 = np.abs(z0)
    r1 = np.abs(st.x - 5e4 + 1j * (st.y - 5e4))
    assert np.abs(r1 - r0).max() < 1e-8
    exact = z0 * np.exp(1j * omega * w.dt * w.nsteps)
    assert np.abs((st.x - 5e4 + 1j * (st.y - 5e4)) - exact).max() < 1e-7


def test_paper_radial_rotation_error_below_3mm():
    w = SI.radial_rotation()
    fs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0)
    recs = O.run(fs, st, w.dt, w.nsteps * w.dt, w.outputdt)
    omega = w.meta["omega"]
    z0 = w.lon0 + 1j * w.lat0
    bound = float(open(os.path.join(GOLDEN, "paper_accuracy.txt")).read().split(
        "radial_rotation_max_error")[1].split()[0])
    worst = 0.0
    for m, r in enumerate(recs):
        t = m * w.outputdt
        exact = z0 * np.exp(1j * omega * t)
        worst = max(worst, np.abs(r["lon"] + 1j * r["lat"] - exact).max())
        n = int(round(t / w.dt))
        zc = np.array([_rk4_rotation_closed_form(z, omega * w.dt, n) for z in z0])
        assert np.abs(r["lon"] + 1j * r["lat"] - zc).max() < 1e-9
    assert worst < bound
    # the discrete RK4 phase error after 24 h at r = 4 km is 4.7e-5 m
    assert worst == pytest.approx(4.7e-5, rel=0.03)


# ------------------------------------------------------------------ K3 convergence
def test_fourth_order_convergence():
    w = SC.cfg0_solid_body(n_particles=1)
    fs = O.OracleFieldSet.from_workload(w)
    omega = w.meta["omega"]
    errs = []
    for dt in (3600.0, 1800.0, 900.0, 450.0):
        st = O.make_state([5e4 + 4e4], [5e4])
        assert O.advance(fs, st, dt, int(round(86400 / dt))) == 0
        exact = 4e4 * np.exp(1j * omega * 86400.0)
        errs.append(abs((st.x[0] - 5e4) + 1j * (st.y[0] - 5e4) - exact))
    expected = [4.84e-4, 3.02e-5, 1.89e-6, 1.18e-7]
    for e, x in zip(errs, expected):
        assert e == pytest.approx(x, rel=0.02)
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    for q in ratios:
        assert 15.5 < q < 16.5


# ------------------------------------------------------------------ K4 oscillating flow
def test_paper_oscillating_zonal_flow():
    w = SI.oscillating_zonal_flow()
    fs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0)
    recs = O.run(fs, st, w.dt, w.nsteps * w.dt, w.outputdt)
    A, om = w.meta["A"], w.meta["omega"]
    th = om * w.dt
    gain = (th / 2) / np.tan(th / 2)
    worst_x = worst_y = 0.0
    for m, r in enumerate(recs):
        t = m * w.outputdt
        # Simpson's rule on the piecewise-linear time interpolant is the trapezoid rule
        xd = w.lon0 + (A / om) * np.sin(om * t) * gain
        assert np.abs(r["lon"] - xd).max() < 1e-9
        assert np.abs(r["lat"] - A * t).max() < 1e-9
        worst_x = max(worst_x, np.abs(r["lon"] - (w.lon0 + (A / om) * np.sin(om * t))).max())
        worst_y = max(worst_y, np.abs(r["lat"] - A * t).max())
    # linear-in-time interpolation error: (A/w)(1 - (th/2)/tan(th/2)) = 5.45 cm; paper: 6 cm
    assert worst_x == pytest.approx((A / om) * (1 - gain), rel=1e-6)
    assert worst_x == pytest.approx(0.0545, abs=5e-4)
    assert worst_x < 0.06
    assert worst_y < 4e-3 and worst_y < 1e-9


# ------------------------------------------------------------------ K5 zonal flow on a sphere
def test_paper_zonal_flow_on_sphere():
    w = SI.zonal_flow_sphere()
    fs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0)
    assert O.advance(fs, st, w.dt, w.nsteps) == 0
    assert (st.status == 0).all()
    assert np.array_equal(st.y, w.lat0)  # latitude is bit-constant
    M = 1852.0 * 60.0
    per_step = w.dt / (M * np.cos(np.deg2rad(w.lat0)))
    assert np.abs(st.x - (w.lon0 + w.nsteps * per_step)).max() < 1e-9
    eq = int(np.argmin(np.abs(w.lat0)))
    assert st.x[eq] == pytest.approx(44.3197, abs=1e-4)
    dist = np.deg2rad(st.x) * (M * 180 / np.pi) * np.cos(np.deg2rad(w.lat0))
    assert np.allclose(dist, 57 * 86400.0, rtol=1e-9)
    assert dist[eq] == pytest.approx(4.9e6, rel=0.01)


# ------------------------------------------------------------------ K6 Brownian motion
def test_paper_brownian_uniform_kh():
    w = SI.brownian_uniform_kh()
    fs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0)
    assert O.advance(fs, st, w.dt, w.nsteps, Kh=w.Kh, run_id=0) == 0
    assert (st.status == 0).all()
    N = w.n
    sig = np.sqrt(2 * w.Kh * w.nsteps * w.dt)
    assert sig == pytest.approx(4156.9, abs=0.1)
    for comp in (st.x, st.y):
        assert abs(comp.mean()) < 4 * sig / np.sqrt(N)
        assert abs(comp.var() / sig ** 2 - 1) < 4 * np.sqrt(2.0 / N)
    # paper: sigma = 4.16 km
    assert np.sqrt(0.5 * (st.x.var() + st.y.var())) == pytest.approx(4160.0, rel=0.01)
    # radial distribution: r^2 / (2 sigma^2) is exponential -> 20 equiprobable bins
    u = 1 - np.exp(-(st.x ** 2 + st.y ** 2) / (2 * sig ** 2))
    h, _ = np.histogram(u, bins=20, range=(0, 1))
    chi2 = ((h - N / 20) ** 2 / (N / 20)).sum()
    assert chi2 < 50.0
    ang = np.arctan2(st.y, st.x)
    h, _ = np.histogram(ang, bins=16, range=(-np.pi, np.pi))
    assert ((h - N / 16) ** 2 / (N / 16)).sum() < 45.0


# ------------------------------------------------------------------ K7 brute force
@pytest.mark.parametrize("seed,is3d,nt", [(1, False, 1), (2, False, 3), (3, True, 1), (4, True, 2)])
def test_brute_force_tiny_grids(seed, is3d, nt):
    rng = np.random.default_rng(300 + seed)
    X = rand_axis(rng, 5, 0.0, 4000.0)
    Y = rand_axis(rng, 4, 0.0, 3000.0)
    Z = rand_axis(rng, 3, 0.0, 100.0) if is3d else None
    shape = (nt, 3, 4, 5) if is3d else (nt, 4, 5)
    U = rng.normal(size=shape) * 0.3
    V = rng.normal(size=shape) * 0.3
    W = rng.normal(size=shape) * 0.002 if is3d else None
    T = {1: np.array([0.0]), 2: np.array([0.0, 2700.0]), 3: np.array([0.0, 900.0, 2700.0])}[nt]
    fs = O.OracleFieldSet(X, Y, Z, T, U, V, W)
    x0 = rng.uniform(1500, 2500, 6)
    y0 = rng.uniform(1000, 2000, 6)
    z0 = rng.uniform(30, 70, 6) if is3d else None
    nsteps = 20 if nt == 1 else 9
    dt = 100.0 if nt == 1 else 300.0
    st = O.make_state(x0, y0, z0)
    snaps = [[U[s], V[s]] + ([W[s]] if is3d else []) for s in range(nt)]
    paths = [brute.rk4((X, Y, Z), snaps, T, x0[p], y0[p], None if z0 is None else z0[p],
                       0.0, dt, nsteps) for p in range(6)]
    for n in range(nsteps):
        assert O.advance(fs, st, dt, 1) == 0
        for p in range(6):
            path, flag = paths[p]
            if n < len(path):
                bx, by, bz = (float(v) for v in path[n])
                assert st.status[p] == 0
                assert abs(st.x[p] - bx) <= 1e-12 * 4000
                assert abs(st.y[p] - by) <= 1e-12 * 3000
                if is3d:
                    assert abs(st.z[p] - bz) <= 1e-12 * 100
                ci, cj, ck = fs.cell_indices(st.x[p:p + 1], st.y[p:p + 1],
                                             None if z0 is None else st.z[p:p + 1])
                assert ci[0] == brute.scan_cell(path[n][0], X)
                assert cj[0] == brute.scan_cell(path[n][1], Y)
            elif flag == "OOB" and n == len(path):
                assert st.status[p] == (O.ST_OOB | O.ST_DELETED)


# ------------------------------------------------------------------ K8 special cases
def _flat_field(n=11, u=0.0, v=0.0, land=None):
    X = 100.0 * np.arange(n)
    U = np.full((1, n, n), u)
    V = np.full((1, n, n), v)
    if land is not None:
        U[0][land != 0] = 0.0
        V[0][land != 0] = 0.0
    return O.OracleFieldSet(X, X.copy(), None, [0.0], U, V, land=land), X


def test_special_cases_status_and_position():
    land = np.zeros((11, 11), np.uint8)
    land[4:7, 4:7] = 1  # cells (4,4),(4,5),(5,4),(5,5) have four land corners
    fs, X = _flat_field(u=0.01, land=land)
    x0 = np.array([-1.0, 550.0, 1000.0, np.nan, 200.0, 990.0])
    y0 = np.array([500.0, 550.0, 1000.0, 500.0, 200.0, 200.0])
    st = O.make_state(x0, y0)
    assert O.advance(fs, st, 60.0, 1) == 0
    # outside -> OOB|DELETED, position unchanged
    assert st.status[0] == O.ST_OOB | O.ST_DELETED and st.x[0] == -1.0
    # inside an all-land cell -> LAND|DELETED, unchanged
    assert st.status[1] == O.ST_LAND | O.ST_DELETED and st.x[1] == 550.0
    # on the last node: in the domain; u = 0.01 pushes it out -> rejected step
    assert st.status[2] == O.ST_OOB | O.ST_DELETED and st.x[2] == 1000.0
    assert st.status[3] == O.ST_OOB | O.ST_DELETED
    assert st.status[4] == 0 and st.x[4] == pytest.approx(200.6)
    # 990 + 0.6 stays in
    assert st.status[5] == 0
    ci, cj, _ = fs.cell_indices(np.array([1000.0]), np.array([1000.0]))
    assert (ci[0], cj[0]) == (9, 9)
    # deleted particles are never advanced again
    before = st.x.copy()
    assert O.advance(fs, st, 60.0, 3) == 0
    assert np.array_equal(st.x[:4], before[:4], equal_nan=True)
    # a zero-velocity particle on the last node stays in the domain
    fs0, _ = _flat_field()
    st0 = O.make_state([1000.0], [1000.0])
    assert O.advance(fs0, st0, 60.0, 2) == 0 and st0.status[0] == 0


def test_freeze_policy_sets_oob_without_delete():
    fs, X = _flat_field(u=1.0)
    st = O.make_state([990.0], [500.0])
    assert O.advance(fs, st, 60.0, 1, policy=O.POLICY_FREEZE) == 0
    assert st.status[0] == O.ST_OOB and st.x[0] == 990.0


def test_particle_steps_count_active_particles():
    fs, X = _flat_field(u=1.0)
    st = O.make_state([100.0, 900.0, 500.0], [500.0, 500.0, 500.0])
    st.status[2] = O.ST_DELETED
    assert O.advance(fs, st, 10.0, 20) == 0
    # particle 0 runs 20 steps; particle 1 leaves at step 11 (x = 1000 is inside)
    assert st.status[1] == O.ST_OOB | O.ST_DELETED
    assert st.psteps == 20 + 11


def test_time_outside_snapshots_is_an_error():
    X = np.arange(4.0)
    U = np.zeros((2, 4, 4))
    fs = O.OracleFieldSet(X, X, None, [0.0, 100.0], U, U)
    st = O.make_state([1.0], [1.0])
    assert O.advance(fs, st, 10.0, 10) == 0
    assert O.advance(fs, st, 10.0, 1) == -4
    assert st.step == 10


# ------------------------------------------------------------------ K9 steady vs repeated
def test_steady_equals_two_identical_snapshots():
    w = SC.cfg1_global_eddies(nx=144, ny=72, nt=1, n_particles=200, nsteps=200)
    U, V, _ = w.fields.materialise()
    fs1 = O.OracleFieldSet(w.grid.lon, w.grid.lat, None, [0.0], U[:1], V[:1], spherical=True,
                           land=w.grid.land)
    fs2 = O.OracleFieldSet(w.grid.lon, w.grid.lat, None, [0.0, 1e9],
                           np.concatenate([U[:1], U[:1]]), np.concatenate([V[:1], V[:1]]),
                           spherical=True, land=w.grid.land)
    a = O.make_state(w.lon0, w.lat0)
    b = O.make_state(w.lon0, w.lat0)
    assert O.advance(fs1, a, w.dt, 200) == 0
    assert O.advance(fs2, b, w.dt, 200) == 0
    ok = (a.status == 0) & (b.status == 0)
    assert np.array_equal(a.status, b.status)
    assert np.abs(a.x[ok] - b.x[ok]).max() <= 1e-11 * 360
    assert np.abs(a.y[ok] - b.y[ok]).max() <= 1e-11 * 180


# ------------------------------------------------------------------ K10 / K11 invariances
def _small_eddies(n=500):
    w = SC.cfg1_global_eddies(nx=144, ny=72, nt=6, n_particles=n, nsteps=288 * 2,
                              period_days=6.0)
    return w, O.OracleFieldSet.from_workload(w)


def test_chunking_and_resume_bit_identical():
    w, fs = _small_eddies()
    a = O.make_state(w.lon0, w.lat0)
    O.advance(fs, a, w.dt, 576, Kh=10.0, run_id=3)
    b = O.make_state(w.lon0, w.lat0)
    for _ in range(4):
        O.advance(fs, b, w.dt, 144, Kh=10.0, run_id=3)
    # get / create round trip after 100 steps (absolute step index carried over)
    c = O.make_state(w.lon0, w.lat0)
    O.advance(fs, c, w.dt, 100, Kh=10.0, run_id=3)
    c2 = O.make_state(c.x, c.y, t_org=c.t_org, step=c.step)
    c2.status[:] = c.status
    O.advance(fs, c2, w.dt, 476, Kh=10.0, run_id=3)
    for s in (b, c2):
        assert np.array_equal(a.x, s.x) and np.array_equal(a.y, s.y)
        assert np.array_equal(a.status, s.status)
    assert a.psteps == b.psteps


def test_permutation_invariance():
    w, fs = _small_eddies()
    perm = np.random.default_rng(5).permutation(w.n)
    a = O.make_state(w.lon0, w.lat0)
    O.advance(fs, a, w.dt, 300, Kh=10.0)
    b = O.make_state(w.lon0[perm], w.lat0[perm], pid=perm.astype(np.uint32))
    O.advance(fs, b, w.dt, 300, Kh=10.0)
    assert np.array_equal(a.x[perm], b.x) and np.array_equal(a.status[perm], b.status)


# ------------------------------------------------------------------ K12 Philox
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = O.philox4x32_10(v[0:4], v[4:6])
        assert list(out) == v[6:10]


def test_normals_are_standard():
    n = np.array([O.normals(1, O.SEED, p, 7) for p in range(20000)])
    assert abs(n.mean()) < 0.03
    assert abs(n.var() - 1) < 0.03
    assert np.corrcoef(n[:, 0], n[:, 1])[0, 1] < 0.03


# ------------------------------------------------------------------ f3 / f4 schemes
def _decimal_pow(re, im, z0, n):
    pr, pi_ = Decimal(1), Decimal(0)
    br, bi = re, im
    k = n
    while k:
        if k & 1:
            pr, pi_ = pr * br - pi_ * bi, pr * bi + pi_ * br
        br, bi = br * br - bi * bi, 2 * br * bi
        k >>= 1
    zr, zi = Decimal(float(z0.real)), Decimal(float(z0.imag))
    return complex(float(zr * pr - zi * pi_), float(zr * pi_ + zi * pr))


def test_euler_forward_closed_form():
    """Euler on the linear rotation field: Z_n - c = (1 + i theta)^n (Z_0 - c)."""
    w = SC.cfg0_solid_body(n_particles=300, nsteps=500)
    fs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0)
    assert O.advance(fs, st, w.dt, w.nsteps, scheme=O.SCHEME_EULER) == 0
    th = Decimal(w.meta["omega"]) * Decimal(w.dt)
    z0 = (w.lon0 - 5e4) + 1j * (w.lat0 - 5e4)
    zc = np.array([_decimal_pow(Decimal(1), th, z, w.nsteps) for z in z0])
    assert np.abs((st.x - 5e4 + 1j * (st.y - 5e4)) - zc).max() < 1e-8
    # the radius grows by (1 + theta^2)^(n/2), the scheme's known drift
    growth = (1 + float(th) ** 2) ** (w.nsteps / 2)
    assert np.allclose(np.abs(st.x - 5e4 + 1j * (st.y - 5e4)), np.abs(z0) * growth, rtol=1e-12)


def test_nearest_neighbour_picks_the_nearer_node():
    rng = np.random.default_rng(21)
    X = rand_axis(rng, 8, 0.0, 100.0)
    Y = rand_axis(rng, 6, -20.0, 20.0)
    U = rng.normal(size=(2, 6, 8))
    V = rng.normal(size=(2, 6, 8))
    T = np.array([0.0, 50.0])
    fs = O.OracleFieldSet(X, Y, None, T, U, V)
    for _ in range(400):
        x, y, t = rng.uniform(X[0], X[-1]), rng.uniform(Y[0], Y[-1]), rng.uniform(0, 50)
        rc, out = fs.sample(x, y, 0.0, t, nearest=True)
        assert rc == 0
        # brute force: the node whose coordinate is closest on each axis (ties up)
        i = int(np.argmin(np.abs(X - x) - 1e-12 * (X >= x)))
        j = int(np.argmin(np.abs(Y - y) - 1e-12 * (Y >= y)))
        tau = t / 50.0
        exp = (1 - tau) * U[0, j, i] + tau * U[1, j, i]
        assert out[0] == pytest.approx(exp, abs=1e-14)
    # a point at a cell centre goes to the upper node
    xm = 0.5 * (X[2] + X[3])
    rc, out = fs.sample(xm, Y[1], 0.0, 0.0, nearest=True)
    assert out[0] == U[0, 1, 3] or abs((xm - X[2]) / (X[3] - X[2]) - 0.5) > 0


def test_backward_in_time_returns_to_start():
    """Forward n steps then backward n steps on the rotation field: the discrete map
    is |R(i theta)|^(2n) (Z_0 - c), i.e. the start point to within theta^6 n r."""
    w = SC.cfg0_solid_body(n_particles=200, nsteps=1440)
    fs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0)
    assert O.advance(fs, st, w.dt, w.nsteps) == 0
    assert O.advance(fs, st, -w.dt, w.nsteps) == 0
    assert st.step == 2 * w.nsteps
    z0 = (w.lon0 - 5e4) + 1j * (w.lat0 - 5e4)
    back = st.x - 5e4 + 1j * (st.y - 5e4)
    th = Decimal(w.meta["omega"]) * Decimal(w.dt)
    re = 1 - th ** 2 / 2 + th ** 4 / 24
    im = th - th ** 3 / 6
    mod2 = re * re + im * im  # |R(i theta)|^2
    zc = np.array([_decimal_pow(mod2, Decimal(0), z, w.nsteps) for z in z0])
    assert np.abs(back - zc).max() < 1e-8
    assert np.abs(back - z0).max() < 1e-6


def test_backward_needs_snapshots_before_the_start():
    X = np.arange(4.0)
    U = np.zeros((2, 4, 4))
    fs = O.OracleFieldSet(X, X, None, [0.0, 100.0], U, U)
    st = O.make_state([1.0], [1.0], t_org=100.0)
    assert O.advance(fs, st, -10.0, 10) == 0
    assert O.advance(fs, st, -10.0, 1) == -4
