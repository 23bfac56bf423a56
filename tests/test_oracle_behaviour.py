"""Pins of the oracle's worked-example kernels (Sect. 3.3): sinking at a fixed
speed to (or, backward in time, back up to) the dwelling depth, age with deletion
at the maximum age, and sampling of a tracer at the particle, run before the RK4
advection of each step.  Checked against closed forms on fields whose answers are
known exactly: still water, uniform currents and a tracer linear in space and
time (reproduced exactly by linear interpolation)."""

from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O

DAY = 86400.0


def _box(u=0.0, v=0.0, w=0.0, nt=2, T=None, tracer=None):
    """Flat 3D box 0..1e5 m x 0..1e5 m x 5..5500 m with uniform U, V, W."""
    X = np.linspace(0.0, 1e5, 11)
    Y = np.linspace(0.0, 1e5, 9)
    Z = np.linspace(5.0, 5500.0, 12)
    times = np.array([0.0, 200 * DAY]) if T is None else T
    shape = (times.size, Z.size, Y.size, X.size)
    U = np.full(shape, u)
    V = np.full(shape, v)
    W = np.full(shape, w)
    return O.OracleFieldSet(X, Y, Z, times, U, V, W, tracer=tracer), X, Y, Z, times


def test_sinking_backward_rises_to_the_dwelling_depth():
    """Time-backward run in still water: depth falls by w_s |dt| per step from
    2,440 m and stops exactly at the dwelling depth (50 m)."""
    fs, *_ = _box()
    ws, dwell, dt = 200.0 / DAY, 50.0, -300.0
    st = O.make_state([5e4, 2e4], [5e4, 7e4], [2440.0, 1000.0], t_org=100 * DAY)
    for n in [1, 10, 100]:
        assert O.advance(fs, st, dt, n, sink_speed=ws, dwell_depth=dwell) == 0
    steps = 111
    expect = np.maximum(dwell, np.array([2440.0, 1000.0]) - ws * 300.0 * steps)
    assert np.allclose(st.z, expect, rtol=0, atol=1e-9)
    assert O.advance(fs, st, dt, 4000, sink_speed=ws, dwell_depth=dwell) == 0
    assert (st.z == dwell).all() and (st.status == 0).all()
    # the number of steps to get there: ceil((2440 - 50) / (w_s |dt|))
    st2 = O.make_state([5e4], [5e4], [2440.0], t_org=100 * DAY)
    k = int(np.ceil((2440.0 - dwell) / (ws * 300.0)))
    assert O.advance(fs, st2, dt, k - 1, sink_speed=ws, dwell_depth=dwell) == 0
    assert st2.z[0] > dwell
    assert O.advance(fs, st2, dt, 1, sink_speed=ws, dwell_depth=dwell) == 0
    assert st2.z[0] == dwell


def test_sinking_forward_leaves_through_the_floor():
    fs, _, _, Z, _ = _box()
    ws, dt = 200.0 / DAY, 3600.0
    st = O.make_state([5e4], [5e4], [5400.0])
    assert O.advance(fs, st, dt, 100, sink_speed=ws, dwell_depth=50.0) == 0
    # 5400 + 200/24 m per hour reaches the last level (still inside) on step 12 and
    # passes it on step 13: the kernels act in order, so the sink's move stands and
    # the advection that follows fails (the particle is deleted where it sank to)
    assert st.status[0] == O.ST_OOB | O.ST_DELETED
    assert st.psteps == 13
    assert st.z[0] == pytest.approx(5400.0 + 13 * 200.0 / 24.0, abs=1e-9)


def test_age_deletes_at_maxage_and_counts_the_step():
    """Uniform current, no sinking: every step ages by |dt|; the step on which the
    age reaches maxage deletes the particle before it moves."""
    fs, *_ = _box(u=0.1, v=-0.05)
    dt, k = 600.0, 10
    st = O.make_state([1e4, 3e4], [5e4, 6e4], [100.0, 100.0])
    assert O.advance(fs, st, dt, 50, maxage=k * dt) == 0
    assert (st.status == O.ST_AGED | O.ST_DELETED).all()
    assert st.psteps == 2 * k
    assert np.allclose(st.age, k * dt)
    assert np.allclose(st.x, [1e4 + 0.1 * dt * (k - 1), 3e4 + 0.1 * dt * (k - 1)], atol=1e-9)
    assert np.allclose(st.y, [5e4 - 0.05 * dt * (k - 1), 6e4 - 0.05 * dt * (k - 1)], atol=1e-9)


def test_age_starts_at_the_dwelling_depth_and_backward_time_ages_forward():
    fs, *_ = _box()
    ws, dwell, dt = 200.0 / DAY, 50.0, -300.0
    st = O.make_state([5e4], [5e4], [50.0 + ws * 300.0 * 20.5], t_org=150 * DAY)
    assert O.advance(fs, st, dt, 30, sink_speed=ws, dwell_depth=dwell, maxage=DAY) == 0
    # 20 steps leave it half a step below the dwelling depth; step 21 brings it up,
    # and it ages on that step and on every later one: 10 steps of |dt|
    assert st.age[0] == 10 * 300.0
    assert st.status[0] == 0


def test_tracer_sample_is_exact_for_a_linear_tracer():
    """T = a + b x + c y + d z + e t is reproduced exactly by trilinear, linear-in-
    time interpolation; the value held after a step is the one at the step's start
    (sampling runs before the advection)."""
    a, b, c, d, e = 20.0, 1e-5, -2e-5, -3e-3, 1e-7
    X = np.linspace(0.0, 1e5, 11)
    Y = np.linspace(0.0, 1e5, 9)
    Z = np.linspace(5.0, 5500.0, 12)
    times = np.array([0.0, 10 * DAY, 20 * DAY])
    TT, ZZ, YY, XX = np.meshgrid(times, Z, Y, X, indexing="ij")
    tracer = a + b * XX + c * YY + d * ZZ + e * TT
    fs, *_ = _box(u=0.2, v=0.1, T=times, tracer=tracer)
    dt = 900.0
    st = O.make_state([2e4], [3e4], [400.0], t_org=DAY)
    for n in range(1, 6):
        assert O.advance(fs, st, dt, 1, sample=True) == 0
        t0 = DAY + (n - 1) * dt
        x0 = 2e4 + 0.2 * dt * (n - 1)
        y0 = 3e4 + 0.1 * dt * (n - 1)
        assert st.temp[0] == pytest.approx(a + b * x0 + c * y0 + d * 400.0 + e * t0,
                                           rel=1e-13, abs=1e-12)
    rc, val = fs.sample_tracer(5e4, 5e4, 1000.0, 5 * DAY)
    assert rc == 0 and val == pytest.approx(a + b * 5e4 + c * 5e4 + d * 1000.0 + e * 5 * DAY,
                                            rel=1e-13)
    assert fs.sample_tracer(-1.0, 5e4, 1000.0, 5 * DAY)[0] == 1


def test_dwelling_phase_is_horizontal_only():
    """With W != 0 the sinking phase moves with the 3D flow, but once at the
    dwelling depth the particle keeps that depth exactly."""
    fs, *_ = _box(u=0.05, w=1e-3)
    ws, dwell, dt = 200.0 / DAY, 50.0, -600.0
    st = O.make_state([5e4], [5e4], [300.0], t_org=100 * DAY)
    assert O.advance(fs, st, dt, 5, sink_speed=ws, dwell_depth=dwell) == 0
    # rising by w_s |dt| and by W |dt| (W is downward, time runs backward)
    assert st.z[0] == pytest.approx(300.0 - 5 * (ws + 1e-3) * 600.0, abs=1e-9)
    assert O.advance(fs, st, dt, 200, sink_speed=ws, dwell_depth=dwell) == 0
    assert st.z[0] == dwell and st.status[0] == 0


def test_sampling_alone_leaves_the_trajectory_unchanged():
    rng = np.random.default_rng(4)
    X = np.linspace(0.0, 1e5, 11)
    Y = np.linspace(0.0, 1e5, 9)
    Z = np.linspace(5.0, 5500.0, 12)
    times = np.array([0.0, 5 * DAY])
    shape = (2, Z.size, Y.size, X.size)
    U, V, W = (rng.normal(0, s, shape) for s in (0.3, 0.3, 1e-4))
    tr = rng.normal(10, 3, shape).astype(np.float32)
    fs = O.OracleFieldSet(X, Y, Z, times, U, V, W, tracer=tr)
    p0 = (rng.uniform(2e4, 8e4, 50), rng.uniform(2e4, 8e4, 50), rng.uniform(100, 5000, 50))
    s1 = O.make_state(*p0)
    s2 = O.make_state(*p0)
    assert O.advance(fs, s1, 600.0, 200) == 0
    assert O.advance(fs, s2, 600.0, 200, sample=True) == 0
    assert np.array_equal(s1.x, s2.x) and np.array_equal(s1.z, s2.z)
    assert np.array_equal(s1.status, s2.status)
    assert np.isfinite(s2.temp[s2.status == 0]).all()


def test_behaviour_needs_a_tracer_to_sample():
    fs, *_ = _box()
    st = O.make_state([5e4], [5e4], [100.0])
    assert O.advance(fs, st, 60.0, 1, sample=True) == -1
