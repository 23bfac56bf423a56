"""Pins of the oracle's adaptive Runge-Kutta-Fehlberg integrator (the RKF45 option
named in Sect. 2.1.1).

The paper names the scheme and nothing more; the reading taken here (Fehlberg 4(5)
pair, fourth-order solution carried, error in metres, step |dt| 2^e halved above
tol and doubled at or below tol/32, last step cut to the end of the interval) is
checked against what the mathematics fixes:

* the local errors of the fourth- and fifth-order solutions shrink as h^5 and h^6
  against an independent high-accuracy solution (scipy's DOP853) of a field that
  the interpolation reproduces exactly (a wrong tableau entry breaks an order);
* the embedded estimate approaches the true local error of the carried solution;
* closed forms of the controller: uniform flow doubles the step up to the cap,
  an unreachable tolerance halves it to the floor once and stays there;
* solid-body rotation stays on its exact circle within the accumulated tolerance,
  and a forward-then-backward run returns to the start;
* a step-by-step replay of the stated control rule on the attempt primitive gives
  the driver's results bit for bit.
"""

from __future__ import annotations

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O
from synthetic import configs as SC


def _bilinear_flow(rng, gamma=2e-5):
    """U, V = (bilinear in x, y) * (1 + gamma t) on a non-uniform flat grid with two
    snapshots (t = 0 and 2e5 s): reproduced exactly by bilinear-in-space,
    linear-in-time interpolation.  Returns the field set and the analytic RHS."""
    X = np.sort(np.concatenate([[0.0, 2e5], rng.uniform(0.0, 2e5, 9)]))
    Y = np.sort(np.concatenate([[0.0, 2e5], rng.uniform(0.0, 2e5, 7)]))
    cu = np.array([0.3, 2e-6, -4e-6, 3e-11])
    cv = np.array([-0.2, 5e-6, 1e-6, -2e-11])

    def B(c, x, y):
        return c[0] + c[1] * x + c[2] * y + c[3] * x * y

    XX, YY = np.meshgrid(X, Y)
    T = np.array([0.0, 2e5])
    U = np.stack([B(cu, XX, YY) * (1 + gamma * t) for t in T])
    V = np.stack([B(cv, XX, YY) * (1 + gamma * t) for t in T])
    fs = O.OracleFieldSet(X, Y, None, T, U, V)

    def rhs(t, p):
        return [B(cu, p[0], p[1]) * (1 + gamma * t), B(cv, p[0], p[1]) * (1 + gamma * t)]

    return fs, rhs


def _exact(rhs, t0, h, p0):
    sol = solve_ivp(rhs, (t0, t0 + h), p0[:2], method="DOP853", rtol=3e-14, atol=1e-12)
    assert sol.success
    return sol.y[:, -1]


def test_rkf45_local_orders_four_and_five():
    rng = np.random.default_rng(3)
    fs, rhs = _bilinear_flow(rng)
    p0 = np.array([8e4, 9e4, 0.0])
    t0 = 1.3e4
    e4, e5 = [], []
    for h in [8e3, 4e3, 2e3]:
        rc, p4, p5, err = fs.rkf45_attempt(t0, h, p0)
        assert rc == 0
        ex = _exact(rhs, t0, h, p0)
        e4.append(np.linalg.norm(p4[:2] - ex))
        e5.append(np.linalg.norm(p5[:2] - ex))
        # the estimate is the difference of the two solutions
        assert np.allclose(err[:2], p5[:2] - p4[:2], rtol=1e-6, atol=1e-9)
    r4 = [e4[0] / e4[1], e4[1] / e4[2]]
    r5 = [e5[0] / e5[1], e5[1] / e5[2]]
    # local error C h^5 (ratio 32 per halving) and C' h^6 (ratio 64)
    assert all(24.0 < r < 40.0 for r in r4), r4
    assert all(45.0 < r < 90.0 for r in r5), r5
    assert e5[-1] > 1e-9  # well above the reference solution's own error


def test_rkf45_estimate_tracks_true_local_error():
    rng = np.random.default_rng(5)
    fs, rhs = _bilinear_flow(rng)
    for p0, t0 in [(np.array([3e4, 1.5e5, 0.0]), 0.0), (np.array([1.2e5, 4e4, 0.0]), 5e4)]:
        h = 2e3
        rc, p4, p5, err = fs.rkf45_attempt(t0, h, p0)
        assert rc == 0
        true = _exact(rhs, t0, h, p0) - p4[:2]
        assert np.linalg.norm(err[:2] - true) < 0.2 * np.linalg.norm(true)
        # metres on a flat mesh: the Euclidean length
        assert fs.metres(p0[1], err) == pytest.approx(np.linalg.norm(err[:2]), rel=1e-15)


def _uniform(u, v, n=21, spacing=1e4):
    X = spacing * np.arange(n)
    U = np.full((1, n, n), u)
    V = np.full((1, n, n), v)
    return O.OracleFieldSet(X, X.copy(), None, [0.0], U, V)


def test_rkf45_uniform_flow_doubles_to_the_cap():
    """Equal slopes: zero error, so every full step doubles the next one until 2^emax;
    the accepted-step count and the end point follow in closed form."""
    fs = _uniform(0.5, -0.25)
    dt, n, emax = 60.0, 500, 4
    st = O.make_state([5e4, 7e4], [1.5e5, 1.2e5])
    assert O.advance(fs, st, dt, n, scheme=O.SCHEME_RKF45, tol=1e-3, emax=emax) == 0
    # steps 1, 2, 4, ..., 2^emax (in units of dt), then 2^emax until the cut step
    left, steps, e = n, 0, 0
    while left > 0:
        k = min(2 ** e, left)
        left -= k
        steps += 1
        if k == 2 ** e and e < emax:
            e += 1
    assert st.psteps == 2 * steps and st.rejected == 0
    assert (st.exps == emax).all()
    T = n * dt
    assert np.allclose(st.x, [5e4 + 0.5 * T, 7e4 + 0.5 * T], rtol=0, atol=1e-9)
    assert np.allclose(st.y, [1.5e5 - 0.25 * T, 1.2e5 - 0.25 * T], rtol=0, atol=1e-9)


def test_rkf45_unreachable_tolerance_sits_at_the_floor():
    """A tolerance no step can meet on a nonlinear field (the estimate is never
    zero there): the first step is halved down to 2^emin, one retry per halving,
    then every step is taken at the floor and never grows."""
    rng = np.random.default_rng(9)
    fs, _ = _bilinear_flow(rng)
    n, dt, nsteps, emin = 20, 2000.0, 12, -3
    st = O.make_state(rng.uniform(4e4, 7e4, n), rng.uniform(4e4, 7e4, n))
    assert O.advance(fs, st, dt, nsteps, scheme=O.SCHEME_RKF45, tol=1e-30, emin=emin) == 0
    assert (st.status == 0).all()
    assert (st.exps == emin).all()
    assert st.rejected == n * (-emin)
    assert st.psteps == n * nsteps * 2 ** (-emin)


def test_rkf45_solid_body_stays_on_the_exact_circle():
    """Linear rotation field (reproduced exactly by the interpolation): the exact
    path is Z0 exp(i omega t); the adaptive run stays within the accumulated
    per-step tolerance of it, and tighter tolerances land closer."""
    w = SC.cfg0_solid_body(n_particles=300, nsteps=1440)
    fs = O.OracleFieldSet.from_workload(w)
    c = 5e4 + 5e4j
    z0 = (w.lon0 + 1j * w.lat0) - c
    T = w.nsteps * w.dt
    zt = z0 * np.exp(1j * w.meta["omega"] * T)
    errs = []
    for tol in [1e-2, 1e-5]:
        st = O.make_state(w.lon0, w.lat0)
        assert O.advance(fs, st, w.dt, w.nsteps, scheme=O.SCHEME_RKF45, tol=tol, emax=8) == 0
        assert (st.status == 0).all()
        d = np.abs((st.x + 1j * st.y) - c - zt)
        per = st.psteps / w.n
        assert d.max() <= 2.0 * tol * per
        errs.append(d.max())
    assert errs[1] < errs[0]


def test_rkf45_forward_then_backward_returns_to_start():
    w = SC.cfg0_solid_body(n_particles=200, nsteps=1440)
    fs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0)
    tol = 1e-4
    assert O.advance(fs, st, w.dt, w.nsteps, scheme=O.SCHEME_RKF45, tol=tol) == 0
    fwd = st.psteps
    assert O.advance(fs, st, -w.dt, w.nsteps, scheme=O.SCHEME_RKF45, tol=tol) == 0
    back = np.abs((st.x - w.lon0) + 1j * (st.y - w.lat0))
    assert back.max() <= 4.0 * tol * st.psteps / w.n
    assert st.psteps > fwd


def _replay(fs, p, t_s, t_e, dt, tol, emin, emax, e):
    """The stated control rule, step by step, on the attempt primitive."""
    sg = 1.0 if dt > 0 else -1.0
    t, acc, rej = t_s, 0, 0
    p = np.array(p, dtype=np.float64)
    while t != t_e:
        h = abs(dt) * 2.0 ** e
        rem = (t_e - t) if sg > 0 else (t - t_e)
        cut = h >= rem
        hs = sg * (rem if cut else h)
        rc, p4, _, err = fs.rkf45_attempt(t, hs, p)
        assert rc == 0
        m = fs.metres(p[1], err)
        if m > tol and e > emin:
            e -= 1
            rej += 1
            continue
        acc += 1
        p = p4
        t = t_e if cut else t + hs
        if not cut and m <= tol / 32 and e < emax:
            e += 1
    return p, e, acc, rej


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_rkf45_driver_matches_replay_of_the_rule(sign):
    w = SC.cfg1_global_eddies(nx=144, ny=72, nt=30, n_particles=40, nsteps=288)
    fs = O.OracleFieldSet.from_workload(w)
    t0 = 0.0 if sign > 0 else 86400.0 * 5
    st = O.make_state(w.lon0, w.lat0, t_org=t0)
    dt, tol, emin, emax, n = sign * 7200.0, 1e-8, -5, 3, 24
    assert O.advance(fs, st, dt, n, scheme=O.SCHEME_RKF45, tol=tol, emin=emin,
                     emax=emax) == 0
    assert st.rejected > 0 and (st.exps > 0).any() and (st.exps < 0).any()
    acc_all = rej_all = 0
    for q in range(w.n):
        if st.status[q]:
            continue
        p, e, acc, rej = _replay(fs, [w.lon0[q], w.lat0[q], 0.0], t0, t0 + n * dt, dt, tol,
                                 emin, emax, 0)
        assert p[0] == st.x[q] and p[1] == st.y[q]
        assert e == st.exps[q]
        acc_all += acc
        rej_all += rej
    ok = st.status == 0
    assert ok.sum() > 30
    if ok.all():
        assert (acc_all, rej_all) == (st.psteps, st.rejected)


def test_rkf45_argument_checks():
    fs = _uniform(0.1, 0.0)
    st = O.make_state([5e4], [5e4])
    with pytest.raises(ValueError):
        O.advance(fs, st, 60.0, 10, scheme=O.SCHEME_RKF45, Kh=1.0)
    assert O.advance(fs, st, 60.0, 10, scheme=O.SCHEME_RKF45, tol=0.0) == -1
    assert O.advance(fs, st, 60.0, 10, scheme=O.SCHEME_RKF45, emin=1) == -1
    # a floor step too small to move the clock
    st2 = O.make_state([5e4], [5e4], t_org=1e12)
    assert O.advance(fs, st2, 1e-3, 10, scheme=O.SCHEME_RKF45, emin=-10) == -1
