"""Adaptive RKF45 (the Runge-Kutta-Fehlberg option of Sect. 2.1.1) on the GPU
against the FP64 oracle: positions to the FP64 parity tolerance, and the integer
outcomes of the step control (every particle's step exponent, the accepted and
retried attempt counts) exactly."""

import numpy as np
import pytest

from oracle import oracle as O
from synthetic import configs as SC

from parity import compare_record, log, slice_record

pytestmark = pytest.mark.gpu


def _check_exps(ps, st, exempt_ok=0):
    g = ps.step_exponents()
    bad = np.flatnonzero(g != st.exps)
    log(f"  step exponents: {np.bincount(g - g.min()) if g.size else []} (min {g.min()}), "
        f"{bad.size} differ")
    assert bad.size <= exempt_ok, bad[:10]


def _run(w, dt, runtime, outputdt, tol, emin, emax, t0=0.0, dtype="f32", fs=None, ofs=None,
         cache=True):
    from paper_1707_05163_amd import FieldSet, ParticleSet
    fs = fs or FieldSet.from_workload(w, dtype=dtype)
    ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0, t0=t0)
    ps.execute(runtime, dt, outputdt, output_stride=1, kernel="rkf45", tol=tol, min_exp=emin,
               max_exp=emax, stencil_cache=cache)
    ofs = ofs or O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0, w.depth0, t_org=t0)
    orecs = O.run(ofs, st, dt, runtime, outputdt, scheme=O.SCHEME_RKF45, tol=tol, emin=emin,
                  emax=emax)
    return ps, ps.records(), orecs, ofs, st


def _compare(ps, recs, orecs, ofs, st, w, extent, label):
    ex = 0
    for m, o in enumerate(orecs):
        ex += compare_record(slice_record(recs, m), o, w.grid, extent, label=f"{label} rec {m}",
                             ofs=ofs)
    c, _ = ps.status()
    log(f"  {label}: accepted {c['particle_steps']} (oracle {st.psteps}), retried "
        f"{c['rejected_steps']} (oracle {st.rejected})")
    if ex == 0:
        assert c["particle_steps"] == st.psteps
        assert c["rejected_steps"] == st.rejected
    _check_exps(ps, st, exempt_ok=ex)
    return c


@pytest.mark.parametrize("cache", [True, False])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rkf45_cfg0_rotation(dtype, cache):
    w = SC.cfg0_solid_body(n_particles=3000, nsteps=1440)
    if dtype == "f32":  # both sides read the same float32 values
        w.fields.U = w.fields.U.astype(np.float32)
        w.fields.V = w.fields.V.astype(np.float32)
    log(f"rkf45 cfg0 {dtype} cache={cache}")
    ps, recs, orecs, ofs, st = _run(w, w.dt, w.nsteps * w.dt, 14400.0, 1e-6, -4, 6,
                                    dtype=dtype, cache=cache)
    _compare(ps, recs, orecs, ofs, st, w, 1e5, "cfg0")


@pytest.mark.parametrize("tol,emin,emax,cache", [(1e-8, -5, 3, True), (1e-8, -5, 3, False),
                                                (1e-3, -6, 5, True)])
def test_rkf45_cfg1_small(tol, emin, emax, cache):
    """Periodic snapshots, spherical mesh, land: retries, growth and the floor all
    occur at the tighter tolerance."""
    w = SC.cfg1_global_eddies(nx=144, ny=72, nt=30, n_particles=5000, nsteps=288)
    log(f"rkf45 cfg1 small tol {tol} cache={cache}")
    ps, recs, orecs, ofs, st = _run(w, 7200.0, 4 * 86400.0, 86400.0, tol, emin, emax,
                                    cache=cache)
    c = _compare(ps, recs, orecs, ofs, st, w, 360.0, "cfg1")
    if tol < 1e-6:
        assert c["rejected_steps"] > 0


def test_rkf45_backward_cfg1():
    w = SC.cfg1_global_eddies(nx=144, ny=72, nt=30, n_particles=4000, nsteps=288)
    log("rkf45 backward cfg1")
    ps, recs, orecs, ofs, st = _run(w, -3600.0, 2 * 86400.0, 43200.0, 1e-7, -5, 4,
                                    t0=10 * 86400.0)
    _compare(ps, recs, orecs, ofs, st, w, 360.0, "back")
    assert ps.status()[0]["time"] == 8 * 86400.0


def test_rkf45_3d_through_the_ring():
    """3D, non-periodic snapshots streamed through a three-slot ring one day at a
    time (each day's stage times bracketed per lane among the resident slots)."""
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.cfg2_global_3d(nx=180, ny=90, nz=20, nt=4, n_particles=3000, nsteps=432)
    log("rkf45 3d ring")
    fs = FieldSet.from_workload(w, capacity=3, push=False, time_period=0.0)
    fs.push_snapshot(w.fields.times[0], *w.fields.snapshot(0))
    fs.push_snapshot(w.fields.times[1], *w.fields.snapshot(1))
    ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0)
    tol, emin, emax = 1e-4, -4, 4
    for d in range(3):
        ps.execute(86400.0, 1800.0, 43200.0, output_stride=1, kernel="rkf45", tol=tol,
                   min_exp=emin, max_exp=emax)
        if d + 2 < w.fields.nt:
            fs.push_snapshot(w.fields.times[d + 2], *w.fields.snapshot(d + 2))
    recs = ps.records()
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0, w.depth0)
    orecs = O.run(ofs, st, 1800.0, 3 * 86400.0, 43200.0, scheme=O.SCHEME_RKF45, tol=tol,
                  emin=emin, emax=emax)
    _compare(ps, recs, orecs, ofs, st, w, 360.0, "3d ring")


def test_rkf45_full_grid_sampled():
    """The benchmark's launch configuration (0.25 degree global grid, 1M particles,
    one-day output segments) for three days; the oracle follows every 997th
    particle."""
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.cfg1_global_eddies(n_particles=1_000_000, nsteps=864)
    log("rkf45 cfg1 full grid, 1M particles, 3 days")
    fs = FieldSet.from_workload(w)
    ps = ParticleSet(fs, w.lon0, w.lat0)
    tol, emin, emax = 1e-3, -6, 5
    ps.execute(3 * 86400.0, w.dt, 86400.0, kernel="rkf45", tol=tol, min_exp=emin, max_exp=emax)
    g = ps.get()
    _, gst = ps.status()
    ge = ps.step_exponents()
    ids = np.arange(0, w.n, 997)
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0[ids], w.lat0[ids], pid=ids.astype(np.uint32))
    O.run(ofs, st, w.dt, 3 * 86400.0, 86400.0, scheme=O.SCHEME_RKF45, tol=tol, emin=emin,
          emax=emax, first_record=False)
    same = gst[ids] == st.status
    assert same.mean() > 0.999
    ok = same & (st.status == 0)
    tolx = 1e-9 * 360.0
    assert np.abs(g["lon"][ids][ok] - st.x[ok]).max() <= tolx
    assert np.abs(g["lat"][ids][ok] - st.y[ok]).max() <= tolx
    assert (ge[ids][ok] == st.exps[ok]).mean() > 0.999


def test_rkf45_argument_errors():
    from paper_1707_05163_amd import FieldSet, ParticleSet, execute_batch
    from paper_1707_05163_amd._lib import LPError
    w = SC.cfg1_global_eddies(nx=72, ny=36, nt=30, n_particles=100, nsteps=288)
    fs = FieldSet.from_workload(w)
    ps = ParticleSet(fs, w.lon0, w.lat0)
    with pytest.raises(LPError):
        ps.execute(3600.0, 300.0, kernel="rkf45", Kh=10.0)
    with pytest.raises(LPError):
        ps.execute(3600.0, 300.0, kernel="rkf45", tol=0.0)
    with pytest.raises(LPError):
        ps.execute(3600.0, 300.0, kernel="rkf45", min_exp=1)
    with pytest.raises(LPError):
        ps.execute(3600.0, 300.0, kernel="rkf45", max_exp=31)
    ps2 = ParticleSet(fs, w.lon0, w.lat0, t0=1e12)
    with pytest.raises(LPError):  # the floor step cannot move a clock at 1e12 s
        ps2.execute(3600.0, 1e-3 * 2 ** 10, kernel="rkf45", min_exp=-30)
    o = ParticleSet.opts(kernel="rkf45")
    with pytest.raises(LPError):
        execute_batch([ps], 3600.0, 300.0, 0.0, [o])
    # nothing ran: the set is still at its start
    assert ps.status()[0]["particle_steps"] == 0
