"""Euler forward, nearest-neighbour interpolation and time-backward execution
against the oracle (the integrator and interpolation alternatives of Sect. 2.1.1,
Sect. 2.3 and the time-backward mode of Sect. 2.2)."""

import numpy as np
import pytest

from oracle import oracle as O
from synthetic import configs as SC

from parity import compare_record, log, slice_record

pytestmark = pytest.mark.gpu


def _run_both(w, dt, runtime, outputdt, kernel="rk4", interp="linear", cache=True,
              dtype="f32", start=None):
    from paper_1707_05163_amd import FieldSet, ParticleSet
    fs = FieldSet.from_workload(w, dtype=dtype)
    t0 = 0.0 if start is None else start
    ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0, t0=t0)
    ps.execute(runtime, dt, outputdt, output_stride=1, kernel=kernel, interp=interp,
               stencil_cache=cache)
    recs = ps.records()
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0, w.depth0, t_org=t0)
    orecs = O.run(ofs, st, dt, runtime, outputdt,
                  scheme=O.SCHEME_EULER if kernel == "euler" else O.SCHEME_RK4,
                  nearest=interp == "nearest")
    return ps, recs, orecs, ofs, st


@pytest.mark.parametrize("cache", [True, False])
def test_euler_cfg0_closed_form(cache):
    w = SC.cfg0_solid_body(n_particles=2000, nsteps=500)
    ps, recs, orecs, ofs, st = _run_both(w, w.dt, w.nsteps * w.dt, 3000.0, kernel="euler",
                                         dtype="f64", cache=cache)
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, w.grid, 1e5, label=f"euler rec {m}")
    z0 = np.abs((w.lon0 - 5e4) + 1j * (w.lat0 - 5e4))
    th = w.meta["omega"] * w.dt
    r = np.abs((recs["lon"][-1] - 5e4) + 1j * (recs["lat"][-1] - 5e4))
    assert np.allclose(r, z0 * (1 + th * th) ** (w.nsteps / 2), rtol=1e-12)


@pytest.mark.parametrize("kernel,interp,cache", [("euler", "linear", True),
                                                 ("rk4", "nearest", True),
                                                 ("rk4", "nearest", False),
                                                 ("euler", "nearest", True)])
def test_cfg1_small_schemes(kernel, interp, cache):
    w = SC.cfg1_global_eddies(nx=144, ny=72, nt=30, n_particles=4000, nsteps=288)
    log(f"cfg1 small {kernel}/{interp} cache={cache}")
    ps, recs, orecs, ofs, st = _run_both(w, w.dt, w.nsteps * w.dt, 6 * 3600.0, kernel, interp,
                                         cache)
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, w.grid, 360.0, label=f"{kernel} rec {m}",
                       ofs=ofs)


def test_euler_3d():
    """Euler forward on the cached 3D kernel: one stage a step, each at a new time, so the
    coefficients the cell carries at the last stage's time advance at every stage (RK4's
    first and third stages skip it)."""
    w = SC.cfg2_global_3d(nx=180, ny=90, nz=20, nt=3, n_particles=4000, nsteps=144)
    ps, recs, orecs, ofs, st = _run_both(w, w.dt, w.nsteps * w.dt, 6 * 3600.0, kernel="euler")
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, w.grid, 360.0, label=f"euler3d rec {m}",
                       ofs=ofs)


def test_nearest_3d():
    w = SC.cfg2_global_3d(nx=180, ny=90, nz=20, nt=3, n_particles=4000, nsteps=144)
    ps, recs, orecs, ofs, st = _run_both(w, w.dt, w.nsteps * w.dt, 6 * 3600.0, interp="nearest")
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, w.grid, 360.0, label=f"nearest3d rec {m}",
                       ofs=ofs)


def test_backward_in_time_cfg1():
    """Forward one day, then backward one day (negative dt), against the oracle."""
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.cfg1_global_eddies(nx=144, ny=72, nt=30, n_particles=4000, nsteps=288)
    fs = FieldSet.from_workload(w)
    ps = ParticleSet(fs, w.lon0, w.lat0, t0=5 * 86400.0)
    ps.execute(86400.0, w.dt, 21600.0, output_stride=1)
    ps.execute(86400.0, -w.dt, 21600.0, output_stride=1)
    recs = ps.records()
    c, _ = ps.status()
    assert c["time"] == 5 * 86400.0 and c["step"] == 576
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0, t_org=5 * 86400.0)
    orecs = O.run(ofs, st, w.dt, 86400.0, 21600.0)
    orecs += O.run(ofs, st, -w.dt, 86400.0, 21600.0, first_record=False)
    assert recs["lon"].shape[0] == len(orecs) == 9
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, w.grid, 360.0, label=f"back rec {m}", ofs=ofs)
    # RK4 forward then backward returns close to the start (the flow is smooth here)
    ok = recs["status"][-1] == 0
    back = np.hypot(recs["lon"][-1][ok] - w.lon0[ok], recs["lat"][-1][ok] - w.lat0[ok])
    assert np.median(back) < 1e-3


def test_backward_through_the_ring_3d():
    """Time-backward through a three-slot ring: load the last snapshots first."""
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.cfg2_global_3d(nx=180, ny=90, nz=20, nt=4, n_particles=3000, nsteps=288)
    fs = FieldSet.from_workload(w, capacity=3, push=False, time_period=0.0)
    for s in (1, 2, 3):
        fs.push_snapshot(w.fields.times[s], *w.fields.snapshot(s))
    t0 = w.fields.times[3]
    ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0, t0=t0)
    ps.execute(2 * 86400.0, -w.dt, 86400.0, output_stride=1)
    recs = ps.records()
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0, w.depth0, t_org=t0)
    orecs = O.run(ofs, st, -w.dt, 2 * 86400.0, 86400.0)
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, w.grid, 360.0, label=f"back3d rec {m}", ofs=ofs)
