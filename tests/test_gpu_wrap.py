"""Time-periodic snapshots across the end of the period, and the Brownian term in
time-backward runs, on the GPU against the FP64 oracle.

With a period P and snapshots T_0 .. T_(nt-1), a time in [T_(nt-1), T_0 + P) lies
between the last snapshot and the first one again at T_0 + P; a later time maps
back into the period.  Each run here starts 1.5 days before the end of a 30-day
period and runs 3 days, so every output segment crosses a bracket change and one
of them the wrap itself: in the cached and gather RK4 kernels (whose stage-time
table the host brackets) and in both RKF45 lanes (which bracket their own stage
times on the device).  A backward run crosses the wrap the other way.
"""

from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from synthetic import configs as SC

from parity import compare_record, log, slice_record

pytestmark = pytest.mark.gpu

DAY = 86400.0


def _workload():
    return SC.cfg1_global_eddies(nx=360, ny=180, nt=30, n_particles=4000, nsteps=864)


@pytest.mark.parametrize("lane", ["cached", "gather", "rkf45_gather", "rkf45_cached",
                                  "cached_backward"])
def test_periodic_wrap(lane):
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = _workload()
    assert w.fields.nt == 30 and w.fields.period == 30 * DAY
    backward = lane.endswith("backward")
    t0 = 1.5 * DAY if backward else 28.5 * DAY
    dt = -w.dt if backward else w.dt
    rkf = lane.startswith("rkf45")
    cache = lane in ("cached", "rkf45_cached", "cached_backward")
    log(f"periodic wrap: {lane}, start {t0 / DAY} d, 3 days")
    fs = FieldSet.from_workload(w)
    ps = ParticleSet(fs, w.lon0, w.lat0, t0=t0)
    kw = dict(kernel="rkf45", tol=1e-2, min_exp=-5, max_exp=3) if rkf else {}
    step = 3600.0 if rkf else dt
    ps.execute(3 * DAY, step, DAY, output_stride=1, stencil_cache=cache, **kw)
    recs = ps.records()
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0, t_org=t0)
    okw = dict(scheme=O.SCHEME_RKF45, tol=1e-2, emin=-5, emax=3) if rkf else {}
    orecs = O.run(ofs, st, step, 3 * DAY, DAY, **okw)
    assert recs["lon"].shape[0] == len(orecs) == 4
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, w.grid, 360.0, label=f"{lane} rec {m}",
                       ofs=ofs)
    c, status = ps.status()
    assert np.array_equal(status, st.status)
    assert c["particle_steps"] == st.psteps
    if rkf:
        assert c["rejected_steps"] == st.rejected
        assert np.array_equal(ps.step_exponents(), st.exps)
    # the clock went round the end of the period (past day 30, or back past day 0)
    assert c["time"] == (-1.5 * DAY if backward else 31.5 * DAY)


@pytest.mark.parametrize("mesh", ["flat", "spherical"])
def test_backward_with_brownian_term(mesh):
    """A negative dt with K_h > 0: the kick is sqrt(2 K_h |dt|) N(0, 1) (a NaN from a
    signed dt would send every particle out of the grid)."""
    from paper_1707_05163_amd import FieldSet, ParticleSet
    if mesh == "flat":
        w = SC.cfg3_ensemble(n_runs=1, np_min=4000, np_max=4000, nsteps=288)[0]
        ext = float(w.grid.lon[-1])
        Kh, t0 = w.Kh, 3 * DAY
    else:
        w = SC.cfg1_global_eddies(nx=144, ny=72, nt=30, n_particles=4000, nsteps=288)
        ext = 360.0
        Kh, t0 = 40.0, 5 * DAY
    log(f"backward Brownian on a {mesh} mesh: {w.n} particles")
    fs = FieldSet.from_workload(w)
    ps = ParticleSet(fs, w.lon0, w.lat0, t0=t0)
    ps.execute(DAY, -w.dt, 6 * 3600.0, output_stride=1, Kh=Kh, run_id=5)
    recs = ps.records()
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0, t_org=t0)
    orecs = O.run(ofs, st, -w.dt, DAY, 6 * 3600.0, Kh=Kh, run_id=5)
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, w.grid, ext, label=f"{mesh} rec {m}",
                       ofs=ofs)
    c, status = ps.status()
    assert np.array_equal(status, st.status)
    # the kicks are finite: particles stay active and keep finite positions
    ok = status == 0
    assert c["active"] > 0 and np.isfinite(recs["lon"][-1][ok]).all()
