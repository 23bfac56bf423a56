"""The worked example's kernels (Sect. 3.3: sinking, age with deletion at maxage,
tracer sampling) on the GPU against the FP64 oracle, on the synthetic stand-in
for the foraminifera experiment run backward in time."""

import numpy as np
import pytest

from oracle import oracle as O
from synthetic import configs as SC

from parity import REL, compare_record, log, slice_record

pytestmark = pytest.mark.gpu

DAY = 86400.0


def _compare_behaviour(recs, orecs, label):
    for m, o in enumerate(orecs):
        g_st = recs["status"][m]
        same = g_st == o["status"]
        assert same.mean() > 0.999, label
        # age is a sum of |dt| terms taken in the same order: exact
        assert np.array_equal(recs["age"][m][same], o["age"][same]), f"{label} age rec {m}"
        gt, ot = recs["temp"][m][same], o["temp"][same]
        nan = np.isnan(ot)
        assert np.array_equal(np.isnan(gt), nan), f"{label} temp NaN pattern rec {m}"
        err = np.abs(gt[~nan] - ot[~nan])
        assert (err <= REL * np.maximum(np.abs(ot[~nan]), 30.0)).all(), \
            f"{label} temp rec {m}: max {err.max() if err.size else 0}"


@pytest.mark.parametrize("maxage_days", [30.0, 8.0])
def test_foram_backward_sink_age_sample(maxage_days):
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.foram_footprint(nx=70, ny=60, nz=20, n_particles=3000, dt=-1800.0, days=24)
    m = w.meta
    log(f"foram small: {w.n} particles, {w.nsteps} steps backward, maxage {maxage_days} d")
    fs = FieldSet.from_workload(w)
    ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0, t0=w.t0)
    runtime = w.nsteps * abs(w.dt)
    ps.execute(runtime, w.dt, DAY, output_stride=1, sink_speed=m["sink_speed"],
               dwell_depth=m["dwell_depth"], maxage=maxage_days * DAY, sample=True)
    recs = ps.records()
    assert "temp" in recs and "age" in recs
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0, w.depth0, t_org=w.t0)
    orecs = O.run(ofs, st, w.dt, runtime, DAY, sink_speed=m["sink_speed"],
                  dwell_depth=m["dwell_depth"], maxage=maxage_days * DAY, sample=True)
    assert recs["lon"].shape[0] == len(orecs)
    for k, o in enumerate(orecs):
        compare_record(slice_record(recs, k), o, w.grid, 360.0, label=f"foram rec {k}",
                       ofs=ofs)
    _compare_behaviour(recs, orecs, "foram")
    c, status = ps.status()
    aged = (status & O.ST_AGED) != 0
    log(f"  aged {aged.sum()}, oob {c['oob']}, active {c['active']}")
    assert np.array_equal(aged, (st.status & O.ST_AGED) != 0)
    if maxage_days < 20:
        assert aged.sum() > 0.5 * w.n  # 12 days rising, then 8 days of life
    # the particles that lived reached the dwelling depth exactly
    alive = status == 0
    assert (recs["depth"][-1][alive] == m["dwell_depth"]).all()
    temp, age = ps.behaviour()
    assert np.array_equal(age, st.age)


@pytest.mark.parametrize("cache", [True, False])
def test_sample_only_keeps_the_plain_trajectory(cache):
    """Sampling alone must not change the advection: positions equal to a run
    without it (same kernel family: the cached 3D kernel, or the gather kernel), and
    the samples match the oracle."""
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.foram_footprint(nx=70, ny=60, nz=20, n_particles=2000, dt=-1800.0, days=4)
    w.depth0 = np.linspace(60.0, 3000.0, w.n)
    fs = FieldSet.from_workload(w)
    a = ParticleSet(fs, w.lon0, w.lat0, w.depth0, t0=w.t0)
    b = ParticleSet(fs, w.lon0, w.lat0, w.depth0, t0=w.t0)
    rt = w.nsteps * abs(w.dt)
    a.execute(rt, w.dt, DAY, stencil_cache=cache)
    b.execute(rt, w.dt, DAY, sample=True, stencil_cache=cache)
    ga, gb = a.get(), b.get()
    assert np.array_equal(ga["lon"], gb["lon"]) and np.array_equal(ga["depth"], gb["depth"])
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0, w.depth0, t_org=w.t0)
    O.run(ofs, st, w.dt, rt, DAY, sample=True)
    temp, _ = b.behaviour()
    ok = st.status == 0
    assert np.allclose(temp[ok], st.temp[ok], rtol=1e-9, atol=1e-9)


def test_cached_and_gather_behaviour_agree():
    """The worked example's kernels in the cached 3D kernel and in the gather kernel:
    the same statuses and ages, positions and samples to the FP64 tolerance."""
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.foram_footprint(nx=70, ny=60, nz=20, n_particles=3000, dt=-1800.0, days=22)
    w.depth0 = np.linspace(60.0, 3000.0, w.n)  # reach the dwelling depth at different times
    m = w.meta
    fs = FieldSet.from_workload(w)
    out = []
    for cache in (True, False):
        ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0, t0=w.t0)
        ps.execute(w.nsteps * abs(w.dt), w.dt, DAY, sink_speed=m["sink_speed"],
                   dwell_depth=m["dwell_depth"], maxage=10 * DAY, sample=True,
                   stencil_cache=cache)
        out.append((ps.get(), ps.status()[1], ps.behaviour()))
    (ga, sa, (ta, aa)), (gb, sb, (tb, ab)) = out
    assert np.array_equal(sa, sb) and np.array_equal(aa, ab)
    ok = sa == 0
    assert ok.sum() > 0 and (sa != 0).sum() > 0
    for k in ("lon", "lat", "depth"):
        assert np.allclose(ga[k][ok], gb[k][ok], rtol=1e-9, atol=1e-9 * 360.0), k
    assert np.allclose(ta[ok], tb[ok], rtol=1e-9, atol=1e-9)


def test_behaviour_argument_errors():
    from paper_1707_05163_amd import FieldSet, ParticleSet, execute_batch
    from paper_1707_05163_amd._lib import LPError
    w = SC.cfg1_global_eddies(nx=72, ny=36, nt=30, n_particles=100, nsteps=288)
    fs = FieldSet.from_workload(w)  # no tracer
    ps = ParticleSet(fs, w.lon0, w.lat0)
    with pytest.raises(LPError):
        ps.execute(3600.0, 300.0, sample=True)          # no tracer pushed
    with pytest.raises(LPError):
        ps.execute(3600.0, 300.0, sink_speed=1e-3)      # sinking needs depth
    with pytest.raises(LPError):
        ps.execute(3600.0, 300.0, maxage=-1.0)
    with pytest.raises(LPError):
        ps.execute(3600.0, 300.0, maxage=DAY, kernel="rkf45")
    o = ParticleSet.opts(maxage=DAY)
    with pytest.raises(LPError):
        execute_batch([ps], 3600.0, 300.0, 0.0, [o])
    with pytest.raises(LPError):                        # no snapshot at that time
        fs.push_tracer(123.0, np.zeros((w.grid.ny, w.grid.nx), np.float32))
    assert ps.status()[0]["particle_steps"] == 0
    # age without a tracer is fine (2D: every step ages)
    ps.execute(3600.0, 300.0, maxage=1800.0)
    c, st = ps.status()
    assert ((st & O.ST_AGED) != 0).sum() == c["n"] - c["oob"] - c["land"]


def test_write_trajectories_from_gpu_records(tmp_path):
    from scipy.io import netcdf_file
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.foram_footprint(nx=70, ny=60, nz=20, n_particles=500, dt=-1800.0, days=16)
    m = w.meta
    fs = FieldSet.from_workload(w)
    ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0, t0=w.t0)
    for _ in range(2):  # two calls: the record times carry on
        ps.execute(8 * DAY, w.dt, DAY, output_stride=2, sink_speed=m["sink_speed"],
                   dwell_depth=m["dwell_depth"], maxage=2 * DAY, sample=True)
    recs = ps.records()
    path = str(tmp_path / "gpu.nc")
    nobs = ps.write_trajectories(path)
    assert nobs == int((recs["status"] == 0).sum())
    with netcdf_file(path, "r", mmap=False) as f:
        t = f.variables["time"][:].copy()
        assert f.dimensions["traj"] == int((recs["status"] == 0).any(axis=0).sum())
        assert set(np.unique(t)) <= set(w.t0 - DAY * np.arange(17))
        assert (f.variables["trajectory"][:] % 2 == 0).all()
