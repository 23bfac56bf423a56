"""The CF-1.6 indexed-ragged trajectory writer (the ParticleFile of Sect. 3.5),
checked on records from the FP64 oracle: CF attributes, the indexed layout, and
that every observation reads back as the record it came from."""

import numpy as np
from scipy.io import netcdf_file

from oracle import oracle as O
from paper_1707_05163_amd.particlefile import record_times, write_indexed
from synthetic import configs as SC

DAY = 86400.0


def _oracle_records(w, maxage):
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0, w.depth0, t_org=w.t0)
    m = w.meta
    rt = w.nsteps * abs(w.dt)
    recs = O.run(ofs, st, w.dt, rt, DAY, sink_speed=m["sink_speed"],
                 dwell_depth=m["dwell_depth"], maxage=maxage, sample=True)
    keys = ["lon", "lat", "depth", "status", "temp", "age"]
    out = {k: np.stack([r[k] for r in recs]) for k in keys}
    return out, record_times(w.t0, rt, DAY, w.dt)


def test_indexed_file_round_trip(tmp_path):
    w = SC.foram_footprint(nx=40, ny=36, nz=12, n_particles=60, dt=-3600.0, days=20)
    recs, times = _oracle_records(w, maxage=5 * DAY)
    assert times.size == recs["lon"].shape[0] == 21
    assert times[0] == w.t0 and times[-1] == w.t0 - 20 * DAY
    path = str(tmp_path / "traj.nc")
    ids = np.arange(w.n)
    nobs = write_indexed(path, recs, times, ids, spherical=True)
    alive = recs["status"] == 0
    assert nobs == int(alive.sum())
    with netcdf_file(path, "r", mmap=False) as f:
        assert f.Conventions == b"CF-1.6" and f.featureType == b"trajectory"
        assert f.dimensions["obs"] == nobs
        traj = f.variables["trajectory"][:].copy()
        assert f.variables["trajectory"].cf_role == b"trajectory_id"
        ti = f.variables["trajectory_index"][:].copy()
        assert f.variables["trajectory_index"].instance_dimension == b"traj"
        t = f.variables["time"][:].copy()
        lon, lat, z = (f.variables[k][:].copy() for k in ("lon", "lat", "z"))
        temp, age = f.variables["temp"][:].copy(), f.variables["age"][:].copy()
        assert f.variables["z"].positive == b"down"
        assert f.variables["lon"].units == b"degrees_east"
    # every observation is the record value of its particle at its time
    rec_of_time = {float(tt): k for k, tt in enumerate(times)}
    for o in range(nobs):
        p = int(traj[ti[o]])
        k = rec_of_time[float(t[o])]
        assert recs["status"][k, p] == 0
        assert lon[o] == recs["lon"][k, p] and lat[o] == recs["lat"][k, p]
        assert z[o] == recs["depth"][k, p] and age[o] == recs["age"][k, p]
        assert temp[o] == recs["temp"][k, p] or (np.isnan(temp[o]) and k == 0)
    # per trajectory: times run in the direction of the run, one per record alive
    for j, p in enumerate(traj):
        tt = t[ti == j]
        assert (np.diff(tt) < 0).all() and tt.size == int(alive[:, p].sum())
    # particles deleted at maxage stop appearing
    aged = (recs["status"][-1] & O.ST_AGED) != 0
    assert aged.any()


def test_all_observations_and_flat_mesh(tmp_path):
    recs = {"lon": np.arange(6.0).reshape(2, 3), "lat": np.ones((2, 3)),
            "status": np.array([[0, 0, 0], [0, 4, 0]], np.uint8)}
    path = str(tmp_path / "flat.nc")
    n = write_indexed(path, recs, [0.0, 10.0], np.array([0, 5, 10]), spherical=False,
                      alive_only=False)
    assert n == 6
    with netcdf_file(path, "r", mmap=False) as f:
        assert f.variables["lon"].units == b"m"
        assert list(f.variables["status"][:]) == [0, 0, 0, 0, 4, 0]
        assert list(f.variables["trajectory"][:]) == [0, 5, 10]
    assert write_indexed(str(tmp_path / "alive.nc"), recs, [0.0, 10.0],
                         np.array([0, 5, 10]), spherical=False) == 5
