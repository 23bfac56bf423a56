"""Trajectory files: NetCDF following the CF-1.6 Discrete Sampling Geometries
conventions for trajectories, in the indexed ragged array representation the
paper's ParticleFile writes (Sect. 3.5): because particles are deleted during a
run, every variable is one long vector over observations, and each observation
names its trajectory through ``trajectory_index``.

Host-side I/O over the output records the library keeps on the device (one
record per output time); the file is written in the classic NetCDF format
(64-bit offsets) with scipy, so nothing beyond the image is needed.
"""

from __future__ import annotations

from typing import Dict, Optional, Sequence

import numpy as np

# variables written per observation when the records hold them, with CF attributes
_POSITION = {
    True: {"lon": dict(standard_name="longitude", units="degrees_east", long_name="longitude"),
           "lat": dict(standard_name="latitude", units="degrees_north", long_name="latitude")},
    False: {"lon": dict(units="m", long_name="x (flat mesh)"),
            "lat": dict(units="m", long_name="y (flat mesh)")},
}
_DEPTH = dict(standard_name="depth", units="m", positive="down", long_name="depth")


def write_indexed(path: str, records: Dict[str, np.ndarray], times: Sequence[float],
                  ids: np.ndarray, spherical: bool = True,
                  time_units: str = "seconds since 2000-01-01 00:00:00",
                  tracer_units: str = "degree_Celsius", title: str = "particle trajectories",
                  alive_only: bool = True) -> int:
    """Write ``records`` (arrays of shape [nrec, nper], as returned by
    ParticleSet.records(): lon, lat, status and optionally depth, temp, age) taken
    at ``times`` (one per record) for the particles ``ids`` (nper) to ``path``.
    An observation is written for every (record, particle) whose status is 0 at
    that record (a particle deleted during a segment is not in the set at its end),
    or for all of them when ``alive_only`` is false.  Returns the number of
    observations."""
    from scipy.io import netcdf_file

    lon = np.asarray(records["lon"])
    nrec, nper = lon.shape
    times = np.asarray(times, dtype=np.float64)
    ids = np.asarray(ids)
    if times.shape != (nrec,) or ids.shape != (nper,):
        raise ValueError(f"need {nrec} record times and {nper} particle ids")
    keep = (np.asarray(records["status"]) == 0) if alive_only else np.ones((nrec, nper), bool)
    rec_idx, par_idx = np.nonzero(keep)  # record-major: observations in time order
    nobs = int(rec_idx.size)
    traj_used = np.unique(par_idx)
    slot = np.full(nper, -1, np.int64)
    slot[traj_used] = np.arange(traj_used.size)

    f = netcdf_file(path, "w", version=2)
    try:
        f.Conventions = "CF-1.6"
        f.featureType = "trajectory"
        f.title = title
        f.source = "paper_1707_05163_amd (GPU Lagrangian particle advection)"
        f.createDimension("obs", nobs)
        f.createDimension("traj", int(traj_used.size))
        v = f.createVariable("trajectory", "i4", ("traj",))
        v[:] = ids[traj_used].astype(np.int32)
        v.cf_role = "trajectory_id"
        v.long_name = "particle id"
        v = f.createVariable("trajectory_index", "i4", ("obs",))
        v[:] = slot[par_idx].astype(np.int32)
        v.instance_dimension = "traj"
        v.long_name = "index of the trajectory (traj dimension) of this observation"
        v = f.createVariable("time", "f8", ("obs",))
        v[:] = times[rec_idx]
        v.standard_name = "time"
        v.units = time_units
        v.long_name = "time"
        coords = "time lat lon"
        for name, attrs in _POSITION[bool(spherical)].items():
            v = f.createVariable(name, "f8", ("obs",))
            v[:] = np.asarray(records[name])[rec_idx, par_idx]
            for k, a in attrs.items():
                setattr(v, k, a)
        if "depth" in records:
            v = f.createVariable("z", "f8", ("obs",))
            v[:] = np.asarray(records["depth"])[rec_idx, par_idx]
            for k, a in _DEPTH.items():
                setattr(v, k, a)
            coords += " z"
        if "temp" in records:
            v = f.createVariable("temp", "f8", ("obs",))
            v[:] = np.asarray(records["temp"])[rec_idx, par_idx]
            v.units = tracer_units
            v.long_name = "tracer sampled along the trajectory"
            v.coordinates = coords
        if "age" in records:
            v = f.createVariable("age", "f8", ("obs",))
            v[:] = np.asarray(records["age"])[rec_idx, par_idx]
            v.units = "s"
            v.long_name = "time lived at the dwelling depth"
            v.coordinates = coords
        if not alive_only:
            v = f.createVariable("status", "i1", ("obs",))
            v[:] = np.asarray(records["status"])[rec_idx, par_idx].astype(np.int8)
            v.long_name = "status bits (1 out of bounds, 2 land, 4 deleted, 8 aged)"
            v.coordinates = coords
    finally:
        f.close()
    return nobs


def record_times(t_start: float, runtime: float, outputdt: float, dt: float,
                 first: bool = True) -> np.ndarray:
    """Times of the records an execute call takes: the start (first call only),
    then the end of every output interval, the last one at start + runtime (in the
    direction of dt)."""
    sg = 1.0 if dt > 0 else -1.0
    out = [t_start] if first else []
    if outputdt <= 0:
        ends = [runtime]
    else:
        n = int(np.ceil(runtime / outputdt - 1e-9))
        ends = [min((k + 1) * outputdt, runtime) for k in range(n)]
    out += [t_start + sg * e for e in ends]
    return np.asarray(out, dtype=np.float64)
