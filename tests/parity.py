"""Helpers for parity tests: run a workload through the HIP C ABI and through the
FP64 oracle on the same seeded inputs, then compare record by record.

Comparison rule for FP64 positions: |gpu - oracle| <= 1e-9 * max(|oracle|, extent)
per coordinate, statuses and cell indices equal.  A status or index mismatch is
accepted only where the oracle's point is within 1e-9 (relative to the extent) of a
cell face or of the domain edge, and the oracle's own cell search applied to the GPU
position then returns the GPU's index; such cases are counted, and none is allowed
unless a test says how many (none has been observed).
"""

from __future__ import annotations

import sys
from typing import Optional

import numpy as np

from oracle import oracle as O

REL = 1e-9


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_fieldset(w):
    return O.OracleFieldSet.from_workload(w)


def run_oracle(w, fs=None, ids=None, runtime=None, outputdt=None, Kh=None, policy=0,
               nthreads=0):
    fs = fs or oracle_fieldset(w)
    ids = np.arange(w.n) if ids is None else np.asarray(ids)
    st = O.make_state(w.lon0[ids], w.lat0[ids], None if w.depth0 is None else w.depth0[ids],
                      pid=ids.astype(np.uint32), t_org=w.t0)
    rt = w.nsteps * w.dt if runtime is None else runtime
    od = w.outputdt if outputdt is None else outputdt
    recs = O.run(fs, st, w.dt, rt, od, Kh=w.Kh if Kh is None else Kh, run_id=w.run_id,
                 policy=policy, nthreads=nthreads)
    return recs, st


def run_gpu(w, dtype="f32", capacity=None, stride=1, sort_every=1, runtime=None, outputdt=None,
            Kh=None, recovery="delete", fs=None):
    from paper_1707_05163_amd import FieldSet, ParticleSet
    fs = fs or FieldSet.from_workload(w, dtype=dtype, capacity=capacity)
    ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0, t0=w.t0)
    rt = w.nsteps * w.dt if runtime is None else runtime
    od = w.outputdt if outputdt is None else outputdt
    ps.execute(rt, w.dt, od, recovery=recovery, Kh=w.Kh if Kh is None else Kh,
               run_id=w.run_id, output_stride=stride, sort_every=sort_every)
    recs = ps.records()
    counts, status = ps.status()
    return ps, fs, recs, counts, status


def _near_face(x, axis, tol):
    """True where x lies within tol of a node of the axis (or outside it)."""
    idx = np.searchsorted(axis, x)
    lo = np.abs(x - axis[np.clip(idx - 1, 0, axis.size - 1)])
    hi = np.abs(x - axis[np.clip(idx, 0, axis.size - 1)])
    return (np.minimum(lo, hi) <= tol) | (x < axis[0]) | (x > axis[-1])


def compare_record(g: dict, o: dict, grid, extent: float, label: str = "", ofs=None,
                   max_exempt: int = 0):
    """Compare one GPU record (arrays over the recorded ids) with the oracle's record
    of the same ids.  Returns the number of exempted particles, which must not exceed
    max_exempt (none has been observed on any workload, so the default is 0)."""
    tolx = REL * np.maximum(np.abs(o["lon"]), extent)
    toly = REL * np.maximum(np.abs(o["lat"]), extent)
    dx = np.abs(g["lon"] - o["lon"])
    dy = np.abs(g["lat"] - o["lat"])
    pos_ok = (dx <= tolx) & (dy <= toly)
    if "depth" in o:
        dz = np.abs(g["depth"] - o["depth"])
        pos_ok &= dz <= REL * np.maximum(np.abs(o["depth"]), extent)
    st_ok = g["status"] == o["status"]
    idx_ok = (g["ci"] == o["ci"]) & (g["cj"] == o["cj"])
    if "ck" in o:
        idx_ok &= g["ck"] == o["ck"]
    bad = ~(pos_ok & st_ok & idx_ok)
    nbad = int(bad.sum())
    if nbad == 0:
        return 0
    # exemption: the oracle's point sits on a decision boundary
    near = _near_face(o["lon"], grid.lon, 10 * REL * (grid.lon[-1] - grid.lon[0]))
    near |= _near_face(o["lat"], grid.lat, 10 * REL * (grid.lat[-1] - grid.lat[0]))
    if "depth" in o:
        near |= _near_face(o["depth"], grid.depth, 10 * REL * (grid.depth[-1] - grid.depth[0]))
    ex = bad & near & pos_ok
    if ofs is not None and ex.any():
        ci, cj, _ = ofs.cell_indices(g["lon"][ex], g["lat"][ex])
        assert np.array_equal(ci, g["ci"][ex]) and np.array_equal(cj, g["cj"][ex]), label
    remaining = bad & ~ex
    if remaining.any():
        k = np.flatnonzero(remaining)[:5]
        detail = [(int(i), g["lon"][i], o["lon"][i], g["lat"][i], o["lat"][i], int(g["status"][i]),
                   int(o["status"][i]), int(g["ci"][i]), int(o["ci"][i]), int(g["cj"][i]),
                   int(o["cj"][i])) for i in k]
        raise AssertionError(f"{label}: {int(remaining.sum())} mismatches, first: {detail}")
    assert ex.sum() <= max_exempt, f"{label}: {int(ex.sum())} exempt (allowed {max_exempt})"
    return int(ex.sum())


def slice_record(recs: dict, m: int, sel: Optional[np.ndarray] = None) -> dict:
    out = {k: v[m] for k, v in recs.items()}
    if sel is not None:
        out = {k: v[sel] for k, v in out.items()}
    return out
