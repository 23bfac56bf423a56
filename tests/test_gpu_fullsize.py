"""Parity at the benchmark sizes, in the benchmark's launch configuration (register /
LDS stencil cache, daily output segments, the benchmark's sort cadence and record
stride), on sampled particles the oracle follows one by one: the 0.25 degree global
2D field with 1M particles for the whole 30 days (through the end of the 30-day
period), the 0.1 degree global 3D field with 10M particles for the whole 10 days
with its 11 snapshots streamed through the three-slot ring, and the 64-run
Brownian ensemble in one batched launch per segment (one day)."""

from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from synthetic import configs as SC

from parity import compare_record, log, slice_record

pytestmark = pytest.mark.gpu

DAY = 86400.0


def test_cfg1_full_size_sampled():
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.cfg1_global_eddies()
    days = 30
    log(f"cfg1 full size: {w.n} particles on {w.grid.nx}x{w.grid.ny}, {days} days")
    fs = FieldSet.from_workload(w)
    ps = ParticleSet(fs, w.lon0, w.lat0)
    ps.execute(days * DAY, w.dt, DAY, output_stride=1, sort_every=10, stencil_cache=True)
    recs = ps.records()
    ids = np.arange(0, w.n, 997)
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0[ids], w.lat0[ids], pid=ids.astype(np.uint32))
    orecs = O.run(ofs, st, w.dt, days * DAY, DAY, nthreads=O.max_threads())
    assert recs["lon"].shape[0] == len(orecs) == days + 1
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m, ids), o, w.grid, 360.0, label=f"cfg1 rec {m}",
                       ofs=ofs)
    c, status = ps.status()
    assert np.array_equal(status[ids], st.status)
    assert c["time"] == days * DAY


def test_cfg2_full_size_sampled():
    import torch
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.cfg2_global_3d()
    days = w.fields.nt - 1
    log(f"cfg2 full size: {w.n} particles on {w.grid.nx}x{w.grid.ny}x{w.grid.nz}, {days} days "
        f"through the ring")
    cache = {}
    snaps = [SC.cfg2_snapshot_torch(w, s, "cuda", cache) for s in range(w.fields.nt)]
    del cache
    stride = 100  # the benchmark's record stride
    fs = FieldSet(w.grid.lon, w.grid.lat, w.grid.depth, "spherical", "f32", 3, 0.0)
    ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0)
    fs.push_snapshot(w.fields.times[0], *snaps[0])
    fs.push_snapshot(w.fields.times[1], *snaps[1])
    for d in range(days):
        ps.execute(DAY, w.dt, DAY, output_stride=stride, sort_every=0, stencil_cache=True)
        if d + 2 < w.fields.nt:
            fs.push_snapshot(w.fields.times[d + 2], *snaps[d + 2])
    recs = ps.records()
    torch.cuda.synchronize()
    shape = (w.fields.nt,) + tuple(snaps[0][0].shape)
    U, V, W = (np.empty(shape, np.float32) for _ in range(3))
    for q in range(w.fields.nt):
        U[q], V[q], W[q] = (snaps[q][v].cpu().numpy() for v in range(3))
    del snaps
    ofs = O.OracleFieldSet(w.grid.lon, w.grid.lat, w.grid.depth, w.fields.times, U, V, W,
                           spherical=True)
    sub = 97  # every 97th recorded particle: ids 0 mod 9700
    ids = np.arange(0, w.n, stride * sub)
    assert recs["lon"].shape[0] == days + 1
    st = O.make_state(w.lon0[ids], w.lat0[ids], w.depth0[ids], pid=ids.astype(np.uint32))
    orecs = O.run(ofs, st, w.dt, days * DAY, DAY, nthreads=O.max_threads())
    sel = np.arange(0, recs["lon"].shape[1], sub)
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m, sel), o, w.grid, 360.0, label=f"cfg2 rec {m}",
                       ofs=ofs)
    c, status = ps.status()
    assert np.array_equal(status[ids], st.status)
    assert c["particle_steps"] >= 144 * days * (w.n - c["oob"])


def test_cfg3_full_size_sampled():
    from paper_1707_05163_amd import FieldSet, ParticleSet, execute_batch
    ws = SC.cfg3_ensemble()
    log(f"cfg3 full size: {len(ws)} runs, {sum(w.n for w in ws)} particles, 1 day batched")
    fss = [FieldSet.from_workload(w) for w in ws]
    pss = [ParticleSet(f, w.lon0, w.lat0) for f, w in zip(fss, ws)]
    opts = [ParticleSet.opts(Kh=w.Kh, run_id=w.run_id, output_stride=1, stencil_cache=True,
                             sort_every=1) for w in ws]
    execute_batch(pss, DAY, ws[0].dt, DAY, opts, block=128)
    for p, w in zip(pss, ws):
        recs = p.records()
        ids = np.arange(0, w.n, max(1, w.n // 40))
        ofs = O.OracleFieldSet.from_workload(w)
        st = O.make_state(w.lon0[ids], w.lat0[ids], pid=ids.astype(np.uint32))
        orecs = O.run(ofs, st, w.dt, DAY, DAY, Kh=w.Kh, run_id=w.run_id)
        for m, o in enumerate(orecs):
            compare_record(slice_record(recs, m, ids), o, w.grid, float(w.grid.lon[-1]),
                           label=f"{w.name} rec {m}", ofs=ofs)
