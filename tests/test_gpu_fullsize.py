"""Parity at the benchmark sizes, in the benchmark's launch configuration (register /
LDS stencil cache, daily output segments, the benchmark's sort cadence), on sampled
particles the oracle follows one by one: the 0.25 degree global 2D field with 1M
particles, the 0.1 degree global 3D field with 10M particles, and the 64-run Brownian
ensemble in one batched launch per segment.  Each run is shortened in time (one or two days); the
kernels, grids and particle counts are those of the benchmark."""

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
    log(f"cfg1 full size: {w.n} particles on {w.grid.nx}x{w.grid.ny}, 2 days")
    fs = FieldSet.from_workload(w)
    ps = ParticleSet(fs, w.lon0, w.lat0)
    ps.execute(2 * DAY, w.dt, DAY, output_stride=1, sort_every=10, stencil_cache=True)
    recs = ps.records()
    ids = np.arange(0, w.n, 997)
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0[ids], w.lat0[ids], pid=ids.astype(np.uint32))
    orecs = O.run(ofs, st, w.dt, 2 * DAY, DAY, nthreads=O.max_threads())
    assert recs["lon"].shape[0] == len(orecs) == 3
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m, ids), o, w.grid, 360.0, label=f"cfg1 rec {m}",
                       ofs=ofs)
    _, status = ps.status()
    assert np.array_equal(status[ids], st.status)


def test_cfg2_full_size_sampled():
    import torch
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.cfg2_global_3d()
    log(f"cfg2 full size: {w.n} particles on {w.grid.nx}x{w.grid.ny}x{w.grid.nz}, 1 day")
    cache = {}
    snaps = [SC.cfg2_snapshot_torch(w, s, "cuda", cache) for s in range(2)]
    del cache
    stride = 10007
    fs = FieldSet(w.grid.lon, w.grid.lat, w.grid.depth, "spherical", "f32", 3, 0.0)
    ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0)
    fs.push_snapshot(w.fields.times[0], *snaps[0])
    fs.push_snapshot(w.fields.times[1], *snaps[1])
    ps.execute(DAY, w.dt, DAY, output_stride=stride, sort_every=0, stencil_cache=True)
    recs = ps.records()
    torch.cuda.synchronize()
    U, V, W = (np.stack([snaps[q][v].cpu().numpy() for q in range(2)]) for v in range(3))
    del snaps
    ofs = O.OracleFieldSet(w.grid.lon, w.grid.lat, w.grid.depth, w.fields.times[:2], U, V, W,
                           spherical=True)
    ids = np.arange(0, w.n, stride)
    assert recs["lon"].shape == (2, ids.size)
    st = O.make_state(w.lon0[ids], w.lat0[ids], w.depth0[ids], pid=ids.astype(np.uint32))
    orecs = O.run(ofs, st, w.dt, DAY, DAY, nthreads=O.max_threads())
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, w.grid, 360.0, label=f"cfg2 rec {m}", ofs=ofs)
    c, status = ps.status()
    assert np.array_equal(status[ids], st.status)
    assert c["particle_steps"] >= 144 * (w.n - c["oob"])


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
