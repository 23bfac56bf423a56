"""Batched persistent launch over uneven runs, and its autotuner."""

from __future__ import annotations

import json

import numpy as np
import pytest

from oracle import oracle as O
from synthetic import configs as SC

from parity import compare_record, log, slice_record

pytestmark = pytest.mark.gpu


def _runs(n_runs=8, scale=0.002, nsteps=288):
    return SC.cfg3_ensemble(n_runs=n_runs, particle_scale=scale, nsteps=nsteps)


def _make(ws):
    from paper_1707_05163_amd import FieldSet, ParticleSet
    fss = [FieldSet.from_workload(w) for w in ws]
    pss = [ParticleSet(f, w.lon0, w.lat0) for f, w in zip(fss, ws)]
    return fss, pss


@pytest.mark.parametrize("block", [64, 256, 512])
def test_batch_equals_individual_runs(block):
    from paper_1707_05163_amd import ParticleSet, execute_batch
    ws = _runs()
    log(f"batch of {len(ws)} runs, particles {[w.n for w in ws]}, block {block}")
    fa, pa = _make(ws)
    fb, pb = _make(ws)
    opts = [ParticleSet.opts(Kh=w.Kh, run_id=w.run_id, output_stride=1) for w in ws]
    for p, w, o in zip(pa, ws, opts):
        p.execute(w.nsteps * w.dt, w.dt, 6 * 3600.0, Kh=w.Kh, run_id=w.run_id, output_stride=1)
    execute_batch(pb, ws[0].nsteps * ws[0].dt, ws[0].dt, 6 * 3600.0, opts, block=block)
    for a, b in zip(pa, pb):
        ra, rb = a.records(), b.records()
        for k in ("lon", "lat", "status", "ci", "cj"):
            assert np.array_equal(ra[k], rb[k]), k
        assert a.status()[0]["particle_steps"] == b.status()[0]["particle_steps"]


def test_batch_matches_oracle():
    from paper_1707_05163_amd import ParticleSet, execute_batch
    ws = _runs(n_runs=5, scale=0.001)
    fs, ps = _make(ws)
    opts = [ParticleSet.opts(Kh=w.Kh, run_id=w.run_id, output_stride=1) for w in ws]
    execute_batch(ps, ws[0].nsteps * ws[0].dt, ws[0].dt, 12 * 3600.0, opts)
    for p, w in zip(ps, ws):
        recs = p.records()
        ofs = O.OracleFieldSet.from_workload(w)
        st = O.make_state(w.lon0, w.lat0)
        orecs = O.run(ofs, st, w.dt, w.nsteps * w.dt, 12 * 3600.0, Kh=w.Kh, run_id=w.run_id)
        for m, o in enumerate(orecs):
            compare_record(slice_record(recs, m), o, w.grid, float(w.grid.lon[-1]),
                           label=f"{w.name} rec {m}", ofs=ofs)


def test_autotune_restores_state_and_caches(tmp_path):
    from paper_1707_05163_amd import ParticleSet, autotune_batch, execute_batch
    ws = _runs(n_runs=6, scale=0.002)
    fs, ps = _make(ws)
    opts = [ParticleSet.opts(Kh=w.Kh, run_id=w.run_id) for w in ws]
    cache = tmp_path / "tune.json"
    best = autotune_batch(ps, ws[0].dt, 12, opts, cache)
    assert best["block"] in (128, 256, 512) and best["stencil_cache"] in (0, 1)
    assert (best["sort_every"], best["sort_steps"]) in ((0, 0), (1, 0), (0, 64), (0, 16), (0, 4))
    assert best["ms"] > 0
    table = json.loads(cache.read_text())
    entry = list(table.values())[0]
    assert len(table) == 1 and entry["block"] == best["block"]
    assert entry["sort_steps"] == best["sort_steps"]
    again = autotune_batch(ps, ws[0].dt, 12, opts, cache)
    keys = ("block", "stencil_cache", "sort_every", "sort_steps")
    assert {k: again[k] for k in keys} == {k: best[k] for k in keys}
    assert again["ms"] == pytest.approx(best["ms"], abs=1e-4)
    for p, w in zip(ps, ws):  # trials left no trace
        g = p.get()
        c, st = p.status()
        assert np.array_equal(g["lon"], w.lon0) and np.array_equal(g["lat"], w.lat0)
        assert c["particle_steps"] == 0 and c["step"] == 0 and (st == 0).all()
    for o in opts:
        o.stencil_cache, o.sort_every = best["stencil_cache"], best["sort_every"]
        o.sort_steps = best["sort_steps"]
    execute_batch(ps, 144 * ws[0].dt, ws[0].dt, 0.0, opts, block=best["block"])
    _, fb = _make(ws)
    for p, w in zip(fb, ws):
        p.execute(144 * w.dt, w.dt, Kh=w.Kh, run_id=w.run_id)
    for a, b in zip(ps, fb):
        assert np.array_equal(a.get()["lon"], b.get()["lon"])


def test_batch_rejects_mixed_kinds():
    from paper_1707_05163_amd import FieldSet, ParticleSet, execute_batch
    from paper_1707_05163_amd._lib import LPError, LP_EINVAL
    ws = _runs(n_runs=2, scale=0.001)
    fs, ps = _make(ws)
    f3 = FieldSet.from_workload(ws[0], dtype="bf16")
    p3 = ParticleSet(f3, ws[0].lon0, ws[0].lat0)
    with pytest.raises(LPError) as e:
        execute_batch([ps[0], p3], 10 * ws[0].dt, ws[0].dt)
    assert e.value.code == LP_EINVAL
    with pytest.raises(LPError) as e:
        execute_batch([ps[0], ps[0]], 10 * ws[0].dt, ws[0].dt)
    assert e.value.code == LP_EINVAL


@pytest.mark.parametrize("cache", [True, False])
def test_graph_replay_equals_direct_launches(cache):
    """Each output segment captured into a HIP graph (made at the first segment,
    updated in place for the others) and launched as one: records equal the direct
    launches bit for bit, at every output time, on two executes in a row with the
    program's own eager work and synchronisation between the graph launches."""
    import torch
    from paper_1707_05163_amd import ParticleSet, execute_batch
    ws = _runs(n_runs=7, scale=0.002)
    log(f"graph replay: {len(ws)} runs, cache={cache}")
    fa, pa = _make(ws)
    fb, pb = _make(ws)
    runtime, out = 2 * 86400.0, 6 * 3600.0
    for graph, ps in ((False, pa), (True, pb)):
        opts = [ParticleSet.opts(Kh=w.Kh, run_id=w.run_id, output_stride=1, sort_every=2,
                                 stencil_cache=cache, graph=graph) for w in ws]
        execute_batch(ps, runtime, ws[0].dt, out, opts, block=128)
        x = torch.ones(1 << 20, device="cuda")  # eager work between the two executes
        assert float((x * 2).sum()) == 2.0 * (1 << 20)
        torch.cuda.synchronize()
        execute_batch(ps, runtime, ws[0].dt, out, opts, block=128)
    for a, b in zip(pa, pb):
        ra, rb = a.records(), b.records()
        assert ra["lon"].shape[0] == 1 + 2 * 8
        for k in ("lon", "lat", "status", "ci", "cj"):
            assert np.array_equal(ra[k], rb[k]), k
        assert a.status()[0]["particle_steps"] == b.status()[0]["particle_steps"]


@pytest.mark.parametrize("sort_steps", [64, 16, 4])
def test_sort_every_k_steps_changes_nothing(sort_steps):
    """Launches cut every K steps with a sort before each: same records, bit for bit,
    as one launch per output segment, in the batched launch and in single runs."""
    from paper_1707_05163_amd import ParticleSet, execute_batch
    ws = _runs(n_runs=4, scale=0.002)
    _, pa = _make(ws)
    _, pb = _make(ws)
    oa = [ParticleSet.opts(Kh=w.Kh, run_id=w.run_id, output_stride=1, sort_every=0) for w in ws]
    ob = [ParticleSet.opts(Kh=w.Kh, run_id=w.run_id, output_stride=1, sort_steps=sort_steps)
          for w in ws]
    execute_batch(pa, 86400.0, ws[0].dt, 6 * 3600.0, oa)
    execute_batch(pb, 86400.0, ws[0].dt, 6 * 3600.0, ob)
    w = ws[0]
    _, pc = _make([w])
    pc[0].execute(86400.0, w.dt, 6 * 3600.0, Kh=w.Kh, run_id=w.run_id, output_stride=1,
                  sort_steps=sort_steps)
    for a, b in zip(pa, pb):
        ra, rb = a.records(), b.records()
        assert ra["lon"].shape[0] == 5
        for k in ("lon", "lat", "status", "ci", "cj"):
            assert np.array_equal(ra[k], rb[k]), k
    rc = pc[0].records()
    ra = pa[0].records()
    for k in ("lon", "lat", "status", "ci", "cj"):
        assert np.array_equal(ra[k], rc[k]), k
