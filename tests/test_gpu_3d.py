"""3D parity (AdvectionRK4_3D): stretched depth levels, U, V, W snapshots streamed
through a three-slot ring, trilinear interpolation in FP64 from float32 storage."""

from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from synthetic import configs as SC

from parity import compare_record, log, slice_record

pytestmark = pytest.mark.gpu


def _run_ring(w, days, cache=True, dtype="f32", stride=1, sort_every=1):
    """The paper's loop: two snapshots resident, execute one day, advancetime."""
    from paper_1707_05163_amd import FieldSet, ParticleSet
    fs = FieldSet.from_workload(w, dtype=dtype, capacity=3, push=False)
    fs.push_snapshot(w.fields.times[0], *w.fields.snapshot(0))
    fs.push_snapshot(w.fields.times[1], *w.fields.snapshot(1))
    ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0)
    for d in range(days):
        ps.execute(86400.0, w.dt, w.outputdt, output_stride=stride, sort_every=sort_every,
                   stencil_cache=cache)
        if d + 2 < w.fields.nt:
            fs.push_snapshot(w.fields.times[d + 2], *w.fields.snapshot(d + 2))
    return ps, fs


@pytest.mark.parametrize("cache", [True, False])
def test_cfg2_reduced_grid_ring(cache):
    w = SC.cfg2_global_3d(nx=360, ny=180, nz=50, nt=4, n_particles=20000, nsteps=432)
    log(f"cfg2 reduced: {w.n} particles, 3 days, cache={cache}")
    ps, fs = _run_ring(w, 3, cache=cache)
    recs = ps.records()
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0, w.depth0)
    orecs = O.run(ofs, st, w.dt, 3 * 86400.0, w.outputdt)
    assert recs["lon"].shape[0] == len(orecs) == 4
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, w.grid, 360.0, label=f"cfg2r rec {m}", ofs=ofs)
    counts, status = ps.status()
    assert counts["particle_steps"] == st.psteps
    assert np.array_equal(status, st.status)


def test_3d_trilinear_field_flat_nonuniform():
    """A steady field that is trilinear in (x, y, z) on a non-uniform flat grid."""
    rng = np.random.default_rng(31)
    X = np.cumsum(rng.uniform(500, 1500, 40))
    Y = np.cumsum(rng.uniform(500, 1500, 30))
    Z = np.cumsum(rng.uniform(2, 20, 25))
    ZZ, YY, XX = np.meshgrid(Z, Y, X, indexing="ij")
    xc, yc, zc = X.mean(), Y.mean(), Z.mean()
    U = (-1e-4 * (YY - yc) + 1e-9 * (XX - xc) * (ZZ - zc)).astype(np.float32)
    V = (1e-4 * (XX - xc) + 2e-10 * (XX - xc) * (YY - yc) / 100).astype(np.float32)
    W = (1e-6 * (ZZ - zc) + 1e-9 * (XX - xc)).astype(np.float32)
    n = 3000
    x0 = rng.uniform(X[5], X[-6], n)
    y0 = rng.uniform(Y[5], Y[-6], n)
    z0 = rng.uniform(Z[3], Z[-4], n)
    from paper_1707_05163_amd import FieldSet, ParticleSet
    for cache in (True, False):
        fs = FieldSet(X, Y, Z, mesh="flat", dtype="f32", capacity=1)
        fs.push_snapshot(0.0, U, V, W)
        ps = ParticleSet(fs, x0, y0, z0)
        ps.execute(3600.0 * 6, 60.0, 3600.0, output_stride=1, stencil_cache=cache)
        recs = ps.records()
        ofs = O.OracleFieldSet(X, Y, Z, [0.0], U[None], V[None], W[None])
        st = O.make_state(x0, y0, z0)
        orecs = O.run(ofs, st, 60.0, 3600.0 * 6, 3600.0)
        grid = SC.Grid(lon=X, lat=Y, depth=Z)
        for m, o in enumerate(orecs):
            compare_record(slice_record(recs, m), o, grid, float(X[-1] - X[0]),
                           label=f"trilinear rec {m}", ofs=ofs)


def test_cfg2_device_generator_bit_identical():
    import torch
    w = SC.cfg2_global_3d(nx=360, ny=180, nz=20, nt=3, n_particles=10)
    cache = {}
    for s in range(3):
        U, V, W = w.fields.snapshot(s)
        Ut, Vt, Wt = SC.cfg2_snapshot_torch(w, s, "cuda", cache)
        torch.cuda.synchronize()
        assert np.array_equal(U, Ut.cpu().numpy())
        assert np.array_equal(V, Vt.cpu().numpy())
        assert np.array_equal(W, Wt.cpu().numpy())


def test_push_from_device_equals_push_from_host():
    import torch
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.cfg2_global_3d(nx=180, ny=90, nz=12, nt=3, n_particles=4000, nsteps=144)
    fa = FieldSet.from_workload(w, capacity=3)
    fb = FieldSet.from_workload(w, capacity=3, push=False)
    cache = {}
    for s in range(3):
        fb.push_snapshot(w.fields.times[s], *SC.cfg2_snapshot_torch(w, s, "cuda", cache))
    a = ParticleSet(fa, w.lon0, w.lat0, w.depth0)
    b = ParticleSet(fb, w.lon0, w.lat0, w.depth0)
    a.execute(2 * 86400.0, w.dt)
    b.execute(2 * 86400.0, w.dt)
    ga, gb = a.get(), b.get()
    for k in ("lon", "lat", "depth"):
        assert np.array_equal(ga[k], gb[k])


def test_host_push_through_pinned_staging_equals_device_push():
    """Snapshots pushed from host memory (through the library's two pinned staging
    chunks, several chunks per variable here) hold the same values and give the same
    trajectories, bit for bit, as the same snapshots pushed from device memory, through
    a ring of three slots; the host arrays may be overwritten as soon as a push
    returns."""
    import torch
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.cfg2_global_3d(nx=1800, ny=900, nz=50, nt=4, n_particles=20000, nsteps=144)
    log(f"host vs device push: {w.grid.nx}x{w.grid.ny}x{w.grid.nz}, 324 MB per variable")
    cache = {}
    dev = [SC.cfg2_snapshot_torch(w, s, "cuda", cache) for s in range(4)]
    torch.cuda.synchronize()
    fa = FieldSet(w.grid.lon, w.grid.lat, w.grid.depth, "spherical", "f32", 3, 0.0)
    fb = FieldSet(w.grid.lon, w.grid.lat, w.grid.depth, "spherical", "f32", 3, 0.0)

    def push(s):
        host = [x.cpu().numpy() for x in dev[s]]
        fa.push_snapshot(w.fields.times[s], *host)
        for h in host:  # the library holds its own copy once the call has returned
            h.fill(np.nan)
        fb.push_snapshot(w.fields.times[s], *dev[s])

    for s in range(3):
        push(s)
    a = ParticleSet(fa, w.lon0, w.lat0, w.depth0)
    b = ParticleSet(fb, w.lon0, w.lat0, w.depth0)
    a.execute(86400.0, w.dt, 86400.0, output_stride=1)
    b.execute(86400.0, w.dt, 86400.0, output_stride=1)
    push(3)
    a.execute(2 * 86400.0, w.dt, 86400.0, output_stride=1)
    b.execute(2 * 86400.0, w.dt, 86400.0, output_stride=1)
    ra, rb = a.records(), b.records()
    for k in ("lon", "lat", "depth", "status", "ci", "cj", "ck"):
        assert np.array_equal(ra[k], rb[k]), k
    assert (ra["status"][-1] == 0).sum() > 0.9 * w.n
    for s in (1, 2, 3):
        ua, va, wa = fa.get_snapshot(w.fields.times[s])
        ub, vb, wb = fb.get_snapshot(w.fields.times[s])
        assert np.array_equal(ua, ub) and np.array_equal(va, vb) and np.array_equal(wa, wb)
    assert np.array_equal(ua, dev[3][0].cpu().numpy())
