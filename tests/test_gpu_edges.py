"""Edge cases of the GPU path against the oracle: single particles and counts that
leave partial waves and blocks, zero runtime, a set with nothing left active, the
smallest grids (one cell in 2D and 3D), an output stride larger than the set, and
the particle-count limit."""

import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from synthetic import configs as SC

from parity import compare_record, log, slice_record

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 63, 65, 257, 1000])
def test_ragged_particle_counts(n):
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.cfg1_global_eddies(nx=144, ny=72, nt=30, n_particles=1000, nsteps=288)
    log(f"ragged n={n}")
    fs = FieldSet.from_workload(w)
    ps = ParticleSet(fs, w.lon0[:n], w.lat0[:n])
    ps.execute(86400.0, w.dt, 21600.0, output_stride=1)
    recs = ps.records()
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0[:n], w.lat0[:n])
    orecs = O.run(ofs, st, w.dt, 86400.0, 21600.0)
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, w.grid, 360.0, label=f"n={n} rec {m}", ofs=ofs)
    assert ps.status()[0]["particle_steps"] == st.psteps


def test_zero_runtime_and_nothing_active():
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = SC.cfg1_global_eddies(nx=72, ny=36, nt=30, n_particles=50, nsteps=288)
    fs = FieldSet.from_workload(w)
    ps = ParticleSet(fs, w.lon0, w.lat0)
    ps.execute(0.0, w.dt)
    c, st = ps.status()
    assert c["particle_steps"] == 0 and (st == 0).all() and c["step"] == 0
    g = ps.get()
    assert np.array_equal(g["lon"], w.lon0) and np.array_equal(g["lat"], w.lat0)
    # every particle starts outside the grid: the first step deletes all of them,
    # and later calls run on an empty active list
    out = ParticleSet(fs, np.full(70, 500.0), np.zeros(70))
    out.execute(3600.0, w.dt, 1800.0, output_stride=7)
    c, st = out.status()
    assert (st == O.ST_OOB | O.ST_DELETED).all() and c["active"] == 0
    assert c["particle_steps"] == 70
    out.execute(3600.0, w.dt, 1800.0, output_stride=7)
    c2, st2 = out.status()
    assert c2["particle_steps"] == 70 and np.array_equal(st, st2) and c2["step"] == 24
    recs = out.records()
    assert recs["lon"].shape == (5, 10)
    assert (recs["ci"][1:] == -1).all()


@pytest.mark.parametrize("cache", [True, False])
def test_one_cell_grids(cache):
    """2 x 2 (x 2) nodes: a single cell, every particle in it; uniform and sheared
    flows that carry some particles out through each face."""
    from paper_1707_05163_amd import FieldSet, ParticleSet
    rng = np.random.default_rng(8)
    X = np.array([0.0, 1000.0])
    Y = np.array([-500.0, 700.0])
    Z = np.array([5.0, 105.0])
    n = 300
    x0, y0, z0 = rng.uniform(0, 1000, n), rng.uniform(-500, 700, n), rng.uniform(5, 105, n)
    U = np.array([[[0.2, 0.5], [-0.3, 0.1]]])        # [t][y][x]
    V = np.array([[[0.1, -0.4], [0.3, 0.25]]])
    fs2 = FieldSet(X, Y, None, "flat", "f64", 1)
    fs2.push_snapshot(0.0, U, V)
    ps = ParticleSet(fs2, x0, y0)
    ps.execute(600.0, 60.0, 120.0, output_stride=1, stencil_cache=cache)
    recs = ps.records()
    ofs = O.OracleFieldSet(X, Y, None, [0.0], U, V)
    st = O.make_state(x0, y0)
    orecs = O.run(ofs, st, 60.0, 600.0, 120.0)
    grid2 = SC.Grid(lon=X, lat=Y)
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, grid2, 1000.0, label=f"2x2 rec {m}")
    assert 0 < (st.status != 0).sum() < n
    # 3D: 2 x 2 x 2 nodes with W
    U3 = np.stack([U[0], 0.5 * U[0]])[None]            # [t][z][y][x]
    V3 = np.stack([V[0], -V[0]])[None]
    W3 = np.full((1, 2, 2, 2), 0.05)
    fs3 = FieldSet(X, Y, Z, "flat", "f64", 1)
    fs3.push_snapshot(0.0, U3, V3, W3)
    p3 = ParticleSet(fs3, x0, y0, z0)
    p3.execute(600.0, 60.0, 120.0, output_stride=1, stencil_cache=cache)
    recs3 = p3.records()
    ofs3 = O.OracleFieldSet(X, Y, Z, [0.0], U3, V3, W3)
    st3 = O.make_state(x0, y0, z0)
    orecs3 = O.run(ofs3, st3, 60.0, 600.0, 120.0)
    grid3 = SC.Grid(lon=X, lat=Y, depth=Z)
    for m, o in enumerate(orecs3):
        compare_record(slice_record(recs3, m), o, grid3, 1000.0, label=f"2x2x2 rec {m}")


def test_particle_count_limit_is_checked_before_any_allocation():
    from paper_1707_05163_amd import FieldSet
    from paper_1707_05163_amd import _lib as L
    fs = FieldSet(np.array([0.0, 1.0]), np.array([0.0, 1.0]), None, "flat", "f32", 1)
    x = np.zeros(4)
    h = C.c_void_p()
    for n in (0, -5, 2 ** 31):
        rc = L.lib.pset_create(fs.handle, n, x.ctypes.data, x.ctypes.data, None, 0.0, 0,
                               C.byref(h))
        assert rc == L.LP_EINVAL and not h.value
