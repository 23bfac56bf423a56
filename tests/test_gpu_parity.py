"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Positions agree to 1e-9 relative (of max(|x|, extent)), statuses and cell indices
exactly, on the same seeded inputs; plus the invariances the method guarantees
(chunking, resume, permutation, sort, snapshot ring)."""

from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from synthetic import configs as SC
from synthetic import idealised as SI

from parity import compare_record, log, run_gpu, run_oracle, slice_record

pytestmark = pytest.mark.gpu


def _lp():
    from paper_1707_05163_amd import FieldSet, ParticleSet
    return FieldSet, ParticleSet


def _compare_all(w, recs, orecs, extent, ofs=None, sel=None, label=""):
    assert recs["lon"].shape[0] == len(orecs)
    ex = 0
    for m, o in enumerate(orecs):
        ex += compare_record(slice_record(recs, m, sel), o, w.grid, extent,
                             label=f"{label} record {m}", ofs=ofs)
    return ex


def test_cfg0_solid_body_full():
    w = SC.cfg0_solid_body()
    log(f"cfg0: {w.n} particles x {w.nsteps} steps, f64 fields")
    ps, fs, recs, counts, status = run_gpu(w, dtype="f64", stride=1)
    orecs, ost = run_oracle(w)
    _compare_all(w, recs, orecs, 1e5, label="cfg0")
    assert counts["particle_steps"] == ost.psteps == w.n * w.nsteps
    assert counts["active"] == w.n
    # closed form: radius conserved and angle = w t
    z0 = (w.lon0 - 5e4) + 1j * (w.lat0 - 5e4)
    z = (recs["lon"][-1] - 5e4) + 1j * (recs["lat"][-1] - 5e4)
    exact = z0 * np.exp(1j * w.meta["omega"] * w.dt * w.nsteps)
    assert np.abs(z - exact).max() < 1e-7


def test_cfg0_f32_fields_match_oracle_on_same_values():
    w = SC.cfg0_solid_body(n_particles=3000, nsteps=300)
    w.fields.U = w.fields.U.astype(np.float32)
    w.fields.V = w.fields.V.astype(np.float32)
    ps, fs, recs, counts, status = run_gpu(w, dtype="f32", stride=1)
    orecs, _ = run_oracle(w)
    _compare_all(w, recs, orecs, 1e5, label="cfg0-f32")


@pytest.mark.parametrize("sort_every", [0, 1])
def test_cfg1_small_grid(sort_every):
    w = SC.cfg1_global_eddies(nx=144, ny=72, nt=30, n_particles=4000, nsteps=576)
    log(f"cfg1 small: {w.n} particles, {w.nsteps} steps, sort_every={sort_every}")
    ps, fs, recs, counts, status = run_gpu(w, stride=1, sort_every=sort_every)
    ofs = O.OracleFieldSet.from_workload(w)
    orecs, ost = run_oracle(w, fs=ofs)
    _compare_all(w, recs, orecs, 360.0, ofs=ofs, label="cfg1-small")
    assert counts["particle_steps"] == ost.psteps
    assert (status == ost.status).all()


def test_cfg1_full_grid_one_day():
    w = SC.cfg1_global_eddies(n_particles=20000, nsteps=288)
    log(f"cfg1 full grid: {w.n} particles, {w.nsteps} steps")
    ps, fs, recs, counts, status = run_gpu(w, stride=1, outputdt=6 * 3600.0)
    ofs = O.OracleFieldSet.from_workload(w)
    orecs, ost = run_oracle(w, fs=ofs, outputdt=6 * 3600.0)
    _compare_all(w, recs, orecs, 360.0, ofs=ofs, label="cfg1")
    assert counts["particle_steps"] == ost.psteps


def test_paper_oscillating_flow_gpu():
    w = SI.oscillating_zonal_flow()
    log(f"oscillating flow: {w.fields.nt} snapshots")
    ps, fs, recs, counts, status = run_gpu(w, dtype="f64", stride=1)
    A, om = w.meta["A"], w.meta["omega"]
    th = om * w.dt
    gain = (th / 2) / np.tan(th / 2)
    for m in range(recs["lon"].shape[0]):
        t = m * w.outputdt
        assert np.abs(recs["lon"][m] - (w.lon0 + (A / om) * np.sin(om * t) * gain)).max() < 1e-9
        assert np.abs(recs["lat"][m] - A * t).max() < 1e-9
    orecs, _ = run_oracle(w)
    _compare_all(w, recs, orecs, 2e5, label="oscillating")


def test_paper_zonal_sphere_gpu():
    w = SI.zonal_flow_sphere()
    ps, fs, recs, counts, status = run_gpu(w, dtype="f64", stride=1)
    assert np.array_equal(recs["lat"][-1], w.lat0)
    M = 1852.0 * 60.0
    per_step = w.dt / (M * np.cos(np.deg2rad(w.lat0)))
    assert np.abs(recs["lon"][-1] - (w.lon0 + w.nsteps * per_step)).max() < 1e-9
    orecs, _ = run_oracle(w)
    _compare_all(w, recs, orecs, 360.0, label="zonal")


def test_special_cases_gpu():
    FieldSet, ParticleSet = _lp()
    n = 11
    X = 100.0 * np.arange(n)
    land = np.zeros((n, n), np.uint8)
    land[4:7, 4:7] = 1
    U = np.full((n, n), 0.01)
    U[land != 0] = 0.0
    V = np.zeros((n, n))
    x0 = np.array([-1.0, 550.0, 1000.0, np.nan, 200.0, 990.0])
    y0 = np.array([500.0, 550.0, 1000.0, 500.0, 200.0, 200.0])
    for policy in ("delete", "freeze"):
        fs = FieldSet(X, X, dtype="f64", capacity=1, land=land)
        fs.push_snapshot(0.0, U, V)
        ps = ParticleSet(fs, x0, y0)
        ps.execute(240.0, 60.0, 60.0, recovery=policy, output_stride=1)
        ofs = O.OracleFieldSet(X, X, None, [0.0], U[None], V[None], land=land)
        st = O.make_state(x0, y0)
        recs = O.run(ofs, st, 60.0, 240.0, 60.0, policy=0 if policy == "delete" else 1)
        g = ps.records()
        for m, o in enumerate(recs):
            assert np.array_equal(g["status"][m], o["status"]), (policy, m)
            assert np.array_equal(g["lon"][m], o["lon"], equal_nan=True)
            assert np.array_equal(g["ci"][m], o["ci"]) and np.array_equal(g["cj"][m], o["cj"])
        counts, status = ps.status()
        assert counts["particle_steps"] == st.psteps


def test_chunking_and_resume_bit_identical_gpu():
    FieldSet, ParticleSet = _lp()
    w = SC.cfg1_global_eddies(nx=144, ny=72, nt=6, n_particles=3000, nsteps=576,
                              period_days=6.0)
    fs = FieldSet.from_workload(w)
    a = ParticleSet(fs, w.lon0, w.lat0)
    a.execute(576 * w.dt, w.dt, Kh=10.0, run_id=3)
    b = ParticleSet(fs, w.lon0, w.lat0)
    for _ in range(4):
        b.execute(144 * w.dt, w.dt, Kh=10.0, run_id=3)
    c = ParticleSet(fs, w.lon0, w.lat0)
    c.execute(100 * w.dt, w.dt, Kh=10.0, run_id=3)
    g = c.get()
    _, st = c.status()
    keep = st == 0
    # resume from the copied state: continue only the still-active particles
    c2 = ParticleSet(fs, g["lon"], g["lat"], t0=0.0, step0=100)
    c2.execute(476 * w.dt, w.dt, Kh=10.0, run_id=3)
    ga, gb, gc = a.get(), b.get(), c2.get()
    _, sa = a.status()
    assert np.array_equal(ga["lon"], gb["lon"]) and np.array_equal(ga["lat"], gb["lat"])
    assert np.array_equal(sa, b.status()[1])
    # ids keep their Philox streams only if they keep their ids: compare the survivors
    # of c (whose ids are unchanged because c2 holds every particle in the same order)
    assert np.array_equal(ga["lon"][keep], gc["lon"][keep])
    assert np.array_equal(ga["lat"][keep], gc["lat"][keep])
    assert a.status()[0]["particle_steps"] == b.status()[0]["particle_steps"]


def test_permutation_invariance_gpu():
    FieldSet, ParticleSet = _lp()
    w = SC.cfg1_global_eddies(nx=144, ny=72, nt=6, n_particles=5000, nsteps=288,
                              period_days=6.0)
    perm = np.random.default_rng(5).permutation(w.n)
    fs = FieldSet.from_workload(w)
    a = ParticleSet(fs, w.lon0, w.lat0)
    a.execute(288 * w.dt, w.dt, 3600.0, sort_every=1)
    b = ParticleSet(fs, w.lon0, w.lat0)
    b.execute(288 * w.dt, w.dt, 3600.0, sort_every=0)
    c = ParticleSet(fs, w.lon0[perm], w.lat0[perm])
    c.execute(288 * w.dt, w.dt, 3600.0, sort_every=3)
    ga, gb, gc = a.get(), b.get(), c.get()
    assert np.array_equal(ga["lon"], gb["lon"]) and np.array_equal(ga["lat"], gb["lat"])
    assert np.array_equal(ga["lon"][perm], gc["lon"]) and np.array_equal(ga["lat"][perm], gc["lat"])


def test_snapshot_ring_streaming_matches_all_resident():
    FieldSet, ParticleSet = _lp()
    w = SC.cfg1_global_eddies(nx=144, ny=72, nt=8, n_particles=3000, nsteps=288 * 6,
                              period_days=8.0)
    # all 8 snapshots resident (periodic)
    fsa = FieldSet.from_workload(w)
    a = ParticleSet(fsa, w.lon0, w.lat0)
    a.execute(6 * 86400.0, w.dt, 86400.0)
    # three-slot ring, the paper's loop: execute one day, then advancetime
    fsr = FieldSet.from_workload(w, capacity=3, push=False, time_period=0.0)
    for s in range(2):
        fsr.push_snapshot(w.fields.times[s], *w.fields.snapshot(s))
    r = ParticleSet(fsr, w.lon0, w.lat0)
    for d in range(6):
        r.execute(86400.0, w.dt, 86400.0)
        fsr.push_snapshot(w.fields.times[d + 2], *w.fields.snapshot(d + 2))
    assert list(fsr.resident()) == list(w.fields.times[5:8])
    ga, gr = a.get(), r.get()
    assert np.array_equal(ga["lon"], gr["lon"]) and np.array_equal(ga["lat"], gr["lat"])
    assert np.array_equal(a.status()[1], r.status()[1])


def test_call_level_errors_gpu():
    from paper_1707_05163_amd._lib import LPError, LP_ETIME, LP_EINVAL, LP_ESTATE
    FieldSet, ParticleSet = _lp()
    X = np.arange(5.0)
    U = np.zeros((5, 5), np.float32)
    fs = FieldSet(X, X, capacity=3)
    fs.push_snapshot(0.0, U, U)
    fs.push_snapshot(100.0, U, U)
    ps = ParticleSet(fs, [1.0], [1.0])
    with pytest.raises(LPError) as e:
        ps.execute(200.0, 10.0)          # past the last snapshot
    assert e.value.code == LP_ETIME
    with pytest.raises(LPError) as e:
        ps.execute(100.0, 30.0)          # dt does not divide runtime
    assert e.value.code == LP_EINVAL
    with pytest.raises(LPError) as e:
        ps.execute(100.0, 10.0, 25.0)    # dt does not divide outputdt
    assert e.value.code == LP_EINVAL
    with pytest.raises(LPError) as e:
        fs.push_snapshot(50.0, U, U)     # time going backwards
    assert e.value.code == LP_EINVAL
    ps.execute(100.0, 10.0)
    assert ps.status()[0]["step"] == 10
    fp = FieldSet(X, X, capacity=2, time_period=300.0)
    fp.push_snapshot(0.0, U, U)
    fp.push_snapshot(100.0, U, U)
    with pytest.raises(LPError) as e:
        fp.push_snapshot(200.0, U, U)    # periodic sets keep every snapshot
    assert e.value.code == LP_ESTATE
