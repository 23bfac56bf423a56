"""Flow-map surrogate end to end: training on RK4 segments, inference with the
residual check and the RK4 fallback (plain RK4 stays the arbiter)."""

import numpy as np
import pytest

from synthetic import configs as SC

from parity import log

pytestmark = pytest.mark.gpu


def _field(nt=10, n=20000, nx=360, ny=180):
    return SC.cfg1_global_eddies(nx=nx, ny=ny, nt=nt, n_particles=n, nsteps=576,
                                 period_days=float(nt), cfg_index=4)


def test_fallback_everywhere_equals_plain_rk4():
    """A zero residual threshold sends every particle to the fine RK4 steps: the
    result must be bit-identical to plain execution.  200 particles start at the centres
    of all-land cells (U = V = 0 there), so they stop at their first step and the
    surrogate's cell sorts (at segments 0 and 12) reorder a state with inactive particles
    behind the active ones; both sets then run another day of plain RK4, which checks
    the state and the active list that the surrogate hands back in id order."""
    from paper_1707_05163_amd import FieldSet, ParticleSet, Surrogate
    w = _field()
    lon0, lat0 = w.lon0.copy(), w.lat0.copy()
    L = np.asarray(w.grid.land) != 0
    cells = np.argwhere(L[:-1, :-1] & L[1:, :-1] & L[:-1, 1:] & L[1:, 1:])
    pick = cells[np.linspace(0, len(cells) - 1, 200).astype(int)]
    lon0[:200] = 0.5 * (w.grid.lon[pick[:, 1]] + w.grid.lon[pick[:, 1] + 1])
    lat0[:200] = 0.5 * (w.grid.lat[pick[:, 0]] + w.grid.lat[pick[:, 0] + 1])
    fs = FieldSet.from_workload(w)
    s = Surrogate(3)
    a = ParticleSet(fs, lon0, lat0)
    st = a.execute_surrogate(s, 2 * 86400.0, residual_m=0.0)
    b = ParticleSet(fs, lon0, lat0)
    b.execute(2 * 86400.0, w.dt)
    ga, gb = a.get(), b.get()
    assert np.array_equal(ga["lon"], gb["lon"]) and np.array_equal(ga["lat"], gb["lat"])
    assert np.array_equal(a.status()[1], b.status()[1])
    assert st["accepted"] == 0 and st["segments"] == 24
    assert st["fallback"] == st["evaluated"]
    off = b.status()[1] != 0
    log(f"surrogate fallback: {int(off.sum())} of {w.n} particles inactive after 2 days")
    assert off[:200].all() and off.sum() < w.n // 2
    a.execute(86400.0, w.dt)
    b.execute(86400.0, w.dt)
    ga, gb = a.get(), b.get()
    assert np.array_equal(ga["lon"], gb["lon"]) and np.array_equal(ga["lat"], gb["lat"])
    assert np.array_equal(a.status()[1], b.status()[1])
    assert a.status()[0]["particle_steps"] == b.status()[0]["particle_steps"]


def test_training_then_inference_on_reduced_field():
    from paper_1707_05163_amd import FieldSet, ParticleSet, Surrogate
    w = _field()
    fs = FieldSet.from_workload(w)
    s = Surrogate(5)
    t = s.train(fs, n_segments=300_000, iterations=3000, round_size=50_000, batch=2048,
                lr=1e-3)
    log(f"train: {t}")
    assert t["segments_kept"] == 300_000
    assert t["final_loss"] < 0.2 * t["first_loss"]
    a = ParticleSet(fs, w.lon0, w.lat0)
    st = a.execute_surrogate(s, 2 * 86400.0, residual_m=50.0)
    log(f"infer: {st}")
    b = ParticleSet(fs, w.lon0, w.lat0)
    b.execute(2 * 86400.0, w.dt)
    ga, gb = a.get(), b.get()
    _, sa = a.status()
    _, sb = b.status()
    both = (sa == 0) & (sb == 0)
    M = 111120.0
    dx = (ga["lon"][both] - gb["lon"][both]) * np.cos(np.deg2rad(gb["lat"][both])) * M
    dy = (ga["lat"][both] - gb["lat"][both]) * M
    km = np.sqrt(dx * dx + dy * dy) / 1e3
    log(f"surrogate vs RK4 after 2 days: median {np.median(km):.4f} km, "
        f"p95 {np.percentile(km, 95):.4f} km, max {km.max():.3f} km")
    assert st["accepted"] + st["fallback"] == st["evaluated"]
    assert np.percentile(km, 95) < 5.0
