"""Reduced-precision storage in 3D (bfloat16, and float16 with a power-of-two scale
per variable, level and snapshot) on the GPU against the FP64 oracle, with the
snapshots streamed through a three-slot ring as in the paper's loop of reading
three time slices and advancing (Sect. 3.1, Sect. 3.4).

The oracle runs in FP64 on exactly the values the storage holds (the reference
quantisers, whose output the device's stored values equal bit for bit); the GPU
interpolates them in FP32 and updates the position in FP64.  The difference is FP32
rounding only, bounded as follows.  One stage's trilinear interpolation in FP32 of
values |v| <= 1 m/s errs by at most about ten roundings of 2^-24 m/s, 6e-7 m/s.
Over T = 3 days that drifts a position by at most 6e-7 T = 0.16 m; neighbouring
trajectories separate at most as exp(L T), with L the largest velocity gradient of
the interpolant (about 2 m/s over a 1 degree cell, 1.8e-5 1/s, so exp(L T) < 110):
17 m, taken as 20 m horizontally.  Vertically |W| <= 1e-4 m/s and its horizontal
gradient is at most 1e-4 m/s over 100 km, so a 20 m horizontal error moves the
depth by at most 2e-8 m/s x T = 5 mm; the bound is 0.05 m.  Cell indices are checked
exactly wherever the oracle's point lies farther than those bounds from a cell face,
and everywhere against the oracle's cell search applied to the GPU's position.
"""

from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from oracle import quantize as Q
from synthetic import configs as SC

from parity import log

pytestmark = pytest.mark.gpu

DAY = 86400.0
M = 111120.0
H_BOUND_M = 20.0
Z_BOUND_M = 0.05


def _near(x, axis, tol):
    idx = np.searchsorted(axis, x)
    lo = np.abs(x - axis[np.clip(idx - 1, 0, axis.size - 1)])
    hi = np.abs(x - axis[np.clip(idx, 0, axis.size - 1)])
    return np.minimum(lo, hi) <= tol


@pytest.mark.parametrize("cache", [True, False])
@pytest.mark.parametrize("dtype", ["bf16", "f16s"])
def test_3d_reduced_storage_through_ring(dtype, cache):
    from paper_1707_05163_amd import FieldSet, ParticleSet
    q = Q.bf16_round if dtype == "bf16" else Q.f16_scaled_round
    w = SC.cfg2_global_3d(nx=120, ny=60, nz=12, nt=4, n_particles=20000, nsteps=432)
    log(f"3D {dtype} cache={cache}: {w.n} particles, 3 days through a 3-slot ring")
    fs = FieldSet.from_workload(w, dtype=dtype, capacity=3, push=False)
    snaps = [w.fields.snapshot(s) for s in range(4)]
    fs.push_snapshot(w.fields.times[0], *snaps[0])
    fs.push_snapshot(w.fields.times[1], *snaps[1])
    fs.push_snapshot(w.fields.times[2], *snaps[2])
    ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0)
    ps.execute(DAY, w.dt, DAY, output_stride=1, stencil_cache=cache)
    # advancetime: snapshot 3 replaces snapshot 0 in the ring, then two more days
    fs.push_snapshot(w.fields.times[3], *snaps[3])
    assert list(fs.resident()) == list(w.fields.times[1:4])
    ps.execute(2 * DAY, w.dt, DAY, output_stride=1, stencil_cache=cache)
    recs = ps.records()
    _, gst = ps.status()
    Uq, Vq, Wq = (np.stack([q(snaps[s][v]) for s in range(4)]) for v in range(3))
    ofs = O.OracleFieldSet(w.grid.lon, w.grid.lat, w.grid.depth, w.fields.times, Uq, Vq, Wq,
                           spherical=True)
    st = O.make_state(w.lon0, w.lat0, w.depth0)
    orecs = O.run(ofs, st, w.dt, 3 * DAY, DAY)
    assert recs["lon"].shape[0] == len(orecs) == 4
    worst_h = worst_z = 0.0
    for m, o in enumerate(orecs):
        g = {k: v[m] for k, v in recs.items()}
        mism = int((g["status"] != o["status"]).sum())
        assert mism <= 2, f"rec {m}: {mism} status mismatches"
        both = (g["status"] == 0) & (o["status"] == 0)
        dx = (g["lon"][both] - o["lon"][both]) * np.cos(np.deg2rad(o["lat"][both])) * M
        dy = (g["lat"][both] - o["lat"][both]) * M
        dh = np.sqrt(dx * dx + dy * dy)
        dz = np.abs(g["depth"][both] - o["depth"][both])
        worst_h, worst_z = max(worst_h, float(dh.max())), max(worst_z, float(dz.max()))
        assert dh.max() <= H_BOUND_M and dz.max() <= Z_BOUND_M, (m, dh.max(), dz.max())
        # cells: the GPU's index is the oracle's cell search at the GPU's position, and
        # the oracle's own index wherever the two positions cannot straddle a face
        ci, cj, ck = ofs.cell_indices(g["lon"][both], g["lat"][both], g["depth"][both])
        assert np.array_equal(ci, g["ci"][both]) and np.array_equal(cj, g["cj"][both])
        assert np.array_equal(ck, g["ck"][both])
        far = ~(_near(o["lon"][both], w.grid.lon, H_BOUND_M / (M * 0.01))
                | _near(o["lat"][both], w.grid.lat, H_BOUND_M / M)
                | _near(o["depth"][both], w.grid.depth, Z_BOUND_M))
        for k in ("ci", "cj", "ck"):
            assert np.array_equal(g[k][both][far], o[k][both][far]), (m, k)
    log(f"  {dtype} cache={cache}: max horizontal {worst_h:.3e} m, depth {worst_z:.3e} m "
        f"(bounds {H_BOUND_M} m, {Z_BOUND_M} m)")
