"""3D parity with a land mask (AdvectionRK4_3D and the land test of Sect. 2.2, with the
recovery of Sect. 3.3): particles that end a step in a land cell are flagged there.
The field is left unchanged over land so that particles do run into land; the mask
is a horizontal property, the same at every depth.  Covers the cached kernel (whose
cell carries the land flag, and whose end-of-step check searches only horizontally)
and the gather kernel, streamed through a three-slot ring, against the FP64 oracle."""

from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from synthetic import configs as SC
from synthetic.fields import ocean_cell_mask, seed_in_cells, smoothed_land_mask

from parity import compare_record, log, slice_record

pytestmark = pytest.mark.gpu

DAYS = 3


def _land_workload(n=20000):
    w = SC.cfg2_global_3d(nx=1440, ny=720, nz=12, nt=DAYS + 1, n_particles=n,
                          nsteps=DAYS * 144)
    rng = np.random.default_rng(2024)
    land = smoothed_land_mask(rng, w.grid.ny, w.grid.nx, land_fraction=0.3, sigma=3.0)
    w.grid.land = land
    x0, y0 = seed_in_cells(rng, ocean_cell_mask(land), n, w.grid.lon, w.grid.lat)
    w.lon0, w.lat0 = x0, y0
    # near the surface, where the eddies are fastest, so that particles reach land
    w.depth0 = rng.uniform(5.0, 100.0, n)
    return w


@pytest.mark.parametrize("cache", [True, False])
def test_3d_land_mask_ring(cache):
    from paper_1707_05163_amd import FieldSet, ParticleSet
    w = _land_workload()
    log(f"3D land: {w.n} particles, {DAYS} days, cache={cache}")
    fs = FieldSet.from_workload(w, capacity=3, push=False)
    fs.push_snapshot(w.fields.times[0], *w.fields.snapshot(0))
    fs.push_snapshot(w.fields.times[1], *w.fields.snapshot(1))
    ps = ParticleSet(fs, w.lon0, w.lat0, w.depth0)
    for d in range(DAYS):
        ps.execute(86400.0, w.dt, w.outputdt, output_stride=1, stencil_cache=cache)
        if d + 2 < w.fields.nt:
            fs.push_snapshot(w.fields.times[d + 2], *w.fields.snapshot(d + 2))
    recs = ps.records()
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0, w.lat0, w.depth0)
    orecs = O.run(ofs, st, w.dt, DAYS * 86400.0, w.outputdt)
    assert recs["lon"].shape[0] == len(orecs) == DAYS + 1
    for m, o in enumerate(orecs):
        compare_record(slice_record(recs, m), o, w.grid, 360.0, label=f"3D land rec {m}",
                       ofs=ofs)
    counts, status = ps.status()
    assert np.array_equal(status, st.status)
    assert counts["particle_steps"] == st.psteps
    # the case is only a test of the land path if particles reach land and others do not
    n_land = int(((status & O.ST_LAND) != 0).sum())
    log(f"3D land: {n_land} of {w.n} particles on land, {int((status == 0).sum())} active")
    assert 0 < n_land < w.n // 2
