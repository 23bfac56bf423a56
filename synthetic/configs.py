"""Seeded synthetic workloads with the shapes of the five benchmark configurations.

Every array is generated from ``numpy.random.Generator(PCG64(SeedSequence(1707051630
+ k)))`` for configuration k, with spawned child streams for the streamfunctions,
the land mask, the particle starts and the ensemble runs.  The generators stand in
for the OGCM data the paper reads (OFES, Sect. 3.1): they reproduce the grid
shapes, resolutions, velocity scales and land fraction, not the data.

Array conventions (read by both the oracle and the HIP library):
  * coordinates are float64, strictly increasing;
  * velocity snapshots are ``[nt, ny, nx]`` (2D) or ``[nt, nz, ny, nx]`` (3D),
    i fastest, in m/s (W positive downward);
  * the land mask is a ``[ny, nx]`` uint8 node mask (1 = land, U = V = 0 there).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from .fields import (
    METRES_PER_DEGREE,
    ocean_cell_mask,
    random_streamfunction,
    seed_in_cells,
    smoothed_land_mask,
    velocity_from_streamfunction,
)

DAY = 86400.0
BASE_SEED = 1707051630

# status policies understood by both sides
POLICY_DELETE = 0
POLICY_FREEZE = 1


def _streams(cfg_index: int, n: int = 6):
    ss = np.random.SeedSequence(BASE_SEED + cfg_index)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


@dataclass
class Grid:
    lon: np.ndarray
    lat: np.ndarray
    depth: Optional[np.ndarray] = None
    spherical: bool = False
    land: Optional[np.ndarray] = None

    @property
    def nx(self) -> int:
        return int(self.lon.size)

    @property
    def ny(self) -> int:
        return int(self.lat.size)

    @property
    def nz(self) -> int:
        return 1 if self.depth is None else int(self.depth.size)

    @property
    def is3d(self) -> bool:
        return self.depth is not None


@dataclass
class Fields:
    """Velocity snapshots.  Either held as arrays (U, V, W with a leading time
    axis) or produced on demand by ``maker(s) -> (U_s, V_s, W_s)``."""
    times: np.ndarray
    period: float = 0.0
    U: Optional[np.ndarray] = None
    V: Optional[np.ndarray] = None
    W: Optional[np.ndarray] = None
    maker: Optional[Callable[[int], tuple]] = None
    # optional scalar tracer (e.g. temperature) on the same grid and snapshots:
    # arrays with the leading time axis, or ``tracer_maker(s) -> T_s``
    tracer: Optional[np.ndarray] = None
    tracer_maker: Optional[Callable[[int], np.ndarray]] = None

    @property
    def nt(self) -> int:
        return int(self.times.size)

    @property
    def has_tracer(self) -> bool:
        return self.tracer is not None or self.tracer_maker is not None

    def tracer_snapshot(self, s: int):
        if self.tracer_maker is not None:
            return self.tracer_maker(s)
        return None if self.tracer is None else self.tracer[s]

    def materialise_tracer(self):
        if self.tracer is not None or self.tracer_maker is None:
            return self.tracer
        return np.stack([self.tracer_maker(s) for s in range(self.nt)])

    def snapshot(self, s: int):
        if self.maker is not None:
            return self.maker(s)
        W = None if self.W is None else self.W[s]
        return self.U[s], self.V[s], W

    def materialise(self):
        """Return (U, V, W) with the leading time axis, generating if needed."""
        if self.U is not None:
            return self.U, self.V, self.W
        parts = [self.maker(s) for s in range(self.nt)]
        U = np.stack([p[0] for p in parts])
        V = np.stack([p[1] for p in parts])
        W = None if parts[0][2] is None else np.stack([p[2] for p in parts])
        return U, V, W


@dataclass
class Workload:
    name: str
    grid: Grid
    fields: Fields
    lon0: np.ndarray
    lat0: np.ndarray
    depth0: Optional[np.ndarray]
    dt: float
    nsteps: int
    outputdt: float
    t0: float = 0.0
    Kh: float = 0.0
    policy: int = POLICY_DELETE
    run_id: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.lon0.size)

    @property
    def particle_steps(self) -> int:
        return self.n * self.nsteps


def _global_axes(nx: int, ny: int):
    lon = -180.0 + (np.arange(nx, dtype=np.float64) + 0.5) * (360.0 / nx)
    lat = -90.0 + (np.arange(ny, dtype=np.float64) + 0.5) * (180.0 / ny)
    return lon, lat


def _kappa0_cells(cell_m: float, wavelength_m: float = 200e3) -> float:
    """Cutoff wavenumber in cycles per cell for a given eddy wavelength."""
    return cell_m / wavelength_m


# --------------------------------------------------------------------------- cfg0
def cfg0_solid_body(n_particles: int = 10_000, nsteps: int = 1440, dt: float = 60.0,
                    omega: float = 1e-5, outputdt: float = 3600.0) -> Workload:
    """Steady solid-body rotation u = -w (y - 5e4), v = w (x - 5e4) on a flat
    101x101 A-grid, x_i = y_j = 1000 i m, float64 fields; particles area-uniform
    within 4e4 m of the centre."""
    rs = _streams(0)
    x = 1000.0 * np.arange(101, dtype=np.float64)
    X, Y = np.meshgrid(x, x)
    U = (-omega * (Y - 5e4))[None]
    V = (omega * (X - 5e4))[None]
    u1 = rs[4].uniform(0.0, 1.0, n_particles)
    u2 = rs[4].uniform(0.0, 1.0, n_particles)
    r = 4e4 * np.sqrt(u1)
    phi = 2.0 * np.pi * u2
    grid = Grid(lon=x, lat=x.copy(), spherical=False)
    f = Fields(times=np.zeros(1), period=0.0, U=U, V=V)
    return Workload("cfg0_solid_body_101x101_10k", grid, f,
                    5e4 + r * np.cos(phi), 5e4 + r * np.sin(phi), None,
                    dt=dt, nsteps=nsteps, outputdt=outputdt,
                    meta=dict(omega=omega, centre=(5e4, 5e4)))


# --------------------------------------------------------------------------- cfg1
def _eddy_pair(rs, ny, nx, lat, cell_m):
    k0 = _kappa0_cells(cell_m)
    A = random_streamfunction(rs[0], ny, nx, k0)
    B = random_streamfunction(rs[1], ny, nx, k0)
    ua, va = velocity_from_streamfunction(A, lat)
    ub, vb = velocity_from_streamfunction(B, lat)
    return ua, va, ub, vb


def _periodic_2d_snapshots(ua, va, ub, vb, times, period, land):
    w = 2.0 * np.pi / period
    nt = times.size
    U = np.empty((nt,) + ua.shape, np.float64)
    V = np.empty_like(U)
    for s, t in enumerate(times):
        c, sn = np.cos(w * t), np.sin(w * t)
        U[s] = c * ua + sn * ub
        V[s] = c * va + sn * vb
    scale = 1.0 / np.sqrt(U * U + V * V).max()
    U *= scale
    V *= scale
    if land is not None:
        U[:, land != 0] = 0.0
        V[:, land != 0] = 0.0
    return U.astype(np.float32), V.astype(np.float32)


def cfg1_global_eddies(nx: int = 1440, ny: int = 720, nt: int = 30,
                       n_particles: int = 1_000_000, nsteps: int = 8640,
                       dt: float = 300.0, outputdt: float = DAY,
                       period_days: float = 30.0, cfg_index: int = 1,
                       land_fraction: float = 0.30) -> Workload:
    """Global lon/lat grid (0.25 degree at the default size), ``nt`` daily float32
    U, V snapshots periodic with ``period_days``, eddies from a kappa^-3 random
    streamfunction with a 200 km cutoff wavelength (100 km eddies), max speed
    1 m/s, 30% land; particles uniform inside ocean cells."""
    rs = _streams(cfg_index)
    lon, lat = _global_axes(nx, ny)
    cell_m = (360.0 / nx) * METRES_PER_DEGREE
    ua, va, ub, vb = _eddy_pair(rs, ny, nx, lat, cell_m)
    land = smoothed_land_mask(rs[3], ny, nx, land_fraction=land_fraction)
    times = DAY * np.arange(nt, dtype=np.float64)
    period = period_days * DAY
    U, V = _periodic_2d_snapshots(ua, va, ub, vb, times, period, land)
    x0, y0 = seed_in_cells(rs[4], ocean_cell_mask(land), n_particles, lon, lat)
    grid = Grid(lon=lon, lat=lat, spherical=True, land=land)
    return Workload(f"cfg1_eddies_{nx}x{ny}_{n_particles}", grid,
                    Fields(times=times, period=period, U=U, V=V),
                    x0, y0, None, dt=dt, nsteps=nsteps, outputdt=outputdt)


def cfg4_surrogate_field(nx: int = 1440, ny: int = 720, n_particles: int = 4_000_000,
                         nsteps: int = 8640, dt: float = 300.0) -> Workload:
    """The cfg1 grid and land with a 10-day period (10 daily snapshots)."""
    w = cfg1_global_eddies(nx=nx, ny=ny, nt=10, n_particles=n_particles, nsteps=nsteps,
                           dt=dt, period_days=10.0, cfg_index=4)
    w.name = f"cfg4_surrogate_{nx}x{ny}_{n_particles}"
    return w


# --------------------------------------------------------------------------- cfg2
def depth_levels(nz: int = 50, top: float = 5.0, bottom: float = 5000.0) -> np.ndarray:
    """Geometrically stretched levels z_k = top * (bottom/top)^(k/(nz-1))."""
    k = np.arange(nz, dtype=np.float64)
    return top * (bottom / top) ** (k / (nz - 1))


def cfg2_global_3d(nx: int = 3600, ny: int = 1800, nz: int = 50, nt: int = 11,
                   n_particles: int = 10_000_000, nsteps: int = 1440,
                   dt: float = 600.0, outputdt: float = DAY) -> Workload:
    """3D spherical grid (0.1 degree x 50 stretched levels at the default size).
    psi = exp(-z/1500) [cos(wt + z/800) A + sin(wt + z/800) B] gives U, V
    (max speed <= 1 m/s); W = 1e-4 C(x,y) sin(pi (z-5)/4995) cos(wt) m/s;
    w = 2 pi / 30 d; ``nt`` daily snapshots, not periodic, no land.  Snapshots
    are produced on demand (each is 3 x nz x ny x nx float32)."""
    rs = _streams(2)
    lon, lat = _global_axes(nx, ny)
    z = depth_levels(nz)
    cell_m = (360.0 / nx) * METRES_PER_DEGREE
    ua, va, ub, vb = _eddy_pair(rs, ny, nx, lat, cell_m)
    sa = 1.0 / (np.sqrt(2.0) * np.sqrt(ua * ua + va * va).max())
    sb = 1.0 / (np.sqrt(2.0) * np.sqrt(ub * ub + vb * vb).max())
    ua *= sa
    va *= sa
    ub *= sb
    vb *= sb
    C = random_streamfunction(rs[2], ny, nx, _kappa0_cells(cell_m))
    omega = 2.0 * np.pi / (30.0 * DAY)
    times = DAY * np.arange(nt, dtype=np.float64)
    decay = np.exp(-z / 1500.0)
    wprof = 1e-4 * np.sin(np.pi * (z - z[0]) / (z[-1] - z[0]))

    def maker(s: int):
        t = times[s]
        U = np.empty((nz, ny, nx), np.float32)
        V = np.empty_like(U)
        W = np.empty_like(U)
        for k in range(nz):
            c = decay[k] * np.cos(omega * t + z[k] / 800.0)
            sn = decay[k] * np.sin(omega * t + z[k] / 800.0)
            U[k] = c * ua + sn * ub
            V[k] = c * va + sn * vb
            W[k] = (wprof[k] * np.cos(omega * t)) * C
        return U, V, W

    g = rs[4]
    x0 = g.uniform(lon[0], lon[-1], n_particles)
    y0 = g.uniform(lat[0], lat[-1], n_particles)
    d0 = g.uniform(z[0], z[-1], n_particles)
    grid = Grid(lon=lon, lat=lat, depth=z, spherical=True)
    meta = dict(base=(ua, va, ub, vb, C), decay=decay, wprof=wprof, omega=omega)
    return Workload(f"cfg2_3d_{nx}x{ny}x{nz}_{n_particles}", grid,
                    Fields(times=times, period=0.0, maker=maker),
                    x0, y0, d0, dt=dt, nsteps=nsteps, outputdt=outputdt, meta=meta)


def cfg2_snapshot_torch(w: Workload, s: int, device="cuda", cache: Optional[dict] = None):
    """Snapshot s of a cfg2 workload built directly in device memory with torch.
    Same arithmetic as the numpy maker (scalar coefficients in numpy float64, then
    separate float64 products and a sum, rounded to float32), so the values are
    bit-identical."""
    import torch
    m = w.meta
    if cache is None:
        cache = {}
    if "base" not in cache:
        cache["base"] = [torch.from_numpy(a).to(device) for a in m["base"]]
    ua, va, ub, vb, C = cache["base"]
    z = w.grid.depth
    t = w.fields.times[s]
    omega = m["omega"]
    nz, ny, nx = z.size, w.grid.ny, w.grid.nx
    U = torch.empty((nz, ny, nx), dtype=torch.float32, device=device)
    V = torch.empty_like(U)
    W = torch.empty_like(U)
    for k in range(nz):
        c = float(m["decay"][k] * np.cos(omega * t + z[k] / 800.0))
        sn = float(m["decay"][k] * np.sin(omega * t + z[k] / 800.0))
        U[k] = (c * ua + sn * ub).to(torch.float32)
        V[k] = (c * va + sn * vb).to(torch.float32)
        W[k] = (float(m["wprof"][k] * np.cos(omega * t)) * C).to(torch.float32)
    return U, V, W


# --------------------------------------------------------------------------- cfg3
def cfg3_ensemble(n_runs: int = 64, side_min: int = 64, side_max: int = 1024,
                  np_min: int = 1000, np_max: int = 2_000_000, nsteps: int = 1440,
                  dt: float = 300.0, Kh: float = 10.0, nt: int = 5,
                  particle_scale: float = 1.0) -> List[Workload]:
    """64 independent flat runs: square grids with side log-uniform in
    [side_min, side_max] (dx = 10 km), ``nt`` daily float32 U, V snapshots
    periodic over nt days, particle counts log-uniform in [np_min, np_max]
    (times ``particle_scale``), Brownian diffusivity Kh, delete at the edge."""
    rs = _streams(3)
    runs_rng = rs[5]
    u = runs_rng.uniform(0.0, 1.0, n_runs)
    v = runs_rng.uniform(0.0, 1.0, n_runs)
    sides = np.rint(side_min * (side_max / side_min) ** u).astype(int)
    counts = np.rint(np_min * (np_max / np_min) ** v * particle_scale).astype(int)
    counts = np.maximum(counts, 1)
    child = np.random.SeedSequence(BASE_SEED + 3).spawn(7)[6].spawn(n_runs)
    out = []
    period = nt * DAY
    times = DAY * np.arange(nt, dtype=np.float64)
    for r in range(n_runs):
        g = [np.random.Generator(np.random.PCG64(s)) for s in child[r].spawn(3)]
        n = int(sides[r])
        x = 1e4 * np.arange(n, dtype=np.float64)
        k0 = _kappa0_cells(1e4)
        A = random_streamfunction(g[0], n, n, k0)
        B = random_streamfunction(g[1], n, n, k0)
        ua, va = velocity_from_streamfunction(A)
        ub, vb = velocity_from_streamfunction(B)
        U, V = _periodic_2d_snapshots(ua, va, ub, vb, times, period, None)
        np_r = int(counts[r])
        x0 = g[2].uniform(x[0], x[-1], np_r)
        y0 = g[2].uniform(x[0], x[-1], np_r)
        grid = Grid(lon=x, lat=x.copy(), spherical=False)
        out.append(Workload(f"cfg3_run{r}_{n}x{n}_{np_r}", grid,
                            Fields(times=times, period=period, U=U, V=V),
                            x0, y0, None, dt=dt, nsteps=nsteps, outputdt=nsteps * dt,
                            Kh=Kh, run_id=r))
    return out


def foram_footprint(nx: int = 350, ny: int = 300, nz: int = 54, nt: int = 21,
                    n_particles: int = 100_000, dt: float = -300.0,
                    days: int = 42) -> Workload:
    """Stand-in for the worked example of Sect. 4 (virtual foraminifera ending on
    the sea floor off Cape Town, tracked backward in time through a regional
    1/10 degree, 54-level OGCM with 3-day snapshots).  The OFES data is not here:
    the domain 5-40 E, 50-20 S at 0.1 degree, 54 stretched levels (5-5500 m),
    3-day snapshots and a temperature tracer are synthesised.  Velocities as in
    cfg2 (eddies decaying with depth, rotating over 30 days, small W); the
    temperature falls with depth and towards the south, plus eddy anomalies:
    T = 26 - 0.4 (-20 - lat) - 14 (1 - exp(-z / 600)) + 1.5 exp(-z / 300) A(x, y, t)
    (deg C).  All particles start at the core site, 17.3 E 34.7 S, at 2,440 m,
    jittered by up to 0.05 degree; the run goes backward from the last snapshot
    (dt < 0) for ``days`` days with daily output."""
    rs = _streams(5)
    lon = np.linspace(5.0, 40.0, nx)
    lat = np.linspace(-50.0, -20.0, ny)
    z = depth_levels(nz, 5.0, 5500.0)
    cell_m = ((lon[-1] - lon[0]) / (nx - 1)) * METRES_PER_DEGREE
    ua, va, ub, vb = _eddy_pair(rs, ny, nx, lat, cell_m)
    sa = 0.8 / np.sqrt(ua * ua + va * va).max()
    sb = 0.8 / np.sqrt(ub * ub + vb * vb).max()
    ua *= sa
    va *= sa
    ub *= sb
    vb *= sb
    C = random_streamfunction(rs[2], ny, nx, _kappa0_cells(cell_m))
    A = random_streamfunction(rs[3], ny, nx, _kappa0_cells(cell_m))
    omega = 2.0 * np.pi / (30.0 * DAY)
    times = 3.0 * DAY * np.arange(nt, dtype=np.float64)
    decay = np.exp(-z / 1500.0)
    wprof = 5e-5 * np.sin(np.pi * (z - z[0]) / (z[-1] - z[0]))
    base_t = 26.0 - 0.4 * (-20.0 - lat)[:, None] + np.zeros((ny, nx))

    def maker(s: int):
        t = times[s]
        U = np.empty((nz, ny, nx), np.float32)
        V = np.empty_like(U)
        W = np.empty_like(U)
        for k in range(nz):
            c = decay[k] * np.cos(omega * t + z[k] / 800.0)
            sn = decay[k] * np.sin(omega * t + z[k] / 800.0)
            U[k] = c * ua + sn * ub
            V[k] = c * va + sn * vb
            W[k] = (wprof[k] * np.cos(omega * t)) * C
        return U, V, W

    def tracer(s: int):
        t = times[s]
        T = np.empty((nz, ny, nx), np.float32)
        for k in range(nz):
            T[k] = (base_t - 14.0 * (1.0 - np.exp(-z[k] / 600.0))
                    + 1.5 * np.exp(-z[k] / 300.0) * np.cos(omega * t) * A)
        return T

    g = rs[4]
    x0 = 17.3 + g.uniform(-0.05, 0.05, n_particles)
    y0 = -34.7 + g.uniform(-0.05, 0.05, n_particles)
    d0 = np.full(n_particles, 2440.0)
    grid = Grid(lon=lon, lat=lat, depth=z, spherical=True)
    nsteps = int(round(days * DAY / abs(dt)))
    meta = dict(sink_speed=200.0 / DAY, dwell_depth=50.0, maxage=30.0 * DAY)
    return Workload(f"foram_{nx}x{ny}x{nz}_{n_particles}", grid,
                    Fields(times=times, period=0.0, maker=maker, tracer_maker=tracer),
                    x0, y0, d0, dt, nsteps, DAY, t0=float(times[-1]), meta=meta)
