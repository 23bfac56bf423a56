"""Inputs of the paper's idealised test cases (Sect. 4.2), built as gridded fields.

Only the inputs are built here: the grid, the sampled velocities and the particle
starts.  Where the paper leaves a number unstated, the value chosen is noted.
"""

from __future__ import annotations

import numpy as np

from .configs import DAY, Fields, Grid, Workload


def radial_rotation(dt: float = 300.0, hours: float = 24.0) -> Workload:
    """Sect. 4.2.1: counter-clockwise solid-body rotation with a 24 h period on a
    20 km x 20 km A-grid centred at the origin, 100 m resolution; four particles
    at x = 0 and y = 1000, 2000, 3000, 4000 (metres: the text's "km" cannot fit
    the 20 km domain); hourly output."""
    omega = 2.0 * np.pi / DAY
    x = -1e4 + 100.0 * np.arange(201, dtype=np.float64)
    X, Y = np.meshgrid(x, x)
    U = (-omega * Y)[None]
    V = (omega * X)[None]
    y0 = np.array([1000.0, 2000.0, 3000.0, 4000.0])
    return Workload("paper_radial_rotation", Grid(lon=x, lat=x.copy()),
                    Fields(times=np.zeros(1), U=U, V=V),
                    np.zeros(4), y0, None, dt=dt, nsteps=int(round(hours * 3600 / dt)),
                    outputdt=3600.0, meta=dict(omega=omega))


def zonal_flow_sphere(days: float = 57.0, dt: float = 300.0) -> Workload:
    """Sect. 4.2.2: uniform 1 m/s zonal flow, no meridional flow, on a 1 degree
    spherical grid (lon in [-180, 180], lat in [-89, 89]); 31 particles on a
    north-south line at lon 0 with 3 degree spacing, lat0 = -45 + 3 m; daily
    output."""
    lon = np.arange(-180.0, 180.0 + 0.5, 1.0)
    lat = np.arange(-89.0, 89.0 + 0.5, 1.0)
    U = np.ones((1, lat.size, lon.size))
    V = np.zeros_like(U)
    lat0 = -45.0 + 3.0 * np.arange(31)
    return Workload("paper_zonal_sphere", Grid(lon=lon, lat=lat, spherical=True),
                    Fields(times=np.zeros(1), U=U, V=V),
                    np.zeros(31), lat0, None, dt=dt, nsteps=int(round(days * DAY / dt)),
                    outputdt=DAY)


def oscillating_zonal_flow(days: float = 4.0, dt: float = 300.0, A: float = 0.1,
                           period: float = DAY, field_dt: float = 300.0) -> Workload:
    """Sect. 4.2.3: v = A, u(t) = A cos(w t), w = 2 pi / 1 day, sampled every
    5 minutes on a grid with two cells per direction (nodes -1e5, 0, 1e5 m);
    20 particles on y = 0 at x0 = 100 m * m, m = 0..19; 3-hourly output."""
    nodes = np.array([-1e5, 0.0, 1e5])
    nt = int(round(days * DAY / field_dt)) + 1
    times = field_dt * np.arange(nt, dtype=np.float64)
    w = 2.0 * np.pi / period
    U = np.empty((nt, 3, 3))
    V = np.empty((nt, 3, 3))
    for s, t in enumerate(times):
        U[s] = A * np.cos(w * t)
        V[s] = A
    x0 = 100.0 * np.arange(20, dtype=np.float64)
    return Workload("paper_oscillating_zonal", Grid(lon=nodes, lat=nodes.copy()),
                    Fields(times=times, U=U, V=V),
                    x0, np.zeros(20), None, dt=dt, nsteps=int(round(days * DAY / dt)),
                    outputdt=3 * 3600.0, meta=dict(A=A, omega=w))


def brownian_uniform_kh(n_particles: int = 100_000, Kh: float = 100.0, days: float = 1.0,
                        dt: float = 300.0) -> Workload:
    """Sect. 4.2.7: zero velocity on a 60 km x 60 km grid centred at the origin
    (1 km resolution, not stated in the text), all particles released at the
    origin, uniform Kh, diffused for one day."""
    x = -3e4 + 1000.0 * np.arange(61, dtype=np.float64)
    U = np.zeros((1, 61, 61))
    return Workload("paper_brownian", Grid(lon=x, lat=x.copy()),
                    Fields(times=np.zeros(1), U=U, V=U.copy()),
                    np.zeros(n_particles), np.zeros(n_particles), None,
                    dt=dt, nsteps=int(round(days * DAY / dt)), outputdt=days * DAY, Kh=Kh)
