"""Building blocks for synthetic ocean velocity fields.

The paper's own workloads read OGCM output (NetCDF, e.g. OFES at 1/10 degree,
Sect. 3.1).  No such data exists here, so every workload is synthesised from a
seeded random streamfunction with the shape, resolution and velocity scale of
those fields.  Nothing in this module advects, locates or interpolates.
"""

from __future__ import annotations

import numpy as np
from scipy import ndimage

# metres per degree of arc used when a workload is on a spherical mesh; the same
# constant is used by the generator only to size the eddy wavelength in cells.
METRES_PER_DEGREE = 1852.0 * 60.0


def random_streamfunction(rng: np.random.Generator, ny: int, nx: int,
                          kappa0: float) -> np.ndarray:
    """Gaussian random field on the (ny, nx) index grid with a kappa^-3 amplitude
    spectrum above ``kappa0`` (cycles per cell) and kappa^-3 (kappa/kappa0)^2
    below it; random phases; normalised to unit maximum magnitude."""
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.rfftfreq(nx)[None, :]
    k = np.sqrt(kx * kx + ky * ky)
    amp = np.zeros_like(k)
    nz = k > 0
    amp[nz] = k[nz] ** -3.0
    low = nz & (k < kappa0)
    amp[low] *= (k[low] / kappa0) ** 2
    phase = rng.uniform(0.0, 2.0 * np.pi, size=k.shape)
    spec = amp * np.exp(1j * phase)
    psi = np.fft.irfft2(spec, s=(ny, nx))
    psi /= np.abs(psi).max()
    return psi


def velocity_from_streamfunction(psi: np.ndarray, lat: np.ndarray | None = None):
    """Geostrophic-style velocities u = -dpsi/dy, v = dpsi/dx by centred
    differences in index space (one-sided at the edges).  On a spherical mesh
    both are multiplied by cos(lat) so the angular speed stays bounded at the
    poles.  Returned unscaled, float64, shape (ny, nx)."""
    dpsi_dy, dpsi_dx = np.gradient(psi)
    u = -dpsi_dy
    v = dpsi_dx
    if lat is not None:
        c = np.cos(np.deg2rad(lat))[:, None]
        u = u * c
        v = v * c
    return u, v


def smoothed_land_mask(rng: np.random.Generator, ny: int, nx: int,
                       land_fraction: float = 0.30, sigma: float = 4.0) -> np.ndarray:
    """Node land mask (uint8, 1 = land): Gaussian-smoothed white noise
    thresholded so that ``land_fraction`` of the nodes are land."""
    noise = rng.standard_normal((ny, nx))
    sm = ndimage.gaussian_filter(noise, sigma=sigma, mode="wrap")
    thr = np.quantile(sm, 1.0 - land_fraction)
    return (sm > thr).astype(np.uint8)


def ocean_cell_mask(land: np.ndarray) -> np.ndarray:
    """Cells (ny-1, nx-1) whose four corner nodes are all ocean: the cells in
    which particles are seeded."""
    oc = land == 0
    return oc[:-1, :-1] & oc[:-1, 1:] & oc[1:, :-1] & oc[1:, 1:]


def seed_in_cells(rng: np.random.Generator, cell_mask: np.ndarray, n: int,
                  xc: np.ndarray, yc: np.ndarray):
    """n positions uniform inside cells drawn uniformly among ``cell_mask``."""
    jj, ii = np.nonzero(cell_mask)
    pick = rng.integers(0, jj.size, size=n)
    j = jj[pick]
    i = ii[pick]
    fx = rng.uniform(0.0, 1.0, size=n)
    fy = rng.uniform(0.0, 1.0, size=n)
    x = xc[i] + fx * (xc[i + 1] - xc[i])
    y = yc[j] + fy * (yc[j + 1] - yc[j])
    return x, y
