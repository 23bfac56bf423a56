"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only builds inputs: grids, velocity snapshots, land masks and
particle start positions.  It contains none of the advection arithmetic
(no cell search, no interpolation, no time stepping), so both sides of every
parity test can read the very same arrays without sharing any of the method.
"""

from .fields import (  # noqa: F401
    random_streamfunction,
    velocity_from_streamfunction,
    smoothed_land_mask,
    ocean_cell_mask,
)
from .configs import (  # noqa: F401
    Grid,
    Fields,
    Workload,
    cfg0_solid_body,
    cfg1_global_eddies,
    cfg2_global_3d,
    cfg3_ensemble,
    cfg4_surrogate_field,
    DAY,
)
