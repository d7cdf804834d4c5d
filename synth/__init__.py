"""Seeded synthetic Lyman-alpha surveys in CSR layout.

This package only *makes inputs*: quasar sky positions, pixel wavelengths,
comoving distances, deltas and weights.  It holds none of the correlation
method's arithmetic (no pair separations, binning, sums or projections), so
both the CPU oracle and the GPU path can read what it writes.
"""
from .survey import (  # noqa: F401
    Forests,
    Grid,
    comoving_distance,
    concat_realisations,
    make_patch,
    sky_cells,
    subset_forests,
    uniform_grid,
)
from .configs import CONFIGS, make_config  # noqa: F401
