"""Seeded synthetic tensor-train inputs shared by the oracle tests, the GPU
parity tests, ``smoke()`` and ``bench.py``.

This package holds no arithmetic of the cross-interpolation method itself:
only random cores, QR/SVD compression of sampled functions (a different
algorithm from the pivoted-LU cross interpolation being tested), quantics
grids, and brute-force evaluation of a TT at points.
"""

from .tt import (
    random_tt,
    left_orthogonalise,
    tt_full,
    tt_eval,
    tt_svd,
    tt_round,
    tt_ranks,
    tt_scale,
)
from .fields import (
    quantics_points_1d,
    quantics_to_grid,
    grid_to_quantics,
    gaussian_pair_full,
    fourier1d_coeffs,
    fourier1d_full,
    fourier1d_product_coeffs,
    fourier3d_modes,
    fourier3d_full,
    gp_vortex_full,
)
from .configs import (
    random_pair,
    fourier3d_pair,
    fourier3d_field,
    gp_field,
    random_init,
    velocity_set,
    min_ranks,
)

__all__ = [
    "random_tt", "left_orthogonalise", "tt_full", "tt_eval", "tt_svd",
    "tt_ranks", "tt_scale", "tt_round",
    "quantics_points_1d", "quantics_to_grid", "grid_to_quantics",
    "gaussian_pair_full", "fourier1d_coeffs", "fourier1d_full",
    "fourier1d_product_coeffs", "fourier3d_modes", "fourier3d_full",
    "gp_vortex_full",
    "random_pair", "fourier3d_pair", "fourier3d_field", "gp_field", "random_init", "velocity_set", "min_ranks",
]
