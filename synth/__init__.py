"""Seeded synthetic inputs for the reaction-diffusion solve.

This package only *generates data*: lattices, masks, tumour-cell labels and
per-species coefficient fields.  It contains none of the solver's arithmetic
(no face conductances, no matrix, no right-hand side), so both the HIP library
and the CPU oracle can consume its arrays without sharing method code.

Conventions shared by every generator:

* lattice arrays are C-ordered ``[z][y][x]`` (x fastest); multi-species arrays
  are ``[S][z][y][x]``;
* sizes, box corners and centres are given in ``(x, y, z)`` order;
* voxel centres sit at ``index + 1/2``;
* every random draw comes from ``numpy.random.Generator(PCG64(seed))``.
"""

from .geometry import (  # noqa: F401
    Problem,
    config1,
    config2,
    config2_dense,
    config3_tumour,
    config4_patch,
    config5,
    cube,
    dilate6,
    fourier_box,
    random_problem,
    species_constants,
    tumour_coefficients,
)
