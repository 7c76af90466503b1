"""MI355X (gfx950) library for the full-multigrid multilevel (quasi-)Monte Carlo
method for single-phase Darcy flow (arXiv:1910.04727).

  fmgmc   - binding of the C ABI (include/fmgmc.h) of the HIP library
  inputs  - seeded synthetic sample points (MC normals, scrambled Sobol')
  build   - builds libfmgmc.so for gfx950 in-tree
"""
