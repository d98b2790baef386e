"""CPU oracle for generalized non-exponential Gaussian splatting (FP64).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the rendering library never does,
and nothing here is a fallback for it.  It shares no code with the HIP path.

Modules
  operators  the discrete image-formation operators on one pixel's sorted
             sequence of opacities (Sec. 4: eq. generalized_gaussian,
             eq. nexp_p, Table 1), plus the back-to-front recursion of the
             Russian-roulette appendix as an independent check.
  sh         real spherical harmonics up to degree 3 (directional emission).
  project    per-Gaussian camera projection in FP64: EWA footprint, conic,
             colour (Sec. 3: opacity alpha = aleph * K).
  keys       the tile-binning key specification replayed in IEEE float32
             (depth bits and covered tiles), and the sorted instance list.
  render     per-pixel plain composite: every visible Gaussian evaluated at
             the pixel centre, sorted front to back, composited in FP64.
  adjoint    the operators' adjoints on one sequence (the appendix "Adjoints"
             for linear and quadratic; the front-to-back form for exponential).
"""
from . import operators, sh, project, keys, render, adjoint  # noqa: F401
