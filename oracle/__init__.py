"""FP64 CPU oracle for the acoustic finite-difference propagator.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the HIP library (paper_2201_05278_amd): its coefficients,
geometry weights, damping and time stepping are computed here from the paper's
equations, independently.

Modules:
  coeffs    finite-difference coefficients, time-step limit, step count
  geometry  Kaiser-windowed sinc and linear point weights
  core      extended model, damping, forward propagation, adjoint, gradient
  wave.c    the per-step stencil update in C (FP64, OpenMP)
"""
from . import coeffs, geometry, core  # noqa: F401
from .core import (Problem, prepare, forward, gradient, gradient_checkpointed,  # noqa: F401
                   geometry_table, ricker, damping, extend, apply_L, step, step_points,
                   injection_terms, fold_to_physical, gradient_vd, face_difference,
                   midpoint_transpose, source_term)
