"""ORACLE - TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 CPU implementation of what the scoring hot path
computes, written from the paper's definitions.  Only ``tests/``, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may
import it.  It shares no code with the GPU package (no kernels, headers,
helpers, tables or constants); both sides only share the seeded input
generators in ``workloads``.

Modules:
  sdf       skeletal density function on grids / points (eq. 10A-17t)
  rotation  unit quaternion -> rotation matrix and its derivative
  spread    cubic B-spline spreading of body-box samples onto the grid
  correlate score volumes f(R, t) = Re sum_p rho_F(p) M_R(p - t) (eq. 8)
  peak      per-rotation peak, 27-neighbourhood, sub-voxel refinement, top-K
  grad      pose value and gradients of the score, finite differences
  octree    octree-adaptive aggregation of the moving samples
  nfft      nonequispaced route: type-1 transform (definition and spread/FFT/
            deconvolution algorithm), trigonometric-interpolation scores

Functions whose result the tests cannot pin to anything but themselves say
"parity unpinned" in their docstring.
"""
