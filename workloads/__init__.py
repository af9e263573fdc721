"""Seeded synthetic inputs shared by the oracle, the tests and the bench.

This package only *generates inputs*: boundary point samples of analytic
solids (position, outward normal, quadrature weight), rotation sets and pose
perturbations, grid and parameter records.  It holds none of the scoring
method's arithmetic (no affinity, no spreading, no correlation), so both the
CPU oracle and the GPU path can consume it without sharing method code.
"""

from .shapes import PointSamples  # noqa: F401
from .configs import GridSpec, SDFParams, PartSpec, PairSpec  # noqa: F401
