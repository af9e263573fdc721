"""ORACLE - TEST INFRASTRUCTURE ONLY.  Octree-adaptive moving samples.

The Implementation section notes that the skeletal density varies most near
the shape's skeleton and proposes sampling it on an octree, subdividing deeper
where it varies more, so that m' << m nonequispaced samples stand in for the
m nodes of the uniform grid; the samples then meet the fixed grid through a
nonequispaced FFT (nfft.py).  The paper gives no subdivision rule.  Reading
used here:

  * The body box of N_M^3 nodes (planar: N_M^2) carries the coefficients
    c_k = w_k rho_M(x_k) of the uniform quadrature of eq. 8.
  * A cube of 2^l nodes per side, aligned to multiples of 2^l, is a cell of
    level l.  A cell of level 1 <= l <= L is "flat" when, over its nodes,
        max Re c - min Re c < tau   and   max Im c - min Im c < tau,
        tau = tol * A,  A = max_k max(|Re c_k|, |Im c_k|).
    Strict inequalities: tol = 0 merges nothing.
  * Each node belongs to the highest flat cell above it (levels <= L), or is a
    leaf of its own (level 0).  A subset has a smaller spread than its cell,
    so the children of a flat cell are flat and the leaves tile the box.
  * A leaf carries the sum of its nodes' coefficients at the cell centre,
    corner + (2^l - 1) / 2, in grid units from the body origin (node k at
    k - N_M / 2).  Leaves whose nodes are all exactly zero carry nothing and
    are dropped.
  * Order: blocks of 8^3 nodes (planar 8^2) in flat x-fastest order, and
    within a block the leaves in Morton order of their first node (x bit
    lowest, then y, then z, per level), which is depth-first child order.

The spreads, A, tau and the comparisons are done in ``dtype`` (the precision
the GPU library decides in); the sums in FP64.
"""

from __future__ import annotations

import numpy as np

BLOCK = 8  # nodes per block side (the ordering unit); max_level <= 3


def _grid(c, n_m: int, planar: bool) -> np.ndarray:
    c = np.asarray(c)
    return c.reshape((1 if planar else n_m), n_m, n_m)


def octree_leaves(c, n_m: int, tol: float, max_level: int, planar: bool = False, dtype=np.float64):
    """Leaves of the adaptive tree.

    Returns (pos, coef, level, corner): pos (m', 3) float64 centres in grid
    units from the body origin, coef (m',) complex128 sums, level (m',) int,
    corner (m', 3) int node indices (i, j, k) of each leaf's first node.
    """
    if n_m % BLOCK or not 0 <= max_level <= 3:
        raise ValueError("N_M must be a multiple of 8 and 0 <= max_level <= 3")
    g = _grid(c, n_m, planar)
    re = g.real.astype(dtype)
    im = g.imag.astype(dtype)
    amax = max(np.max(np.abs(re)), np.max(np.abs(im)))
    tau = dtype(tol) * dtype(amax)

    out_corner, out_level = [], []

    def flat(i0, j0, k0, s):
        ks = slice(k0, k0 + (1 if planar else s))
        sl = (ks, slice(j0, j0 + s), slice(i0, i0 + s))
        r, m = re[sl], im[sl]
        return (dtype(np.max(r) - np.min(r)) < tau) and (dtype(np.max(m) - np.min(m)) < tau)

    def visit(i0, j0, k0, lev):
        s = 1 << lev
        if lev == 0 or (lev <= max_level and flat(i0, j0, k0, s)):
            out_corner.append((i0, j0, k0))
            out_level.append(lev)
            return
        h = s >> 1
        for ch in range(4 if planar else 8):
            visit(i0 + h * (ch & 1), j0 + h * ((ch >> 1) & 1), k0 + h * ((ch >> 2) & 1), lev - 1)

    nb = n_m // BLOCK
    for bz in range(1 if planar else nb):
        for by in range(nb):
            for bx in range(nb):
                visit(bx * BLOCK, by * BLOCK, bz * BLOCK, 3)

    c64 = g.astype(np.complex128)
    pos, coef, level, corner = [], [], [], []
    for (i0, j0, k0), lev in zip(out_corner, out_level):
        s = 1 << lev
        ks = slice(k0, k0 + (1 if planar else s))
        cell = c64[ks, j0:j0 + s, i0:i0 + s]
        if not np.any(cell != 0):
            continue
        half = 0.5 * (s - 1)
        pos.append((i0 + half - n_m / 2.0, j0 + half - n_m / 2.0, 0.0 if planar else k0 + half - n_m / 2.0))
        coef.append(np.sum(cell))
        level.append(lev)
        corner.append((i0, j0, k0))
    return (np.array(pos, dtype=np.float64).reshape(-1, 3), np.array(coef, dtype=np.complex128),
            np.array(level, dtype=np.int64), np.array(corner, dtype=np.int64).reshape(-1, 3))
