"""ORACLE - TEST INFRASTRUCTURE ONLY.  Peak picking and refinement, FP64.

The search returns the best placements f(tau*) = max f (Formulation
section).  Per rotation:
  * s = max_t Re f(R, t), t* the lowest flat index among exact maxima;
  * the 3 x 3 x 3 values around t* (periodic), ordered dz, dy, dx with dx
    fastest, offsets -1, 0, +1;
  * sub-voxel refinement per axis by the vertex of the parabola through
    (f-, f0, f+): delta = (f- - f+) / (2 (f- - 2 f0 + f+)), clamped to
    [-1/2, 1/2], and 0 when the curvature f- - 2 f0 + f+ is not negative
    (the paper refines by local search; this parabola is the adopted reading).
Across rotations, top-K orders by score descending, ties by rotation index.
"""

from __future__ import annotations

import numpy as np


def peak(vol):
    """-> (score, flat index, (tx, ty, tz))."""
    vol = np.asarray(vol)
    flat = int(np.argmax(vol))  # first maximiser in C order = lowest flat index
    nz, ny, nx = vol.shape
    tz, rem = divmod(flat, ny * nx)
    ty, tx = divmod(rem, nx)
    return float(vol.reshape(-1)[flat]), flat, (tx, ty, tz)


def neighbourhood(vol, t) -> np.ndarray:
    nz, ny, nx = vol.shape
    tx, ty, tz = t
    out = np.empty(27)
    i = 0
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                out[i] = vol[(tz + dz) % nz, (ty + dy) % ny, (tx + dx) % nx]
                i += 1
    return out


def subvoxel(nbhd, t) -> np.ndarray:
    """t + delta (FP64) from the 27 values."""
    f = np.asarray(nbhd, dtype=np.float64).reshape(3, 3, 3)  # [dz, dy, dx]
    f0 = f[1, 1, 1]
    lines = [(f[1, 1, 0], f[1, 1, 2]), (f[1, 0, 1], f[1, 2, 1]), (f[0, 1, 1], f[2, 1, 1])]
    out = np.asarray(t, dtype=np.float64).copy()
    for a, (fm, fp) in enumerate(lines):
        den = fm - 2.0 * f0 + fp
        if den < 0.0:
            out[a] += float(np.clip((fm - fp) / (2.0 * den), -0.5, 0.5))
    return out


def top_k(scores, k: int) -> np.ndarray:
    scores = np.asarray(scores, dtype=np.float64)
    order = np.lexsort((np.arange(len(scores)), -scores))
    return order[:k]
