"""ORACLE - TEST INFRASTRUCTURE ONLY.  Cubic B-spline spreading, FP64.

The score of eq. 8 integrates rho_F(p) rho_M(tau^-1 p).  The moving part's
affinity is sampled once on its body box (its nodes x_k, weights w_k); a
rotated copy meets the fixed grid through the tensor cubic B-spline window

    M_R(u) = sum_k c_k B3(u - y_k),  c_k = w_k rho_M(x_k),  y_k = R x_k / h,
    B3(s) = beta(s_x) beta(s_y) beta(s_z),
    beta(s) = 2/3 - s^2 + |s|^3 / 2      for |s| < 1,
              (2 - |s|)^3 / 6            for 1 <= |s| < 2,
              0                          otherwise,

with u taken modulo the grid (the correlation is circular).  This is the
window reading adopted for the paper's unspecified resampling step (the
nonequispaced route of the Implementation section moves SDF samples).
"""

from __future__ import annotations

import numpy as np


def bspline3(s):
    a = np.abs(np.asarray(s, dtype=np.float64))
    return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3,
                    np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def bspline3_deriv(s):
    s = np.asarray(s, dtype=np.float64)
    a = np.abs(s)
    sg = np.sign(s)
    return np.where(a < 1.0, -2.0 * s + 1.5 * a * s,
                    np.where(a < 2.0, -0.5 * sg * (2.0 - a) ** 2, 0.0))


def body_positions(n_m: int, planar: bool = False) -> np.ndarray:
    """Body-box node positions in grid units, k - n_m/2, flat x-fastest order.
    Planar boxes have one layer at body height 0."""
    if planar:
        j, i = np.meshgrid(np.arange(n_m), np.arange(n_m), indexing="ij")
        return np.stack([i.ravel() - n_m / 2.0, j.ravel() - n_m / 2.0, np.zeros(i.size)], axis=1)
    k, j, i = np.meshgrid(np.arange(n_m), np.arange(n_m), np.arange(n_m), indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) - n_m / 2.0


def spread(c, pos, shape) -> np.ndarray:
    """M(u) = sum_k c_k B3(u - pos_k), u on the periodic grid of ``shape``
    = (nz, ny, nx).  Each sample touches its 4 x 4 x 4 support nodes."""
    nz, ny, nx = shape
    c = np.asarray(c, dtype=np.complex128).ravel()
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    base = np.floor(pos).astype(np.int64) - 1
    out = np.zeros(nz * ny * nx, dtype=np.complex128)
    wx = [bspline3(base[:, 0] + a - pos[:, 0]) for a in range(4)]
    wy = [bspline3(base[:, 1] + a - pos[:, 1]) for a in range(4)]
    wz = [bspline3(base[:, 2] + a - pos[:, 2]) for a in range(4)]
    for cz in range(4):
        iz = np.mod(base[:, 2] + cz, nz)
        for cy in range(4):
            iy = np.mod(base[:, 1] + cy, ny)
            for cx in range(4):
                ix = np.mod(base[:, 0] + cx, nx)
                val = c * (wx[cx] * wy[cy] * wz[cz])
                flat = (iz * ny + iy) * nx + ix
                out += np.bincount(flat, weights=val.real, minlength=out.size) \
                    + 1j * np.bincount(flat, weights=val.imag, minlength=out.size)
    return out.reshape(shape)


def spread_bruteforce(c, pos, shape) -> np.ndarray:
    """Same quantity by summing every sample's periodised window at every node
    (O(nodes x samples); tiny grids only)."""
    nz, ny, nx = shape
    c = np.asarray(c, dtype=np.complex128).ravel()
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(shape, dtype=np.complex128)
    dims = (nx, ny, nz)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                u = np.array([x, y, z], dtype=np.float64)
                tot = 0.0
                w = np.ones(len(c))
                for a in range(3):
                    d = u[a] - pos[:, a]
                    # periodise: sum over images within the window's support
                    acc = np.zeros(len(c))
                    for m in range(-3, 4):
                        acc += bspline3(d + m * dims[a])
                    w = w * acc
                tot = (c * w).sum()
                out[z, y, x] = tot
    return out
