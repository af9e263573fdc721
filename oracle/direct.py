"""ORACLE - TEST INFRASTRUCTURE ONLY.  Reference search without the spreading
window, FP64.

Eq. 8 scores a placement tau by f(tau) = int rho_1(p) rho_2(tau^-1 p) dv, and
the affinity is covariant under rigid motions: rho(p, tau S) = rho(tau^-1 p, S).
So the moving part turned by R about its body-box centre c has, at the body
position x (relative to c), the affinity of its turned boundary samples
(q -> c + R (q - c), n -> R n) at c + x, which equals rho_M(c + R^T x).

Here that affinity is evaluated on the body-box nodes themselves, x_k =
h (k - N_M / 2) with N_M even, so the nodes sit on fixed-grid nodes and

    f(R, t) = sum_k w_node rho_R(x_k) rho_F((x_k / h + t) mod N),  score Re f,

with no spreading window and no resampling.  The windowed search of
correlate.py spreads the unturned node values at R x_k with a cubic B-spline
instead; the difference between the two is what the window changes.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import correlate, rotation, sdf


@dataclass
class TurnedSamples:
    q: np.ndarray
    n: np.ndarray
    w: np.ndarray


def body_centre(grid_m, planar: bool = False) -> np.ndarray:
    """c = o_M + h N_M / 2 (a planar box keeps c_z = o_M,z)."""
    o = np.asarray(grid_m.origin, dtype=np.float64)
    nm = grid_m.n[0]
    c = o + 0.5 * grid_m.h * nm
    if planar:
        c[2] = o[2]
    return c


def turned_samples(samples, grid_m, quat, planar: bool = False) -> TurnedSamples:
    """Boundary samples turned by R(quat) about the body-box centre."""
    r = rotation.quat_to_matrix(quat)
    c = body_centre(grid_m, planar)
    q = np.asarray(samples.q, dtype=np.float64)
    n = np.asarray(samples.n, dtype=np.float64)
    return TurnedSamples(c + (q - c) @ r.T, n @ r.T, np.asarray(samples.w, dtype=np.float64).copy())


def turned_box_sdf(samples, grid_m, params, quat, planar: bool = False) -> np.ndarray:
    """rho_R on the body-box nodes, complex (nz, ny, nx)."""
    return sdf.sdf_grid(turned_samples(samples, grid_m, quat, planar), grid_m, params)


def placed_grid(rho_box, n_m: int, shape, w_node: float, planar: bool = False) -> np.ndarray:
    """M(u) = w_node rho_R(x_k) at u = (k - N_M / 2) mod N, zero elsewhere."""
    if n_m % 2:
        raise ValueError("the direct placement needs an even N_M")
    nz, ny, nx = shape
    m = np.zeros(shape, dtype=np.complex128)
    rb = np.asarray(rho_box, dtype=np.complex128).reshape((1 if planar else n_m), n_m, n_m)
    h = n_m // 2
    ks = np.arange(n_m)
    ix = np.mod(ks - h, nx)
    iy = np.mod(ks - h, ny)
    iz = np.zeros(1, dtype=np.int64) if planar else np.mod(ks - h, nz)
    m[np.ix_(iz, iy, ix)] = w_node * rb
    return m


def direct_volume(rho_f, samples, grid_m, params, quat, w_node: float, planar: bool = False) -> np.ndarray:
    """Re f(R, t) for every grid shift t (FFT correlation of correlate.py)."""
    rho_box = turned_box_sdf(samples, grid_m, params, quat, planar)
    m = placed_grid(rho_box, grid_m.n[0], np.asarray(rho_f).shape, w_node, planar)
    return correlate.correlate_fft(rho_f, m).real
