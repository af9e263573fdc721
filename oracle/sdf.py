"""ORACLE - TEST INFRASTRUCTURE ONLY.  Skeletal density function in FP64.

rho(p, S) = sum over boundary samples of phi(zeta(p, q_j)) cos theta_j w_j
(eq. 13, a point quadrature of the boundary integral) with the kernel of
eq. 15 / 16c, the zeta-map of eq. 11 ("+" branch), signed distance and
membership of eq. 10A, the gaze angle of eq. 12a, and the truncation to the
eps-approximate contact region of eq. 10b / 17t.  rho := 0 where the query
point is classified on the boundary (pmc = 0) or closer to it than the floor
xi_floor (the kernel is singular there; the paper leaves rho undefined on
the boundary).

Two implementations of the same definition:
  * ``sdf_points_numpy``: vectorised NumPy, complex arithmetic written as
    the paper's formulas, for small inputs;
  * ``sdf_points``: the plain C loop in csdf.c (OpenMP), for grids.
"""

from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(_build.build())
        d = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        lib.oracle_sdf_points.argtypes = [d, d, d, ctypes.c_long, d, ctypes.c_long,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, d, d, d, lp, d, d, d, ctypes.c_double]
        lib.oracle_sdf_points.restype = None
        _lib = lib
    return _lib


def _ptr(a, t=ctypes.c_double):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(t))


def sdf_points(samples, points, params, diagnostics: bool = False, band_rel: float = 1e-4):
    """rho at arbitrary points (m, 3) -> complex128 (m,).  With diagnostics,
    also returns a dict of per-point signed xi, nearest index, truncation
    margin, near-edge band magnitude and opposite-side gap."""
    lib = _load()
    q = np.ascontiguousarray(samples.q, dtype=np.float64)
    n = np.ascontiguousarray(samples.n, dtype=np.float64)
    w = np.ascontiguousarray(samples.w, dtype=np.float64)
    p = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 3))
    m = len(p)
    re = np.empty(m)
    im = np.empty(m)
    diag = None
    if diagnostics:
        diag = {"xi": np.empty(m), "nearest": np.empty(m, dtype=np.int64), "trunc_margin": np.empty(m),
                "band_mag": np.empty(m), "pmc_gap": np.empty(m)}
    lib.oracle_sdf_points(_ptr(q), _ptr(n), _ptr(w), len(w), _ptr(p), m,
                          params.lambda1, params.lambda2, params.sigma, params.eps, params.xi_floor,
                          _ptr(re), _ptr(im),
                          _ptr(diag["xi"]) if diag else None,
                          _ptr(diag["nearest"], ctypes.c_long) if diag else None,
                          _ptr(diag["trunc_margin"]) if diag else None,
                          _ptr(diag["band_mag"]) if diag else None,
                          _ptr(diag["pmc_gap"]) if diag else None,
                          band_rel)
    rho = re + 1j * im
    return (rho, diag) if diagnostics else rho


def sdf_grid(samples, grid, params):
    """rho on every node of ``grid`` -> complex128 array shaped (nz, ny, nx)."""
    rho = sdf_points(samples, grid.node_positions(), params)
    nx, ny, nz = grid.n
    return rho.reshape(nz, ny, nx)


def sdf_points_numpy(samples, points, params, chunk: int = 256):
    """Same definition, NumPy, complex arithmetic as printed (small inputs)."""
    q, nrm, w = samples.q, samples.n, samples.w
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(len(p), dtype=np.complex128)
    s2pi = math.sqrt(2.0 * math.pi)
    sig = params.sigma
    for a in range(0, len(p), chunk):
        pp = p[a:a + chunk]
        d = pp[:, None, :] - q[None, :, :]                    # p - q
        d2 = (d * d).sum(-1)
        eta = np.sqrt(d2)                                      # eq. 10A, pairwise distance
        # nearest sample: the minimiser of the exact distance, decided on the
        # squared distance (two distinct squared distances can round to one
        # square root); the first minimiser = lowest index on exact ties
        j = np.argmin(d2, axis=1)
        xi_abs = eta[np.arange(len(pp)), j]
        dot = (d[np.arange(len(pp)), j] * nrm[j]).sum(-1)
        pmc = np.sign(dot)
        xi = pmc * xi_abs
        valid = (pmc != 0) & (xi_abs >= params.xi_floor)
        lam = np.where(xi > 0, params.lambda1, -params.lambda2)   # eq. 16c
        with np.errstate(divide="ignore", invalid="ignore"):
            zeta = xi[:, None] + 1j * eta                          # eq. 11
            tan_abs = eta / xi_abs[:, None]                        # |tan arg zeta|
            g = np.exp(-0.5 * ((tan_abs - 1.0) / sig) ** 2) / (s2pi * sig)
            phi = lam[:, None] / s2pi / zeta ** 2 * g              # eq. 15
            cos_t = (d * nrm[None, :, :]).sum(-1) / eta            # eq. 12a
            term = phi * cos_t * w[None, :]
        inside = eta <= (1.0 + params.eps) * xi_abs[:, None]       # eq. 10b
        term = np.where(inside & valid[:, None], term, 0.0)
        out[a:a + chunk] = term.sum(axis=1)
    return out
