"""ORACLE - TEST INFRASTRUCTURE ONLY.  Alternative phi-kernels of the affinity, FP64.

The paper presents the boundary integral of eq. 13 as a platform on which
scoring schemes differ only in their kernel phi (Formulation section, the
discussion before eq. 15 and Figure 8), and compares its own kernel (eq. 15)
with the radial-basis affinities of eq. 2 and the double-skin-layer (DSL)
affinity of eq. 3a (Our Approach section).  This module evaluates those
alternatives by brute force over the boundary samples, in plain NumPy:

  "skeletal"        eq. 15 / 16c / 17t, delegated to ``oracle.sdf``.
  "inverse_square"  phi(zeta) = lambda(zeta) / sqrt(2 pi) * g_sigma(0) * zeta^-2:
                    eq. 15 with its medial component (the Gaussian of
                    |tan arg zeta| - 1) held at its peak value, so |phi| is
                    proportional to |zeta|^-2 (Figure 8, middle) and the phase
                    -2 arg zeta of the proximal component is kept.  Membership,
                    the distance floor and the contact-region truncation
                    |p - q| <= (1 + eps) |xi| are those of the skeletal kernel.
  "radial"          eq. 2 in the continuum form the paper derives from it: the
                    skin and the core are the +R and -R offsets of the boundary
                    (the core as a negative offset shell), every offset point a
                    Gaussian shell of radius R, integrated by point quadrature
                    over the same samples:
                      rho(p) = sum_j w_j [lambda1 gb(|p - q_j - R n_j| / R - 1)
                                          + i lambda2 gb(|p - q_j + R n_j| / R - 1)].
  "dsl"             eq. 3a on the signed distance xi of the nearest sample:
                      rho(p) = lambda1 gb(xi / R - 1) + i lambda2 gb(xi / R + 1).

g_sigma(x) = exp(-x^2 / (2 sigma^2)) / (sqrt(2 pi) sigma) is the Gauss function
of eq. 15 and gb its truncation to |x| <= eps, the truncated Gaussian the
Formulation section defines next to eq. 17t.  R > 0 is the probe radius of
eq. 2 / 3a (grid units of length, like the sample positions).
"""

from __future__ import annotations

import math

import numpy as np

from . import sdf as osdf

KINDS = ("skeletal", "inverse_square", "radial", "dsl")


def gauss(x, sigma):
    """g_sigma of eq. 15."""
    return np.exp(-0.5 * (np.asarray(x) / sigma) ** 2) / (math.sqrt(2.0 * math.pi) * sigma)


def gauss_trunc(x, sigma, eps):
    """The truncated Gaussian: g_sigma(x) where |x| <= eps, else 0."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(np.abs(x) <= eps, gauss(x, sigma), 0.0)


def _nearest(q, nrm, pp):
    """Signed distance of eq. 10A for sampled boundaries: nearest sample by
    squared distance (lowest index on exact ties), sign from its normal."""
    d = pp[:, None, :] - q[None, :, :]
    d2 = (d * d).sum(-1)
    j = np.argmin(d2, axis=1)
    rows = np.arange(len(pp))
    xi_abs = np.sqrt(d2[rows, j])
    pmc = np.sign((d[rows, j] * nrm[j]).sum(-1))
    return pmc, xi_abs, d, d2


def inverse_square_points(samples, points, params, chunk: int = 256):
    """eq. 13 with phi = lambda(zeta) g_sigma(0) / (sqrt(2 pi) zeta^2), truncated as eq. 17t."""
    q, nrm, w = samples.q, samples.n, samples.w
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(len(p), dtype=np.complex128)
    peak = gauss(0.0, params.sigma)
    for a in range(0, len(p), chunk):
        pp = p[a:a + chunk]
        pmc, xi_abs, d, d2 = _nearest(q, nrm, pp)
        eta = np.sqrt(d2)
        xi = pmc * xi_abs
        valid = (pmc != 0) & (xi_abs >= params.xi_floor)
        lam = np.where(xi > 0, params.lambda1, -params.lambda2)             # eq. 16c
        with np.errstate(divide="ignore", invalid="ignore"):
            zeta = xi[:, None] + 1j * eta                                      # eq. 11
            phi = lam[:, None] / math.sqrt(2.0 * math.pi) * peak / zeta ** 2
            cos_t = (d * nrm[None, :, :]).sum(-1) / eta                        # eq. 12a
            term = phi * cos_t * w[None, :]
        inside = eta <= (1.0 + params.eps) * xi_abs[:, None]                   # eq. 10b / 17t
        out[a:a + chunk] = np.where(inside & valid[:, None], term, 0.0).sum(axis=1)
    return out


def radial_points(samples, points, params, radius, chunk: int = 256):
    """eq. 2 with skin and core shells on the +R / -R offsets of the boundary."""
    q, nrm, w = samples.q, samples.n, samples.w
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    skin = q + radius * nrm
    core = q - radius * nrm
    out = np.zeros(len(p), dtype=np.complex128)
    for a in range(0, len(p), chunk):
        pp = p[a:a + chunk]
        e_skin = np.sqrt(((pp[:, None, :] - skin[None, :, :]) ** 2).sum(-1))
        e_core = np.sqrt(((pp[:, None, :] - core[None, :, :]) ** 2).sum(-1))
        g_skin = gauss_trunc(e_skin / radius - 1.0, params.sigma, params.eps)
        g_core = gauss_trunc(e_core / radius - 1.0, params.sigma, params.eps)
        out[a:a + chunk] = params.lambda1 * (g_skin * w[None, :]).sum(1) + \
            1j * params.lambda2 * (g_core * w[None, :]).sum(1)
    return out


def dsl_points(samples, points, params, radius, chunk: int = 256):
    """eq. 3a on the sampled signed distance (defined on the boundary too)."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(len(p), dtype=np.complex128)
    for a in range(0, len(p), chunk):
        pmc, xi_abs, _, _ = _nearest(samples.q, samples.n, p[a:a + chunk])
        xi = pmc * xi_abs
        out[a:a + chunk] = params.lambda1 * gauss_trunc(xi / radius - 1.0, params.sigma, params.eps) + \
            1j * params.lambda2 * gauss_trunc(xi / radius + 1.0, params.sigma, params.eps)
    return out


def phi_points(samples, points, params, kind: str, radius: float = 0.0):
    """Affinity with kernel ``kind`` at points (m, 3) -> complex128 (m,)."""
    if kind == "skeletal":
        return osdf.sdf_points(samples, points, params)
    if kind == "inverse_square":
        return inverse_square_points(samples, points, params)
    if kind == "radial":
        return radial_points(samples, points, params, radius)
    if kind == "dsl":
        return dsl_points(samples, points, params, radius)
    raise ValueError(f"unknown kernel {kind}")


def phi_grid(samples, grid, params, kind: str, radius: float = 0.0):
    """Affinity on every node of ``grid`` -> complex128 (nz, ny, nx)."""
    nx, ny, nz = grid.n
    return phi_points(samples, grid.node_positions(), params, kind, radius).reshape(nz, ny, nx)
