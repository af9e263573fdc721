"""ORACLE - TEST INFRASTRUCTURE ONLY.  Adjoint of the skeletal density
function with respect to its boundary samples, FP64.

For a complex cotangent field g on the query points, L = Re sum_p g(p) rho(p)
with rho the SDF of sdf.py (eq. 13, kernel of eq. 15 / 16c, truncated as in
eq. 17t).  At a live point p with nearest sample q* (distance xi), sign
lambda and the samples j of its contact ball (eta_j <= (1 + eps) xi):

    rho = A sum_j w_j c_j K(r_j),   A = lambda / (2 pi sigma xi^2),
    d_j = p - q_j, eta_j = |d_j|, u_j = d_j / eta_j, c_j = u_j . n_j, r_j = eta_j / xi,
    K(r) = G(r) P(r) / (1 + r^2)^2,  G = exp(-(r - 1)^2 / (2 sigma^2)),
    P(r) = (1 - r^2) + i s r  (s = -2 outside, +2 inside),
    K'(r) = -K (r - 1) / sigma^2 + G (-2 r + i s) / (1 + r^2)^2 - 4 r K / (1 + r^2).

With the discrete choices held (nearest sample, membership, ball), the
derivatives are
    d rho / d w_j = A c_j K(r_j),
    d rho / d n_j = A w_j K(r_j) u_j,
    d rho / d q_j = A w_j [ -K(r_j) (n_j - c_j u_j) / eta_j - c_j K'(r_j) u_j / xi ],
and through xi = |p - q*|, for the nearest sample only,
    d rho / d xi = -(2 rho + A sum_j w_j c_j K'(r_j) r_j) / xi,  d xi / d q* = -u*.
The gradients are dL/d theta = Re sum_p g(p) d rho(p) / d theta.
"""

from __future__ import annotations

import math

import numpy as np


def sdf_adjoint_points(samples, points, params, cot):
    """(dL/dq (n, 3), dL/dn (n, 3), dL/dw (n,)) for L = Re sum_p cot_p rho(p)."""
    q = np.asarray(samples.q, dtype=np.float64)
    nrm = np.asarray(samples.n, dtype=np.float64)
    w = np.asarray(samples.w, dtype=np.float64)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    cot = np.asarray(cot, dtype=np.complex128).ravel()
    sig = params.sigma
    gq = np.zeros_like(q)
    gn = np.zeros_like(q)
    gw = np.zeros(len(w))
    for p, g in zip(pts, cot):
        if g == 0:
            continue
        d = p - q
        eta2 = np.einsum("ij,ij->i", d, d)
        js = int(np.argmin(eta2))  # lowest index on exact ties
        xi = math.sqrt(eta2[js])
        dot = float(d[js] @ nrm[js])
        pmc = 1 if dot > 0 else (-1 if dot < 0 else 0)
        if pmc == 0 or xi < params.xi_floor:
            continue
        lam = params.lambda1 if pmc > 0 else -params.lambda2
        s = -2.0 if pmc > 0 else 2.0
        A = lam / (2.0 * math.pi * sig * xi * xi)
        ball = np.nonzero(eta2 <= (1.0 + params.eps) ** 2 * eta2[js])[0]
        db = d[ball]
        eta = np.sqrt(eta2[ball])
        u = db / eta[:, None]
        c = np.einsum("ij,ij->i", u, nrm[ball])
        r = eta / xi
        G = np.exp(-(r - 1.0) ** 2 / (2.0 * sig * sig))
        P = (1.0 - r * r) + 1j * s * r
        den = 1.0 + r * r
        K = G * P / den ** 2
        Kp = -K * (r - 1.0) / sig ** 2 + G * (-2.0 * r + 1j * s) / den ** 2 - 4.0 * r * K / den
        wb = w[ball]
        rho = A * np.sum(wb * c * K)
        gw[ball] += np.real(g * A * c * K)
        gn[ball] += np.real(g * A * wb * K)[:, None] * u
        t1 = np.real(g * A * wb * K)[:, None] * (-(nrm[ball] - c[:, None] * u) / eta[:, None])
        t2 = np.real(g * A * wb * c * Kp)[:, None] * (-u / xi)
        gq[ball] += t1 + t2
        dxi = -(2.0 * rho + A * np.sum(wb * c * Kp * r)) / xi
        gq[js] += np.real(g * dxi) * (-(d[js] / xi))
    return gq, gn, gw


def sdf_adjoint_grid(samples, grid, params, cot):
    """Same, with the query points the nodes of ``grid`` and cot shaped like it."""
    return sdf_adjoint_points(samples, grid.node_positions(), params, np.asarray(cot).ravel())
