"""Rotation sets and pose perturbations (inputs only).

Quaternions are unit, Hamilton convention, scalar first: (w, x, y, z).
The search decomposes rigid motions into a finite rotation set times all
grid translations (Implementation section); these generators produce the
rotation sets used by the synthetic workloads:

  * planar: rotations by 10 degree steps about +z (2D workload);
  * Hopf-fibration grid (Yershova, Jain, LaValle & Mitchell 2010): HEALPix
    pixel centres on S^2 (Gorski et al. 2005, ring scheme) times equally
    spaced points on the S^1 fibre;
  * seeded uniform random unit quaternions (Shoemake 1992).
"""

from __future__ import annotations

import math

import numpy as np


def planar_rotations(step_deg: float = 10.0, count: int = 36) -> np.ndarray:
    """Rotations by k * step about +z, right-handed, k = 0..count-1."""
    th = np.deg2rad(step_deg) * np.arange(count)
    q = np.zeros((count, 4))
    q[:, 0] = np.cos(th / 2.0)
    q[:, 3] = np.sin(th / 2.0)
    return q


def healpix_ring_centres(nside: int):
    """(theta, phi) of the 12 nside^2 HEALPix pixel centres, ring ordering.

    Closed forms from Gorski et al. (2005), pix2ang in the RING scheme.
    """
    npix = 12 * nside * nside
    ncap = 2 * nside * (nside - 1)
    th = np.empty(npix)
    ph = np.empty(npix)
    for p in range(npix):
        if p < ncap:  # north polar cap
            i = int((1 + math.isqrt(1 + 2 * p)) // 2)
            # guard the integer square root against off-by-one on boundaries
            while 2 * i * (i - 1) > p:
                i -= 1
            while 2 * (i + 1) * i <= p:
                i += 1
            j = p + 1 - 2 * i * (i - 1)
            z = 1.0 - i * i / (3.0 * nside * nside)
            phi = math.pi / (2.0 * i) * (j - 0.5)
        elif p < npix - ncap:  # equatorial belt
            pp = p - ncap
            i = pp // (4 * nside) + nside
            j = pp % (4 * nside) + 1
            s = (i - nside + 1) % 2
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
            phi = math.pi / (2.0 * nside) * (j - s / 2.0)
        else:  # south polar cap
            pp = npix - p
            i = int((1 + math.isqrt(2 * pp - 1)) // 2)
            while 2 * i * (i - 1) >= pp:
                i -= 1
            while 2 * (i + 1) * i < pp:
                i += 1
            j = 4 * i + 1 - (pp - 2 * i * (i - 1))
            z = -1.0 + i * i / (3.0 * nside * nside)
            phi = math.pi / (2.0 * i) * (j - 0.5)
        th[p] = math.acos(max(-1.0, min(1.0, z)))
        ph[p] = phi
    return th, ph


def hopf_grid(level: int = 1) -> np.ndarray:
    """Hopf-fibration SO(3) grid: 72 * 8^level quaternions.

    Level l uses HEALPix nside = 2^l (12 * 4^l cells on S^2) and 6 * 2^l
    fibre angles psi_k = (k + 1/2) * 2 pi / (6 * 2^l).
    q = (cos(t/2) cos(psi/2), cos(t/2) sin(psi/2),
         sin(t/2) cos(phi + psi/2), sin(t/2) sin(phi + psi/2)).
    """
    nside = 2 ** level
    th, ph = healpix_ring_centres(nside)
    m = 6 * 2 ** level
    psi = (np.arange(m) + 0.5) * (2.0 * math.pi / m)
    T, P = np.repeat(th, m), np.repeat(ph, m)
    S = np.tile(psi, len(th))
    q = np.stack([np.cos(T / 2) * np.cos(S / 2), np.cos(T / 2) * np.sin(S / 2),
                  np.sin(T / 2) * np.cos(P + S / 2), np.sin(T / 2) * np.sin(P + S / 2)], axis=1)
    return q


def uniform_quaternions(count: int, seed: int) -> np.ndarray:
    """Shoemake's uniform random unit quaternions, seeded, scalar first."""
    rng = np.random.default_rng(seed)
    u1, u2, u3 = rng.uniform(size=(3, count))
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    return np.stack([b * np.cos(2 * math.pi * u3), a * np.sin(2 * math.pi * u2),
                     a * np.cos(2 * math.pi * u2), b * np.sin(2 * math.pi * u3)], axis=1)


def quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product a * b for arrays (..., 4), scalar first."""
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def axis_angle_quaternions(axes: np.ndarray, angles: np.ndarray) -> np.ndarray:
    axes = axes / np.linalg.norm(axes, axis=-1, keepdims=True)
    h = np.asarray(angles)[..., None] / 2.0
    return np.concatenate([np.cos(h), np.sin(h) * axes], axis=-1)


def perturb_poses(t: np.ndarray, q: np.ndarray, sigma_t: float, sigma_deg: float, seed: int):
    """Perturb poses: t + N(0, sigma_t) per axis; q <- dq * q with dq a
    rotation about a uniform random axis by an angle ~ N(0, sigma_deg)."""
    rng = np.random.default_rng(seed)
    n = len(t)
    t2 = np.asarray(t, dtype=np.float64) + rng.normal(0.0, sigma_t, size=(n, 3))
    axes = rng.normal(size=(n, 3))
    ang = np.deg2rad(rng.normal(0.0, sigma_deg, size=n))
    q2 = quat_mul(axis_angle_quaternions(axes, ang), np.asarray(q, dtype=np.float64))
    q2 /= np.linalg.norm(q2, axis=1, keepdims=True)
    return t2, q2
