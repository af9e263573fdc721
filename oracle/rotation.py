"""ORACLE - TEST INFRASTRUCTURE ONLY.  Rotations from quaternions, FP64.

The search samples rotations tau_r in a finite set T_r (Implementation
section); rotations are given as quaternions q (scalar first, Hamilton
convention) and used as R(q / |q|).
"""

from __future__ import annotations

import numpy as np


def quat_to_matrix(q) -> np.ndarray:
    """R(q / |q|) for q of shape (..., 4) -> (..., 3, 3)."""
    q = np.asarray(q, dtype=np.float64)
    u = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = np.moveaxis(u, -1, 0)
    r = np.empty(q.shape[:-1] + (3, 3))
    r[..., 0, 0] = 1 - 2 * (y * y + z * z)
    r[..., 0, 1] = 2 * (x * y - w * z)
    r[..., 0, 2] = 2 * (x * z + w * y)
    r[..., 1, 0] = 2 * (x * y + w * z)
    r[..., 1, 1] = 1 - 2 * (x * x + z * z)
    r[..., 1, 2] = 2 * (y * z - w * x)
    r[..., 2, 0] = 2 * (x * z - w * y)
    r[..., 2, 1] = 2 * (y * z + w * x)
    r[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def quat_rotate(q, v) -> np.ndarray:
    """Rotate vectors v (..., 3) by the sandwich product u v u* (independent
    of the matrix formula; used to pin it)."""
    q = np.asarray(q, dtype=np.float64)
    u = q / np.linalg.norm(q)
    v = np.asarray(v, dtype=np.float64)

    def mul(a, b):
        return np.array([a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3],
                         a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2],
                         a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1],
                         a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0]])

    conj = u * np.array([1.0, -1.0, -1.0, -1.0])
    out = []
    for vv in v.reshape(-1, 3):
        r = mul(mul(u, np.concatenate([[0.0], vv])), conj)
        out.append(r[1:])
    return np.array(out).reshape(v.shape)


def dmatrix_dquat(q) -> np.ndarray:
    """d R(q/|q|)_{ab} / d q_c for one quaternion -> (3, 3, 4).

    Chain rule: dR/dq = dR/du (I - u u^T) / |q| with u = q / |q|, where
    dR/du is the derivative of the polynomial entries above.
    """
    q = np.asarray(q, dtype=np.float64)
    nq = np.linalg.norm(q)
    u = q / nq
    w, x, y, z = u
    d = np.zeros((3, 3, 4))  # dR_ab / du_c, c = (w, x, y, z)
    d[0, 0] = [0, 0, -4 * y, -4 * z]
    d[0, 1] = [-2 * z, 2 * y, 2 * x, -2 * w]
    d[0, 2] = [2 * y, 2 * z, 2 * w, 2 * x]
    d[1, 0] = [2 * z, 2 * y, 2 * x, 2 * w]
    d[1, 1] = [0, -4 * x, 0, -4 * z]
    d[1, 2] = [-2 * x, -2 * w, 2 * z, 2 * y]
    d[2, 0] = [-2 * y, 2 * z, -2 * w, 2 * x]
    d[2, 1] = [2 * x, 2 * w, 2 * z, 2 * y]
    d[2, 2] = [0, -4 * x, -4 * y, 0]
    proj = (np.eye(4) - np.outer(u, u)) / nq
    return d @ proj
