"""ORACLE - TEST INFRASTRUCTURE ONLY.  Pose value and gradients, FP64.

For a continuous pose (t in grid units, q a quaternion, R = R(q/|q|)) the
score of eq. 8 with the spread window of spread.py is

    f(t, q) = Re sum_k c_k Phi(y_k),   y_k = R x_k / h + t,
    Phi(y)  = sum_p rho_F(p) B3(p - y)            (periodic grid),

which equals the FFT correlation exactly when t is an integer shift.  The
paper refines poses with gradient-based search (validation section);
gradients here follow by the chain rule:

    df/dt   = Re sum_k c_k grad Phi(y_k)
    df/dq   = sum_ab G_ab dR_ab/dq,   G = sum_k Re(c_k grad Phi(y_k)) (x_k/h)^T
    df/dw_k = Re(rho_M(x_k) Phi(y_k))

and ``fd_gradient`` gives central differences of the FP64 value.
"""

from __future__ import annotations

import numpy as np

from . import rotation, spread


def phi_and_grad(rho_f, y, want_grad: bool = True):
    """Phi(y) and its gradient (d/dy_x, d/dy_y, d/dy_z) for points y (K, 3)."""
    rho_f = np.asarray(rho_f, dtype=np.complex128)
    nz, ny, nx = rho_f.shape
    y = np.asarray(y, dtype=np.float64).reshape(-1, 3)
    base = np.floor(y).astype(np.int64) - 1
    val = np.zeros(len(y), dtype=np.complex128)
    grad = np.zeros((len(y), 3), dtype=np.complex128) if want_grad else None
    bx = [spread.bspline3(base[:, 0] + a - y[:, 0]) for a in range(4)]
    by = [spread.bspline3(base[:, 1] + a - y[:, 1]) for a in range(4)]
    bz = [spread.bspline3(base[:, 2] + a - y[:, 2]) for a in range(4)]
    # d/dy of B(p - y) = -B'(p - y)
    dx = [-spread.bspline3_deriv(base[:, 0] + a - y[:, 0]) for a in range(4)]
    dy = [-spread.bspline3_deriv(base[:, 1] + a - y[:, 1]) for a in range(4)]
    dz = [-spread.bspline3_deriv(base[:, 2] + a - y[:, 2]) for a in range(4)]
    for cz in range(4):
        iz = np.mod(base[:, 2] + cz, nz)
        for cy in range(4):
            iy = np.mod(base[:, 1] + cy, ny)
            for cx in range(4):
                ix = np.mod(base[:, 0] + cx, nx)
                r = rho_f[iz, iy, ix]
                val += r * (bx[cx] * by[cy] * bz[cz])
                if want_grad:
                    grad[:, 0] += r * (dx[cx] * by[cy] * bz[cz])
                    grad[:, 1] += r * (bx[cx] * dy[cy] * bz[cz])
                    grad[:, 2] += r * (bx[cx] * by[cy] * dz[cz])
    return val, grad


def pose_value(rho_f, c, xb, t, q) -> float:
    """f(t, q) with body positions xb = x_k / h (K, 3)."""
    r = rotation.quat_to_matrix(q)
    y = xb @ r.T + np.asarray(t, dtype=np.float64)
    val, _ = phi_and_grad(rho_f, y, want_grad=False)
    return float(np.sum(np.asarray(c).ravel() * val).real)


def pose_value_and_grad(rho_f, c, rho_m, xb, t, q):
    """-> (f, df/dt (3,), df/dq (4,), df/dw (K,))."""
    c = np.asarray(c, dtype=np.complex128).ravel()
    r = rotation.quat_to_matrix(q)
    y = xb @ r.T + np.asarray(t, dtype=np.float64)
    val, grad = phi_and_grad(rho_f, y)
    f = float(np.sum(c * val).real)
    cg = (c[:, None] * grad).real  # (K, 3): Re(c_k dPhi/dy_a)
    dfdt = cg.sum(axis=0)
    g = cg.T @ xb  # G_ab = sum_k Re(c_k d_a Phi) xb_kb
    dfdq = np.einsum("ab,abc->c", g, rotation.dmatrix_dquat(q))
    dfdw = (np.asarray(rho_m, dtype=np.complex128).ravel() * val).real
    return f, dfdt, dfdq, dfdw


def fd_gradient(fun, x, h: float = 1e-3) -> np.ndarray:
    """Central differences of a scalar function of a vector."""
    x = np.asarray(x, dtype=np.float64)
    g = np.empty_like(x)
    for i in range(len(x)):
        e = np.zeros_like(x)
        e[i] = h
        g[i] = (fun(x + e) - fun(x - e)) / (2.0 * h)
    return g


def fixed_cotangent(c, xb, poses, grad_scale, shape) -> np.ndarray:
    """Cotangent of sum_b s_b f_b with respect to rho_F: f_b is linear in
    rho_F, f_b = Re sum_p rho_F(p) sum_k c_k B3(p - y_kb), so the cotangent is
    the periodic spread sum_b s_b sum_k c_k B3(p - y_kb), y_kb = R_b x_k + t_b."""
    out = np.zeros(shape, dtype=np.complex128)
    c = np.asarray(c, dtype=np.complex128).ravel()
    for b, pose in enumerate(np.asarray(poses, dtype=np.float64).reshape(-1, 7)):
        r = rotation.quat_to_matrix(pose[3:])
        y = xb @ r.T + pose[:3]
        out += grad_scale[b] * spread.spread(c, y, shape)
    return out
