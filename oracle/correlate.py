"""ORACLE - TEST INFRASTRUCTURE ONLY.  Cross-correlation scores, FP64.

Eq. 8 scores a relative placement tau by f(tau) = int rho_1(p) rho_2(tau^-1 p) dv.
With the fixed part on the periodic grid and the rotated moving part spread
onto it (see spread.py), a pose (R, t) with t an integer grid shift gives

    f(R, t) = sum_p rho_F(p) M_R((p - t) mod N),      score s = Re f.

The Implementation section evaluates all translations of one rotation at
once with an FFT; that route must reach exactly this sum.  Two evaluations:
  * ``correlate_direct``: the sum above for every t (O(N^6), tiny grids);
  * ``correlate_fft``: numpy FFTs of rho_F and of the reflected M_R.
"""

from __future__ import annotations

import numpy as np

from . import rotation, spread


def moving_coefficients(rho_m, w_m) -> np.ndarray:
    """c_k = w_k rho_M(x_k), flat x-fastest order."""
    return (np.asarray(w_m, dtype=np.float64).ravel() * np.asarray(rho_m, dtype=np.complex128).ravel())


def rotated_spread(c, quat, n_m: int, shape, planar: bool = False) -> np.ndarray:
    """M_R on the fixed grid for rotation R(quat): samples at y_k = R x_k / h."""
    r = rotation.quat_to_matrix(quat)
    pos = spread.body_positions(n_m, planar) @ r.T
    return spread.spread(c, pos, shape)


def correlate_direct(rho_f, m) -> np.ndarray:
    """f(t) = sum_p rho_F(p) M((p - t) mod N) for every shift t (brute force)."""
    rho_f = np.asarray(rho_f, dtype=np.complex128)
    m = np.asarray(m, dtype=np.complex128)
    nz, ny, nx = rho_f.shape
    out = np.empty(rho_f.shape, dtype=np.complex128)
    for tz in range(nz):
        for ty in range(ny):
            for tx in range(nx):
                # np.roll(m, s)[p] = m[p - s]
                out[tz, ty, tx] = np.sum(rho_f * np.roll(m, (tz, ty, tx), axis=(0, 1, 2)))
    return out


def correlate_fft(rho_f, m) -> np.ndarray:
    """Same sum: with Mr(u) = M(-u), f = rho_F (*) Mr (circular convolution),
    so fft(f) = fft(rho_F) * fft(Mr)."""
    rho_f = np.asarray(rho_f, dtype=np.complex128)
    m = np.asarray(m, dtype=np.complex128)
    mr = np.roll(np.flip(m, axis=(0, 1, 2)), 1, axis=(0, 1, 2))  # mr[u] = m[-u mod N]
    return np.fft.ifftn(np.fft.fftn(rho_f) * np.fft.fftn(mr))


def score_volume(rho_f, c, quat, n_m: int, planar: bool = False, direct: bool = False) -> np.ndarray:
    """Re f(R, t) for all grid shifts t of one rotation."""
    m = rotated_spread(c, quat, n_m, rho_f.shape, planar)
    f = correlate_direct(rho_f, m) if direct else correlate_fft(rho_f, m)
    return f.real
