"""ORACLE - TEST INFRASTRUCTURE ONLY.  Nonequispaced route of the search, FP64.

The Implementation section proposes replacing the uniform-grid FFT by a
nonequispaced FFT with oversampling factor alpha > 1 (Potts et al.) once
the moving affinity is sampled at m' nonequispaced points (octree.py).
Without a resampling window, the samples y_k = R x_k (grid units) meet the
fixed affinity through its trigonometric interpolant

    rho_F^trig(z) = N^-d sum_kappa rho_F^(kappa) exp(2 pi i kappa.z / N),
    kappa in [-N/2, N/2)^d,  rho_F^ = DFT(rho_F),

and the score of eq. 8 at an integer shift t is

    f(R, t) = sum_k c_k rho_F^trig(t + y_k)
            = N^-d sum_kappa rho_F^(kappa) Mhat(kappa) exp(2 pi i kappa.t / N),
    Mhat(kappa) = sum_k c_k exp(-2 pi i kappa.(-y_k) / N),

so one rotation needs the type-1 transform Mhat of the reflected samples and
one inverse FFT.  ``ndft_type1`` is that sum as written (the definition);
``nufft_type1`` is the fast algorithm the GPU runs: spread each sample with
the "exponential of semicircle" kernel
    phi(z) = exp(beta (sqrt(1 - z^2) - 1)),  |z| <= 1,  beta = 2.30 w
(Barnett, Magland and af Klinteberg, 2019) over w nodes of the grid
oversampled by alpha = 2, FFT it, keep the N^d central frequencies and
divide by the kernel's Fourier transform.  Its error against the definition
falls roughly as 10^(1 - w).
"""

from __future__ import annotations

import numpy as np
from scipy import integrate

from . import rotation

ALPHA = 2


def mode_index(n: int) -> np.ndarray:
    """kappa for FFT-order index j: j for j < N/2, j - N otherwise."""
    j = np.arange(n)
    return np.where(j < n // 2, j, j - n)


def ndft_type1(pos, c, n: int, planar: bool = False) -> np.ndarray:
    """Mhat[kz, ky, kx] = sum_k c_k exp(-2 pi i kappa.pos_k / N), FFT order.

    pos (m, 3) in grid units (any real value); planar grids drop z."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    c = np.asarray(c, dtype=np.complex128).ravel()
    kap = mode_index(n).astype(np.float64)
    ex = np.exp(-2j * np.pi * np.outer(pos[:, 0], kap) / n)  # (m, N)
    ey = np.exp(-2j * np.pi * np.outer(pos[:, 1], kap) / n)
    if planar:
        return ((ey * c[:, None]).T @ ex)[None, :, :]
    ez = np.exp(-2j * np.pi * np.outer(pos[:, 2], kap) / n)
    m = pos.shape[0]
    out = np.zeros((n, n, n), dtype=np.complex128)
    for s in range(0, m, 2048):  # chunked (m, N, N) tensor of x-y factors
        sl = slice(s, s + 2048)
        xy = (ey[sl, :, None] * ex[sl, None, :]).reshape(ey[sl].shape[0], n * n)
        out += ((ez[sl] * c[sl, None]).T @ xy).reshape(n, n, n)
    return out


def es_beta(w: int) -> float:
    return 2.30 * w


def es_kernel(z, w: int) -> np.ndarray:
    z = np.asarray(z, dtype=np.float64)
    inside = np.abs(z) <= 1.0
    return np.where(inside, np.exp(es_beta(w) * (np.sqrt(np.clip(1.0 - z * z, 0.0, None)) - 1.0)), 0.0)


def es_transform(kappa, w: int, n_fine: int) -> np.ndarray:
    """phihat(kappa) = int phi(2x/w) exp(-2 pi i kappa x / n_fine) dx over
    |x| <= w/2 (x in fine-grid cells); real since phi is even."""
    out = []
    for k in np.atleast_1d(kappa):
        f = lambda x, k=k: float(es_kernel(2.0 * x / w, w)) * np.cos(2.0 * np.pi * k * x / n_fine)
        v, _ = integrate.quad(f, -w / 2.0, w / 2.0, limit=200, epsabs=1e-13, epsrel=1e-12)
        out.append(v)
    return np.array(out)


def nufft_type1(pos, c, n: int, w: int, planar: bool = False) -> np.ndarray:
    """Mhat by spreading on the (2N)^d grid, FFT, crop and deconvolution."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    c = np.asarray(c, dtype=np.complex128).ravel()
    nf = ALPHA * n
    v = np.mod(ALPHA * pos, nf)  # fine-grid units on the torus
    axes = (0, 1) if planar else (0, 1, 2)
    l0 = {a: np.ceil(v[:, a] - w / 2.0).astype(np.int64) for a in axes}
    wt = {a: [es_kernel(2.0 * (l0[a] + j - v[:, a]) / w, w) for j in range(w)] for a in axes}
    fine = np.zeros((1 if planar else nf, nf, nf), dtype=np.complex128)
    for jz in range(1 if planar else w):
        iz = np.zeros_like(l0[0]) if planar else np.mod(l0[2] + jz, nf)
        wz = 1.0 if planar else wt[2][jz]
        for jy in range(w):
            iy = np.mod(l0[1] + jy, nf)
            for jx in range(w):
                ix = np.mod(l0[0] + jx, nf)
                np.add.at(fine, (iz, iy, ix), c * wz * wt[1][jy] * wt[0][jx])
    big = np.fft.fftn(fine, axes=(1, 2) if planar else (0, 1, 2))
    kap = mode_index(n)
    fine_idx = np.mod(kap, nf)
    inv = 1.0 / es_transform(kap, w, nf)
    if planar:
        crop = big[0][np.ix_(fine_idx, fine_idx)]
        return (crop * inv[:, None] * inv[None, :])[None, :, :]
    crop = big[np.ix_(fine_idx, fine_idx, fine_idx)]
    return crop * inv[:, None, None] * inv[None, :, None] * inv[None, None, :]


def rotated_reflected(pos, quat) -> np.ndarray:
    """-R pos: the reflected rotated samples whose transform the correlation needs."""
    r = rotation.quat_to_matrix(quat)
    return -(np.asarray(pos, dtype=np.float64).reshape(-1, 3) @ r.T)


def score_volume_trig(rho_f, pos, c, quat, planar: bool = False, w: int | None = None) -> np.ndarray:
    """Re f(R, t) for every shift t: sum_k c_k rho_F^trig(t + R pos_k).

    w None: the exact type-1 sum; w given: the spread/FFT/deconvolution
    algorithm with kernel width w."""
    rho_f = np.asarray(rho_f, dtype=np.complex128)
    n = rho_f.shape[-1]
    y = rotated_reflected(pos, quat)
    mhat = ndft_type1(y, c, n, planar) if w is None else nufft_type1(y, c, n, w, planar)
    axes = (1, 2) if planar else (0, 1, 2)
    return np.fft.ifftn(np.fft.fftn(rho_f, axes=axes) * mhat, axes=axes).real


def trig_interpolant(rho_f, z, planar: bool = False) -> np.ndarray:
    """rho_F^trig at points z (m, 3) in grid units, by its defining sum."""
    rho_f = np.asarray(rho_f, dtype=np.complex128)
    n = rho_f.shape[-1]
    axes = (1, 2) if planar else (0, 1, 2)
    spec = np.fft.fftn(rho_f, axes=axes)
    kap = mode_index(n).astype(np.float64)
    z = np.asarray(z, dtype=np.float64).reshape(-1, 3)
    out = np.empty(z.shape[0], dtype=np.complex128)
    for i, p in enumerate(z):
        ex = np.exp(2j * np.pi * kap * p[0] / n)
        ey = np.exp(2j * np.pi * kap * p[1] / n)
        if planar:
            out[i] = np.einsum("yx,y,x->", spec[0], ey, ex)
        else:
            ez = np.exp(2j * np.pi * kap * p[2] / n)
            out[i] = np.einsum("zyx,z,y,x->", spec, ez, ey, ex)
    return out / spec.size
