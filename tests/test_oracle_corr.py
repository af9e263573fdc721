"""Pins of the oracle's spreading, correlation, peak and gradient to brute
force, textbook identities and invariants (eq. 8 and the Implementation
section's FFT route)."""

import math

import numpy as np
import pytest

from oracle import correlate as oc
from oracle import grad as og
from oracle import peak as op
from oracle import rotation as orot
from oracle import spread as osp
from workloads import rotations as wr


def rand_complex(rng, shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


# --------------------------------------------------------------------------- rotation

def test_rotation_matrix_pins():
    qs = wr.uniform_quaternions(50, 1)
    r = orot.quat_to_matrix(qs * 1.7)  # unnormalised input is normalised
    assert np.allclose(r @ np.swapaxes(r, 1, 2), np.eye(3), atol=1e-14)
    assert np.allclose(np.linalg.det(r), 1.0, atol=1e-14)
    v = np.random.default_rng(0).normal(size=(4, 3))
    for q, m in zip(qs[:10], r[:10]):
        assert np.allclose(v @ m.T, orot.quat_rotate(q, v), atol=1e-13)
    # 90 degrees about +z maps x to y (right-handed)
    q = np.array([math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)])
    assert np.allclose(orot.quat_to_matrix(q) @ [1, 0, 0], [0, 1, 0], atol=1e-15)


def test_rotation_derivative_matches_fd():
    q = np.array([0.3, -0.5, 0.7, 0.2]) * 1.3
    d = orot.dmatrix_dquat(q)
    h = 1e-6
    for c in range(4):
        e = np.zeros(4)
        e[c] = h
        fd = (orot.quat_to_matrix(q + e) - orot.quat_to_matrix(q - e)) / (2 * h)
        assert np.allclose(d[:, :, c], fd, atol=1e-8)


def test_hopf_grid_is_a_uniform_cover():
    q = wr.hopf_grid(1)
    assert q.shape == (576, 4)
    r = orot.quat_to_matrix(q)
    # distinct rotations, and the mean rotation matrix vanishes (uniform set)
    g = np.abs(np.einsum("ik,jk->ij", q, q))
    np.fill_diagonal(g, 0)
    assert g.max() < 0.999
    assert np.abs(r.mean(axis=0)).max() < 0.05


# --------------------------------------------------------------------------- spread

def test_bspline_partition_of_unity_and_linear_reproduction():
    s = np.linspace(-0.5, 0.5, 11)
    k = np.arange(-3, 4)[:, None]
    assert np.allclose(osp.bspline3(k - s).sum(0), 1.0, atol=1e-15)
    assert np.allclose((k * osp.bspline3(k - s)).sum(0), s, atol=1e-15)
    assert np.allclose(osp.bspline3_deriv(k - s).sum(0), 0.0, atol=1e-15)
    # derivative is the slope of the piecewise cubic
    x = np.linspace(-2.2, 2.2, 97)
    h = 1e-6
    assert np.allclose(osp.bspline3_deriv(x), (osp.bspline3(x + h) - osp.bspline3(x - h)) / (2 * h), atol=1e-8)


def test_spread_matches_bruteforce_and_moments():
    rng = np.random.default_rng(2)
    shape = (6, 7, 8)
    pos = rng.uniform(-9, 14, size=(25, 3))
    c = rand_complex(rng, 25)
    m = osp.spread(c, pos, shape)
    assert np.allclose(m, osp.spread_bruteforce(c, pos, shape), atol=1e-12)
    assert abs(m.sum() - c.sum()) < 1e-12
    # first moment away from the wrap
    pos2 = rng.uniform(3, 9, size=(10, 3))
    big = (16, 16, 16)
    m2 = osp.spread(c[:10], pos2, big)
    k, j, i = np.meshgrid(np.arange(16), np.arange(16), np.arange(16), indexing="ij")
    mom = np.array([(i * m2).sum(), (j * m2).sum(), (k * m2).sum()])
    assert np.allclose(mom, (c[:10, None] * pos2).sum(0), atol=1e-11)


def test_spread_at_integer_positions_is_a_blur():
    # at integer positions the window is [1/6, 2/3, 1/6] per axis
    rng = np.random.default_rng(4)
    shape = (8, 8, 8)
    vals = rand_complex(rng, shape)
    k, j, i = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    pos = np.stack([i.ravel(), j.ravel(), k.ravel()], 1).astype(float)
    m = osp.spread(vals.ravel(), pos, shape)
    blur = vals.copy()
    for ax in range(3):
        blur = 2 / 3 * blur + 1 / 6 * (np.roll(blur, 1, ax) + np.roll(blur, -1, ax))
    assert np.allclose(m, blur, atol=1e-13)


# --------------------------------------------------------------------------- correlation

@pytest.mark.parametrize("shape", [(5, 6, 7), (8, 8, 8), (1, 9, 10)])
def test_direct_equals_fft(shape):
    rng = np.random.default_rng(sum(shape))
    a = rand_complex(rng, shape)
    b = rand_complex(rng, shape)
    d = oc.correlate_direct(a, b)
    f = oc.correlate_fft(a, b)
    assert np.max(np.abs(d - f)) < 1e-11 * np.max(np.abs(d))


def test_parseval_and_shift_theorem_of_the_fft_route():
    rng = np.random.default_rng(8)
    a = rand_complex(rng, (8, 8, 8))
    big = np.fft.fftn(a)
    assert abs((np.abs(a) ** 2).sum() - (np.abs(big) ** 2).sum() / a.size) < 1e-9
    # impulse correlates to a shifted copy
    imp = np.zeros((8, 8, 8), complex)
    imp[0, 0, 0] = 1.0
    f = oc.correlate_fft(a, imp)   # f(t) = a(t)
    assert np.allclose(f, a, atol=1e-12)


def test_hermitian_self_correlation_peaks_at_zero():
    rng = np.random.default_rng(12)
    rho = rand_complex(rng, (8, 8, 8))
    h = oc.correlate_fft(np.conj(rho), rho)  # sum_p conj(rho(p)) rho(p - t)
    assert np.argmax(h.real) == 0
    assert np.all(np.abs(h) <= abs(h.flat[0]) * (1 + 1e-12))
    assert abs(h.flat[0] - (np.abs(rho) ** 2).sum()) < 1e-9


def test_integer_shift_of_fixed_part_shifts_peak():
    rng = np.random.default_rng(13)
    rho_f = rand_complex(rng, (8, 8, 8))
    c = rand_complex(rng, 4 ** 3)
    q = wr.uniform_quaternions(1, 3)[0]
    v0 = oc.score_volume(rho_f, c, q, 4)
    s = (2, 5, 3)  # (dz, dy, dx)
    v1 = oc.score_volume(np.roll(rho_f, s, axis=(0, 1, 2)), c, q, 4)
    assert np.allclose(v1, np.roll(v0, s, axis=(0, 1, 2)), atol=1e-12)
    _, _, t0 = op.peak(v0)
    _, _, t1 = op.peak(v1)
    assert t1 == ((t0[0] + 3) % 8, (t0[1] + 5) % 8, (t0[2] + 2) % 8)


def test_grid_quarter_turn_invariance():
    # rho_F'(p) = rho_F(Q^-1 p) and rotation QR give f'(QR, Q t) = f(R, t)
    rng = np.random.default_rng(14)
    n = 8
    rho_f = rand_complex(rng, (n, n, n))
    c = rand_complex(rng, 4 ** 3)
    qr = wr.uniform_quaternions(1, 5)[0]
    qz = np.array([math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)])  # (x, y) -> (-y, x)
    rho_q = np.empty_like(rho_f)
    for z in range(n):
        for y in range(n):
            for x in range(n):
                rho_q[z, x % n, (-y) % n] = rho_f[z, y, x]
    v = oc.score_volume(rho_f, c, qr, 4)
    vq = oc.score_volume(rho_q, c, wr.quat_mul(qz, qr), 4)
    for z in range(n):
        for y in range(n):
            for x in range(n):
                assert abs(vq[z, x % n, (-y) % n] - v[z, y, x]) < 1e-12


# --------------------------------------------------------------------------- peak

def test_peak_tie_rule_and_neighbourhood():
    v = np.zeros((4, 5, 6))
    v[1, 2, 3] = 5.0
    v[3, 0, 0] = 5.0
    s, flat, t = op.peak(v)
    assert s == 5.0 and t == (3, 2, 1) and flat == (1 * 5 + 2) * 6 + 3
    nb = op.neighbourhood(v, (0, 0, 3))  # wraps in every axis
    assert nb[13] == 5.0 and nb.sum() == 5.0


def test_subvoxel_recovers_parabola_vertex():
    rng = np.random.default_rng(6)
    for _ in range(20):
        d = rng.uniform(-0.5, 0.5, 3)
        a = -rng.uniform(0.5, 2.0, 3)
        t = np.array([3, 4, 5])
        nb = np.empty((3, 3, 3))
        for iz, dz in enumerate((-1, 0, 1)):
            for iy, dy in enumerate((-1, 0, 1)):
                for ix, dx in enumerate((-1, 0, 1)):
                    off = np.array([dx, dy, dz])
                    nb[iz, iy, ix] = 7.0 + (a * (off - d) ** 2).sum()
        assert np.allclose(op.subvoxel(nb.ravel(), t), t + d, atol=1e-12)
    flat = np.ones(27)
    assert np.allclose(op.subvoxel(flat, (1, 2, 3)), (1, 2, 3))


def test_top_k_order():
    s = np.array([1.0, 3.0, 2.0, 3.0, -1.0])
    assert list(op.top_k(s, 3)) == [1, 3, 2]


# --------------------------------------------------------------------------- gradient

def small_pose_problem(seed=21, n=10, n_m=4):
    rng = np.random.default_rng(seed)
    rho_f = rand_complex(rng, (n, n, n))
    rho_m = rand_complex(rng, n_m ** 3)
    w = rng.uniform(0.5, 1.5, n_m ** 3)
    return rho_f, rho_m, w, osp.body_positions(n_m)


def test_pose_value_at_integer_shift_equals_correlation():
    rho_f, rho_m, w, xb = small_pose_problem()
    c = oc.moving_coefficients(rho_m, w)
    for q in wr.uniform_quaternions(3, 9):
        vol = oc.score_volume(rho_f, c, q, 4)
        for t in [(0, 0, 0), (3, 7, 1), (9, 2, 5)]:
            f = og.pose_value(rho_f, c, xb, t, q)
            assert abs(f - vol[t[2], t[1], t[0]]) < 1e-10 * max(1, abs(f))


def test_pose_gradient_matches_central_differences():
    rho_f, rho_m, w, xb = small_pose_problem()
    c = oc.moving_coefficients(rho_m, w)
    t = np.array([3.3, 4.6, 5.1])
    q = np.array([0.8, 0.1, -0.3, 0.4])
    f, dt, dq, dw = og.pose_value_and_grad(rho_f, c, rho_m, xb, t, q)
    x = np.concatenate([t, q])
    fd = og.fd_gradient(lambda v: og.pose_value(rho_f, c, xb, v[:3], v[3:]), x, 1e-4)
    g = np.concatenate([dt, dq])
    assert np.max(np.abs(fd - g)) < 1e-6 * max(1.0, np.max(np.abs(g)))
    # f is linear in the per-sample weights: an exact difference
    k = 17
    w2 = w.copy()
    w2[k] += 1.0
    f2 = og.pose_value(rho_f, oc.moving_coefficients(rho_m, w2), xb, t, q)
    assert abs((f2 - f) - dw[k]) < 1e-10 * max(1, abs(f))
    # the quaternion gradient is orthogonal to q (scale invariance of R(q/|q|))
    assert abs(np.dot(dq, q)) < 1e-10 * max(1, np.abs(dq).max())
