"""Pins of the oracle's nonequispaced route (oracle/nfft.py) and of the
octree-adaptive samples (oracle/octree.py) against definitions, closed forms
and library routines (Implementation section: octree sampling and NFFT)."""

import numpy as np
import pytest

from oracle import nfft, octree, rotation

RNG = np.random.default_rng(1712)


def _quat(rng):
    q = rng.normal(size=4)
    return q / np.linalg.norm(q)


def _pos(rng, m, span, planar):
    p = rng.uniform(-span, span, (m, 3))
    if planar:
        p[:, 2] = 0.0
    return p


@pytest.mark.parametrize("planar", [False, True])
def test_ndft_at_integer_positions_is_the_fft_of_a_delta_grid(planar):
    n = 16
    rng = np.random.default_rng(3)
    pos = rng.integers(-40, 40, (200, 3)).astype(np.float64)
    if planar:
        pos[:, 2] = 0
    c = rng.normal(size=200) + 1j * rng.normal(size=200)
    grid = np.zeros((1 if planar else n, n, n), dtype=np.complex128)
    idx = np.mod(pos.astype(np.int64), n)
    np.add.at(grid, (idx[:, 2], idx[:, 1], idx[:, 0]), c)
    ref = np.fft.fftn(grid, axes=(1, 2) if planar else (0, 1, 2))
    got = nfft.ndft_type1(pos, c, n, planar)
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("planar", [False, True])
def test_nufft_error_against_the_definition_follows_the_kernel_width(planar):
    # The ES kernel at oversampling 2 reaches about 10^(1 - w) relative error
    # (Barnett, Magland and af Klinteberg, 2019); a wrong deconvolution, crop
    # index or periodisation gives O(1) errors.
    n = 16
    rng = np.random.default_rng(5)
    pos = _pos(rng, 300, 25.0, planar)
    c = rng.normal(size=300) + 1j * rng.normal(size=300)
    ex = nfft.ndft_type1(pos, c, n, planar)
    errs = []
    for w in (4, 6, 8):
        ap = nfft.nufft_type1(pos, c, n, w, planar)
        errs.append(np.max(np.abs(ap - ex)) / np.max(np.abs(ex)))
    for w, e in zip((4, 6, 8), errs):
        assert e < 5.0 * 10.0 ** (1 - w), (w, e)
    assert errs[0] > errs[1] > errs[2]


@pytest.mark.parametrize("planar", [False, True])
def test_trig_score_of_one_fourier_mode_is_closed_form(planar):
    # rho_F(p) = exp(2 pi i kappa0.p / N) with kappa0 inside the band is its
    # own trigonometric interpolant, so f(R, t) = sum_k c_k exp(2 pi i kappa0.(t + R x_k) / N).
    n = 16
    rng = np.random.default_rng(7)
    k0 = np.array([3, -5, 0 if planar else 2])
    if planar:
        j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        rho = np.exp(2j * np.pi * (k0[0] * i + k0[1] * j) / n)[None]
    else:
        k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        rho = np.exp(2j * np.pi * (k0[0] * i + k0[1] * j + k0[2] * k) / n)
    pos = _pos(rng, 150, 6.0, planar)
    c = rng.normal(size=150) + 1j * rng.normal(size=150)
    q = _quat(rng)
    if planar:
        q = np.array([np.cos(0.4), 0.0, 0.0, np.sin(0.4)])
    y = pos @ rotation.quat_to_matrix(q).T
    phase = np.sum(c * np.exp(2j * np.pi * (y @ k0) / n))
    shape = rho.shape
    tz, ty, tx = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    ref = (phase * np.exp(2j * np.pi * (k0[0] * tx + k0[1] * ty + k0[2] * tz) / n)).real
    got = nfft.score_volume_trig(rho, pos, c, q, planar)
    assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))
    got6 = nfft.score_volume_trig(rho, pos, c, q, planar, w=6)
    assert np.max(np.abs(got6 - ref)) < 1e-4 * np.max(np.abs(ref))


def test_trig_score_interpolates_at_integer_samples():
    # Identity rotation, integer sample positions: the interpolant takes the
    # grid values, f(t) = sum_k c_k rho_F((t + x_k) mod N).
    n = 8
    rng = np.random.default_rng(11)
    rho = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    pos = rng.integers(-3, 4, (40, 3)).astype(np.float64)
    c = rng.normal(size=40) + 1j * rng.normal(size=40)
    got = nfft.score_volume_trig(rho, pos, c, np.array([1.0, 0, 0, 0]))
    ref = np.zeros((n, n, n))
    for tz in range(n):
        for ty in range(n):
            for tx in range(n):
                idx = np.mod(pos.astype(np.int64) + [tx, ty, tz], n)
                ref[tz, ty, tx] = np.sum(c * rho[idx[:, 2], idx[:, 1], idx[:, 0]]).real
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))


def test_trig_score_equals_the_interpolant_at_moved_samples():
    # A generic field and rotation: the spectral route equals the defining sum
    # of the interpolant at t + R x_k, itself pinned at grid points.
    n = 8
    rng = np.random.default_rng(13)
    rho = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    ipts = rng.integers(0, n, (5, 3)).astype(np.float64)
    assert np.allclose(nfft.trig_interpolant(rho, ipts), rho[ipts[:, 2].astype(int), ipts[:, 1].astype(int),
                                                              ipts[:, 0].astype(int)], atol=1e-12)
    pos = _pos(rng, 30, 3.0, False)
    c = rng.normal(size=30) + 1j * rng.normal(size=30)
    q = _quat(rng)
    vol = nfft.score_volume_trig(rho, pos, c, q)
    y = pos @ rotation.quat_to_matrix(q).T
    for t in ([0, 0, 0], [3, 1, 7], [5, 6, 2]):
        ref = np.sum(c * nfft.trig_interpolant(rho, y + np.array(t, dtype=np.float64))).real
        assert abs(vol[t[2], t[1], t[0]] - ref) < 1e-10 * np.max(np.abs(vol))


def _random_field(rng, n_m, planar, smooth=True, damping=60.0):
    shape = (1 if planar else n_m, n_m, n_m)
    f = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    if smooth:
        spec = np.fft.fftn(f, axes=(1, 2) if planar else (0, 1, 2))
        k = np.fft.fftfreq(n_m)
        damp = np.exp(-(k[None, None, :] ** 2 + k[None, :, None] ** 2 + (0 if planar else k[:, None, None] ** 2)) * damping)
        f = np.fft.ifftn(spec * damp, axes=(1, 2) if planar else (0, 1, 2))
    return f


def _nodes(n_m, planar):
    if planar:
        j, i = np.meshgrid(np.arange(n_m), np.arange(n_m), indexing="ij")
        return np.stack([i.ravel(), j.ravel(), np.zeros(i.size, dtype=np.int64)], 1)
    k, j, i = np.meshgrid(np.arange(n_m), np.arange(n_m), np.arange(n_m), indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], 1)


@pytest.mark.parametrize("planar", [False, True])
def test_octree_with_zero_tolerance_keeps_every_nonzero_node(planar):
    n_m = 16
    rng = np.random.default_rng(17)
    f = _random_field(rng, n_m, planar, smooth=False)
    f.ravel()[rng.choice(f.size, f.size // 5, replace=False)] = 0
    pos, coef, lev, corner = octree.octree_leaves(f, n_m, 0.0, 3, planar)
    nodes = _nodes(n_m, planar)
    keep = f.ravel() != 0
    assert np.all(lev == 0)
    assert len(coef) == int(np.sum(keep))
    got = {tuple(cr): cf for cr, cf in zip(corner, coef)}
    for nd, v in zip(nodes[keep], f.ravel()[keep]):
        assert got[tuple(nd)] == v
    ref_pos = corner - n_m / 2.0
    if planar:
        ref_pos[:, 2] = 0
    assert np.array_equal(pos, ref_pos)


@pytest.mark.parametrize("planar", [False, True])
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_octree_of_a_constant_field_is_one_leaf_per_top_cell(planar, levels):
    n_m = 16
    f = np.full((1 if planar else n_m, n_m, n_m), 0.5 - 0.25j)
    pos, coef, lev, corner = octree.octree_leaves(f, n_m, 1e-3, levels, planar)
    s = 1 << levels
    per = s * s * (1 if planar else s)
    assert np.all(lev == levels)
    assert len(coef) == f.size // per
    assert np.allclose(coef, per * (0.5 - 0.25j), rtol=0, atol=1e-14)
    assert np.all(np.mod(corner[:, :2], s) == 0)
    assert np.allclose(pos[:, 0], corner[:, 0] + (s - 1) / 2.0 - n_m / 2.0)


@pytest.mark.parametrize("planar", [False, True])
def test_octree_of_a_ramp_stops_at_the_level_its_slope_allows(planar):
    # Re c = i (node index along x): a cell of 2^l nodes spans 2^l - 1, so
    # with tau = tol * (N_M - 1) every leaf sits at the highest level l with
    # 2^l - 1 < tau, and the nodes at i = 0 only vanish at level 0.
    n_m = 16
    i = np.arange(n_m, dtype=np.float64)
    f = np.broadcast_to(i, (1 if planar else n_m, n_m, n_m)).astype(np.complex128)
    for tau, want in ((0.5, 0), (1.5, 1), (3.5, 2), (7.5, 3), (100.0, 3)):
        pos, coef, lev, corner = octree.octree_leaves(f, n_m, tau / (n_m - 1), 3, planar)
        assert np.all(lev == want), (tau, np.unique(lev))
        s = 1 << want
        per = s * s * (1 if planar else s)
        n_zero_cells = 0 if want else f.size // n_m
        assert len(coef) == f.size // per - n_zero_cells
        assert np.isclose(np.sum(coef), np.sum(f))


@pytest.mark.parametrize("planar", [False, True])
def test_octree_leaves_tile_the_box_flat_and_maximal(planar):
    n_m = 16
    rng = np.random.default_rng(19)
    f = _random_field(rng, n_m, planar)
    f[..., :3] = 0  # a slab of exact zeros
    for tol, levels in ((0.02, 3), (0.1, 3), (0.1, 2), (0.3, 1)):
        pos, coef, lev, corner = octree.octree_leaves(f, n_m, tol, levels, planar)
        assert np.isclose(np.sum(coef), np.sum(f), rtol=1e-12)
        cover = np.zeros(f.shape, dtype=np.int64)
        re, im = f.real, f.imag
        tau = tol * max(np.abs(re).max(), np.abs(im).max())

        def spread_of(a, i0, j0, k0, s):
            blk = a[k0:k0 + (1 if planar else s), j0:j0 + s, i0:i0 + s]
            return blk.max() - blk.min()

        for (i0, j0, k0), l in zip(corner, lev):
            s = 1 << l
            cover[k0:k0 + (1 if planar else s), j0:j0 + s, i0:i0 + s] += 1
            if l > 0:
                assert spread_of(re, i0, j0, k0, s) < tau and spread_of(im, i0, j0, k0, s) < tau
            if l < levels:
                ps = s * 2
                pi, pj, pk = (i0 // ps) * ps, (j0 // ps) * ps, (0 if planar else (k0 // ps) * ps)
                assert not (spread_of(re, pi, pj, pk, ps) < tau and spread_of(im, pi, pj, pk, ps) < tau)
        assert cover.max() == 1
        assert np.all(f[cover == 0] == 0)
        # leaf order: blocks of 8 in flat order, Morton order inside
        blk = (corner[:, 2] // 8 * (n_m // 8) + corner[:, 1] // 8) * (n_m // 8) + corner[:, 0] // 8
        mort = np.zeros(len(corner), dtype=np.int64)
        for b in range(3):
            mort |= ((corner[:, 0] >> b) & 1) << (3 * b) | ((corner[:, 1] >> b) & 1) << (3 * b + 1) | \
                    ((corner[:, 2] >> b) & 1) << (3 * b + 2)
        key = blk * 512 + mort
        assert np.all(np.diff(key) > 0)


def test_octree_samples_approach_the_full_grid_score_as_the_tolerance_falls():
    # Merged leaves move a cell's mass to its centre; on smooth fields the
    # score error shrinks with the tolerance and vanishes at tol = 0.
    n, n_m = 16, 16
    rng = np.random.default_rng(23)
    rho = _random_field(rng, n, False)
    f = _random_field(rng, n_m, False, damping=400.0)
    q = _quat(rng)
    full_pos = _nodes(n_m, False) - n_m / 2.0
    ref = nfft.score_volume_trig(rho, full_pos, f.ravel(), q)
    errs = []
    for tol in (0.3, 0.1, 0.03, 0.0):
        pos, coef, _, _ = octree.octree_leaves(f, n_m, tol, 3)
        errs.append(np.max(np.abs(nfft.score_volume_trig(rho, pos, coef, q) - ref)) / np.max(np.abs(ref)))
    assert errs[-1] < 1e-12
    assert errs[0] > errs[1] > errs[2] > errs[-1]
