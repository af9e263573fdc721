"""GPU parity of the nonequispaced route (Implementation section: octree-
adaptive samples and a nonequispaced FFT) against oracle/octree.py and
oracle/nfft.py, through the C ABI.

  * octree_samples: leaf levels, positions and order bit-exact (both sides
    decide in the context's precision on the same coefficients), leaf sums
    within rounding of FP64 sums;
  * score_volume_nfft: whole volumes against the oracle's spread/FFT/
    deconvolution algorithm (FP64: 1e-9, FP32: 2e-5 of the largest score) and
    against the exact type-1 sum within the kernel's error bound;
  * score_rotations_nfft: peaks against the oracle volumes.
"""

import numpy as np
import pytest

from helpers import flush_print
from oracle import nfft as onf
from oracle import octree as ooc
from oracle import pipeline
from workloads import configs as C
from workloads import rotations as wr

pytestmark = pytest.mark.gpu

REAL = {"f32": np.float32, "f64": np.float64}
CPLX = {"f32": np.complex64, "f64": np.complex128}


@pytest.fixture(scope="module")
def ctxs():
    import torch  # noqa: F401
    from paper_1712_00238_amd.api import Context
    c32, c64 = Context(0, "f32"), Context(0, "f64")
    yield {"f32": c32, "f64": c64}
    c32.close()
    c64.close()


def to_np(t):
    return t.detach().cpu().numpy()


def smooth_field(rng, n, planar, damping=300.0):
    """Seeded smooth complex field (input generation only)."""
    shape = (1 if planar else n, n, n)
    f = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    axes = (1, 2) if planar else (0, 1, 2)
    k = np.fft.fftfreq(n)
    k2 = k[None, None, :] ** 2 + k[None, :, None] ** 2 + (0.0 if planar else k[:, None, None] ** 2)
    return np.fft.ifftn(np.fft.fftn(f, axes=axes) * np.exp(-k2 * damping), axes=axes)


def grid_spec(n, planar):
    return C.GridSpec((n, n, 1 if planar else n), (0.0, 0.0, 0.0), 1.0)


def coefficients(rho, w, dtype):
    """c = rho * w rounded as the context computes it."""
    return rho.astype(CPLX[dtype]) * w.astype(REAL[dtype])


def planar_quats(n, seed):
    th = np.random.default_rng(seed).uniform(0, 2 * np.pi, n)
    return np.stack([np.cos(th / 2), np.zeros(n), np.zeros(n), np.sin(th / 2)], 1)


# ----------------------------------------------------------------------------- octree

@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("planar,nm", [(False, 24), (True, 40)])
@pytest.mark.parametrize("tol,levels", [(0.0, 3), (0.02, 3), (0.08, 2), (0.3, 1), (0.05, 0), (1e9, 3)])
def test_octree_samples_match_oracle(ctxs, dtype, planar, nm, tol, levels):
    ctx = ctxs[dtype]
    rng = np.random.default_rng(nm + 7 * levels)
    rho = smooth_field(rng, nm, planar)
    rho[..., : nm // 4] = 0  # a slab of exact zeros (dropped leaves)
    w = rng.uniform(0.5, 1.5, rho.shape)
    flush_print("octree", dtype, planar, nm, tol, levels)
    pos, c, lev = ctx.octree_samples(rho.astype(CPLX[dtype]), w.astype(REAL[dtype]), grid_spec(nm, planar), tol,
                                     levels)
    cin = coefficients(rho, w, dtype)
    rpos, rc, rlev, _ = ooc.octree_leaves(cin, nm, tol, levels, planar, dtype=REAL[dtype])
    pos, c, lev = to_np(pos).astype(np.float64), to_np(c).astype(np.complex128), to_np(lev)
    assert len(lev) == len(rlev), (len(lev), len(rlev))
    assert np.array_equal(lev, rlev)
    assert np.array_equal(pos, rpos)
    scale = np.abs(rc).max()
    rt = 2e-7 if dtype == "f32" else 1e-14
    assert np.all(np.abs(c - rc) <= rt * np.abs(rc) + 1e-12 * scale)


def test_octree_samples_reject_bad_boxes(ctxs):
    from paper_1712_00238_amd._lib import SdfError
    ctx = ctxs["f32"]
    rho = np.zeros((12, 12, 12), dtype=np.complex64)
    w = np.ones((12, 12, 12), dtype=np.float32)
    with pytest.raises(SdfError):
        ctx.octree_samples(rho, w, grid_spec(12, False), 0.1, 3)
    rho = np.zeros((16, 16, 16), dtype=np.complex64)
    w = np.ones((16, 16, 16), dtype=np.float32)
    with pytest.raises(SdfError):
        ctx.octree_samples(rho, w, grid_spec(16, False), 0.1, 4)
    with pytest.raises(SdfError):
        ctx.octree_samples(rho, w, grid_spec(16, False), -1.0, 3)


# ----------------------------------------------------------------------------- type-1 route

def small_pair_fields():
    pair = C.small_3d(seed=3, n=16, n_m=8, n_rot=3)
    return pair, pipeline.build_fields(pair)


def check_volumes(gpu, fields_rho, pos, coef, quats, planar, dtype, w):
    alg_tol = 2e-5 if dtype == "f32" else 1e-9
    def_tol = 5.0 * 10.0 ** (1 - w) + (2e-5 if dtype == "f32" else 0.0)
    for r, q in enumerate(quats):
        alg = onf.score_volume_trig(fields_rho, pos, coef, q, planar, w=w)
        exact = onf.score_volume_trig(fields_rho, pos, coef, q, planar)
        scale = np.abs(exact).max()
        e_alg = np.abs(gpu[r] - alg).max() / scale
        e_def = np.abs(gpu[r] - exact).max() / scale
        flush_print("  rotation", r, "err vs algorithm", e_alg, "vs definition", e_def)
        assert e_alg <= alg_tol, (r, e_alg)
        assert e_def <= def_tol, (r, e_def)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_nfft_volume_matches_oracle_3d(ctxs, dtype):
    ctx = ctxs[dtype]
    pair, f = small_pair_fields()
    pos, coef, _, _ = ooc.octree_leaves(f.c, f.n_m, 0.02, 2)
    pos = pos.astype(REAL[dtype]).astype(np.float64)
    coef = coef.astype(CPLX[dtype]).astype(np.complex128)
    gf = pair.fixed.grid
    spec = ctx.spectrum(f.rho_f.astype(CPLX[dtype]), gf)
    quats = pair.quats[:3]
    flush_print("nfft 3d", dtype, "leaves", len(coef))
    vol = to_np(ctx.score_volume_nfft(spec, gf, pos.astype(REAL[dtype]), coef.astype(CPLX[dtype]), quats, width=6))
    check_volumes(vol.astype(np.float64), f.rho_f, pos, coef, quats, False, dtype, 6)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_nfft_volume_matches_oracle_planar(ctxs, dtype):
    ctx = ctxs[dtype]
    rng = np.random.default_rng(41)
    n, nm = 32, 16
    rho_f = smooth_field(rng, n, True, damping=30.0)
    rho_m = smooth_field(rng, nm, True, damping=200.0)
    c = rho_m.ravel()
    pos, coef, _, _ = ooc.octree_leaves(c, nm, 0.05, 3, planar=True)
    pos = pos.astype(REAL[dtype]).astype(np.float64)
    coef = coef.astype(CPLX[dtype]).astype(np.complex128)
    gf = grid_spec(n, True)
    spec = ctx.spectrum(rho_f.astype(CPLX[dtype]), gf)
    quats = planar_quats(3, 5)
    flush_print("nfft planar", dtype, "leaves", len(coef))
    vol = to_np(ctx.score_volume_nfft(spec, gf, pos.astype(REAL[dtype]), coef.astype(CPLX[dtype]), quats, width=6))
    check_volumes(vol.astype(np.float64), rho_f, pos, coef, quats, True, dtype, 6)


@pytest.mark.parametrize("w", [2, 3, 4, 5, 7, 8])
def test_nfft_every_kernel_width(ctxs, w):
    ctx = ctxs["f64"]
    rng = np.random.default_rng(100 + w)
    n = 16
    rho_f = smooth_field(rng, n, False, damping=20.0)
    pos = rng.uniform(-5, 5, (200, 3))
    coef = rng.normal(size=200) + 1j * rng.normal(size=200)
    gf = grid_spec(n, False)
    spec = ctx.spectrum(rho_f, gf)
    q = wr.uniform_quaternions(1, 9 + w)
    vol = to_np(ctx.score_volume_nfft(spec, gf, pos, coef, q, width=w))[0]
    alg = onf.score_volume_trig(rho_f, pos, coef, q[0], False, w=w)
    err = np.abs(vol - alg).max() / np.abs(alg).max()
    flush_print("width", w, "err vs algorithm", err)
    assert err <= 1e-9


@pytest.mark.parametrize("w", [2, 3, 4, 5, 6, 7, 8])
def test_nfft_every_kernel_width_fp32_line_tiles(ctxs, w):
    # FP32 3D grids spread in line tiles with the first FFT pass fused in
    ctx = ctxs["f32"]
    rng = np.random.default_rng(200 + w)
    n = 32
    rho_f = smooth_field(rng, n, False, damping=60.0).astype(np.complex64)
    pos = rng.uniform(-9, 9, (1500, 3)).astype(np.float32)
    coef = (rng.normal(size=1500) + 1j * rng.normal(size=1500)).astype(np.complex64)
    gf = grid_spec(n, False)
    spec = ctx.spectrum(rho_f, gf)
    q = wr.uniform_quaternions(2, 31 + w)
    vol = to_np(ctx.score_volume_nfft(spec, gf, pos, coef, q, width=w)).astype(np.float64)
    for r in range(2):
        alg = onf.score_volume_trig(rho_f.astype(np.complex128), pos.astype(np.float64), coef.astype(np.complex128),
                                    q[r], False, w=w)
        err = np.abs(vol[r] - alg).max() / np.abs(alg).max()
        flush_print("fp32 width", w, "rotation", r, "err vs algorithm", err)
        assert err <= 2e-5


@pytest.mark.parametrize("n", [32, 64, 96])
def test_nfft_fp32_line_tiles_crowded_tile(ctxs, n):
    # A tight cluster of 2 600 samples puts far more than the 4 x 512
    # candidates the fused line tile sorts into one tile's 2 x 3 bins, so the
    # tile also runs its unsorted loop; 900 samples spread over the box fill
    # the other tiles.  N = 64 runs the 128-point line transform and the
    # 128-point pruned y / z passes.
    ctx = ctxs["f32"]
    rng = np.random.default_rng(400 + n)
    rho_f = smooth_field(rng, n, False, damping=0.06 * n * n).astype(np.complex64)
    centre = rng.uniform(-0.2 * n, 0.2 * n, 3)
    pos = np.concatenate([centre + rng.normal(scale=0.7, size=(2600, 3)),
                          rng.uniform(-0.45 * n, 0.45 * n, (900, 3))]).astype(np.float32)
    coef = (rng.normal(size=len(pos)) + 1j * rng.normal(size=len(pos))).astype(np.complex64)
    gf = grid_spec(n, False)
    spec = ctx.spectrum(rho_f, gf)
    quats = wr.uniform_quaternions(2, 500 + n)
    # the crowded tile, counted on the host the way the bins are defined: the
    # fine-grid tile of the first window node, 8 (y) x 4 (z) rows per tile
    # (N = 96: 192-point lines, whose transform has a radix-3 pass)
    w, nf = 6, 2 * n
    from oracle import rotation
    for q in quats:
        v = np.mod(-2.0 * (pos.astype(np.float64) @ rotation.quat_to_matrix(q).T), nf)
        l0 = np.ceil(v - w / 2.0).astype(np.int64)
        by, bz = np.mod(l0[:, 1], nf) // 8, np.mod(l0[:, 2], nf) // 4
        bins = np.zeros((nf // 4, nf // 8), dtype=np.int64)
        np.add.at(bins, (bz, by), 1)
        most = max(sum(bins[(tz - dz) % (nf // 4), (ty - dy) % (nf // 8)] for dy in range(2) for dz in range(3))
                   for tz in range(nf // 4) for ty in range(nf // 8))
        assert most > 2048, most
    flush_print("crowded line tile n", n, "samples", len(pos))
    vol = to_np(ctx.score_volume_nfft(spec, gf, pos, coef, quats, width=w)).astype(np.float64)
    check_volumes(vol, rho_f.astype(np.complex128), pos.astype(np.float64), coef.astype(np.complex128), quats,
                  False, "f32", w)


@pytest.mark.parametrize("dtype,planar,n", [("f32", False, 8), ("f64", False, 8), ("f64", False, 32),
                                             ("f32", True, 64), ("f64", True, 64), ("f32", True, 16),
                                             ("f32", False, 96), ("f64", False, 96), ("f32", True, 96),
                                             ("f64", True, 96)])
def test_nfft_grid_sizes_and_tilings(ctxs, dtype, planar, n):
    # every spreading path: FP32 line tiles without the fused x pass (N = 8),
    # general tiles split along every axis (FP64 3D N = 32, planar N = 64);
    # N = 96 runs 192-point lines (not a power of two: wrapped offsets, a
    # radix-3 pass) through the fused line tiles, the general tiles in 3D and
    # in the plane, and the pruned passes
    ctx = ctxs[dtype]
    rng = np.random.default_rng(300 + n + planar)
    rho_f = smooth_field(rng, n, planar, damping=0.3 * n * n / 16)
    m = 700
    pos = rng.uniform(-0.6 * n, 0.6 * n, (m, 3))
    if planar:
        pos[:, 2] = 0
    coef = rng.normal(size=m) + 1j * rng.normal(size=m)
    pos = pos.astype(REAL[dtype]).astype(np.float64)
    coef = coef.astype(CPLX[dtype]).astype(np.complex128)
    gf = grid_spec(n, planar)
    spec = ctx.spectrum(rho_f.astype(CPLX[dtype]), gf)
    quats = planar_quats(2, n) if planar else wr.uniform_quaternions(2, n)
    flush_print("sizes", dtype, planar, n)
    vol = to_np(ctx.score_volume_nfft(spec, gf, pos.astype(REAL[dtype]), coef.astype(CPLX[dtype]), quats, width=6))
    check_volumes(vol.astype(np.float64), rho_f, pos, coef, quats, planar, dtype, 6)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_nfft_peaks_match_oracle_volumes(ctxs, dtype):
    ctx = ctxs[dtype]
    pair, f = small_pair_fields()
    pos, coef, _, _ = ooc.octree_leaves(f.c, f.n_m, 0.0, 3)
    pos = pos.astype(REAL[dtype]).astype(np.float64)
    coef = coef.astype(CPLX[dtype]).astype(np.complex128)
    gf = pair.fixed.grid
    spec = ctx.spectrum(f.rho_f.astype(CPLX[dtype]), gf)
    quats = pair.quats[:3]
    out = ctx.score_rotations_nfft(spec, gf, pos.astype(REAL[dtype]), coef.astype(CPLX[dtype]), quats, width=6)
    s, t, nb = to_np(out["score"]).astype(np.float64), to_np(out["t"]), to_np(out["nbhd"]).astype(np.float64)
    tol = 1e-4 if dtype == "f32" else 1e-9
    for r, q in enumerate(quats):
        vol = onf.score_volume_trig(f.rho_f, pos, coef, q, False, w=6)
        scale = np.abs(vol).max()
        ref = vol.max()
        assert abs(s[r] - ref) <= tol * scale, (r, s[r], ref)
        # the GPU's t scores the peak value in the oracle volume (ties allowed)
        assert abs(vol[t[r][2], t[r][1], t[r][0]] - ref) <= tol * scale
        tz, ty, tx = t[r][2], t[r][1], t[r][0]
        k = 0
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    v = vol[(tz + dz) % 16, (ty + dy) % 16, (tx + dx) % 16]
                    assert abs(nb[r][k] - v) <= tol * scale
                    k += 1


@pytest.mark.parametrize("n,nrot", [(64, 5), (128, 3)])
def test_nfft_peaks_fp32_through_folded_inverse(ctxs, n, nrot):
    """FP32 3D peaks at N = 64 and 128 take the search path's inverse kernels
    (column-tile modes, rotation pairs folded into one inverse transform, the
    slab argmax and the FP64 finish): peaks, 27-neighbourhoods and sub-voxel
    refinement against the oracle's algorithm, with an odd rotation count so
    the last pair holds one rotation."""
    from oracle import peak as op
    ctx = ctxs["f32"]
    rng = np.random.default_rng(600 + n)
    rho_f = smooth_field(rng, n, False, damping=0.08 * n * n).astype(np.complex64)
    m = 2500
    pos = rng.uniform(-0.3 * n, 0.3 * n, (m, 3)).astype(np.float32)
    coef = (rng.normal(size=m) + 1j * rng.normal(size=m)).astype(np.complex64)
    gf = grid_spec(n, False)
    spec = ctx.spectrum(rho_f, gf)
    quats = wr.uniform_quaternions(nrot, 700 + n)
    flush_print("nfft fused peaks n", n, "rotations", nrot)
    out = ctx.score_rotations_nfft(spec, gf, pos, coef, quats, width=6)
    s, t = to_np(out["score"]).astype(np.float64), to_np(out["t"])
    nb, ref_t = to_np(out["nbhd"]).astype(np.float64), to_np(out["refined"])
    for r, q in enumerate(quats):
        vol = onf.score_volume_trig(rho_f.astype(np.complex128), pos.astype(np.float64), coef.astype(np.complex128),
                                    q, False, w=6)
        scale = np.abs(vol).max()
        s0, _, t0 = op.peak(vol)
        flush_print("  rotation", r, "score", s[r], "oracle", s0, "t", tuple(t[r]), t0)
        assert abs(s[r] - s0) <= 2e-5 * scale, (r, s[r], s0)
        if tuple(t[r]) != t0:  # a near-tie: the oracle's value there must match the max
            assert abs(vol[t[r][2], t[r][1], t[r][0]] - s0) <= 2e-5 * scale
        nb0 = op.neighbourhood(vol, tuple(t[r]))
        assert np.max(np.abs(nb[r] - nb0)) <= 2e-5 * scale
        assert np.max(np.abs(ref_t[r] - op.subvoxel(nb0, tuple(t[r])))) <= 1e-3


@pytest.mark.parametrize("dtype,planar,n", [("f32", False, 64), ("f64", False, 32), ("f32", True, 64)])
def test_nfft_repeats_bit_for_bit(ctxs, dtype, planar, n):
    """The bins list their samples in arrival order, which varies from run to
    run; each tile's fixed-point scale is an order-free sum, so repeated
    calls give identical volumes and peaks (FP32 line tiles with a tile
    crowded past the sorted candidates, FP64 general tiles, planar tiles)."""
    ctx = ctxs[dtype]
    rng = np.random.default_rng(800 + n + (1 if planar else 0))
    rho_f = smooth_field(rng, n, planar, damping=0.06 * n * n).astype(CPLX[dtype])
    dim = 2 if planar else 3
    centre = rng.uniform(-0.2 * n, 0.2 * n, dim)
    pts = np.concatenate([centre + rng.normal(scale=0.7, size=(2600, dim)),
                          rng.uniform(-0.45 * n, 0.45 * n, (900, dim))])
    if planar:
        pts = np.concatenate([pts, np.zeros((len(pts), 1))], axis=1)
    pos = pts.astype(REAL[dtype])
    coef = (rng.normal(size=len(pos)) + 1j * rng.normal(size=len(pos))).astype(CPLX[dtype])
    gf = grid_spec(n, planar)
    spec = ctx.spectrum(rho_f, gf)
    quats = planar_quats(3, 17) if planar else wr.uniform_quaternions(3, 900 + n)
    flush_print("nfft repeat", dtype, "planar" if planar else "3D", n)
    vols = [to_np(ctx.score_volume_nfft(spec, gf, pos, coef, quats, width=6)) for _ in range(3)]
    assert all(np.array_equal(vols[0], v) for v in vols[1:])
    outs = [ctx.score_rotations_nfft(spec, gf, pos, coef, quats, width=6) for _ in range(3)]
    for key in ("score", "t", "nbhd", "refined"):
        ref = to_np(outs[0][key])
        assert all(np.array_equal(ref, to_np(o[key])) for o in outs[1:]), key


def test_nfft_without_samples_scores_zero(ctxs):
    ctx = ctxs["f32"]
    gf = grid_spec(16, False)
    rng = np.random.default_rng(2)
    spec = ctx.spectrum(smooth_field(rng, 16, False).astype(np.complex64), gf)
    vol = to_np(ctx.score_volume_nfft(spec, gf, np.zeros((0, 3), np.float32), np.zeros(0, np.complex64),
                                      wr.uniform_quaternions(2, 1)))
    assert np.all(vol == 0)


def test_nfft_rejects_unsupported_grids(ctxs):
    from paper_1712_00238_amd._lib import SdfError
    ctx = ctxs["f32"]
    gf = grid_spec(16, False)
    spec = ctx.spectrum(np.zeros((16, 16, 16), np.complex64), gf)
    pos = np.zeros((4, 3), np.float32)
    c = np.ones(4, np.complex64)
    q = wr.uniform_quaternions(1, 1)
    with pytest.raises(SdfError):
        ctx.score_volume_nfft(spec, gf, pos, c, q, width=9)
    with pytest.raises(SdfError):
        ctx.score_volume_nfft(spec, gf, pos, c, q, width=1)
    # N = 48 has no transform plan: refused before any device work (the
    # spectrum passed is never read)
    with pytest.raises(SdfError):
        ctx.score_volume_nfft(spec, grid_spec(48, False), pos, c, q)


# ----------------------------------------------------------------------------- full size

def test_nfft_full_size_mechanical(ctxs):
    """128^3 fixed grid, 64^3 body box, FP32, in bench.py's configuration of
    the route: GPU SDFs, octree leaves (tol 0.01, 3 levels) checked against
    the oracle's decision on the same coefficients, and one rotation's whole
    volume against the oracle's algorithm on the GPU's leaves."""
    ctx = ctxs["f32"]
    pair = C.mechanical_3d()
    fx, mv = pair.fixed, pair.moving
    rho_f = ctx.sdf_build(fx.samples.q, fx.samples.n, fx.samples.w, fx.grid, pair.params)
    rho_m = ctx.sdf_build(mv.samples.q, mv.samples.n, mv.samples.w, mv.grid, pair.params)
    nm = mv.grid.n[0]
    w = np.ones((nm, nm, nm), np.float32)
    flush_print("full size: octree")
    pos, c, lev = ctx.octree_samples(rho_m, w, mv.grid, 0.01, 3)
    cin = to_np(rho_m).astype(np.complex64) * w
    rpos, rc, rlev, _ = ooc.octree_leaves(cin, nm, 0.01, 3, dtype=np.float32)
    flush_print("leaves", len(rlev), "of", nm ** 3)
    assert np.array_equal(to_np(lev), rlev)
    assert np.array_equal(to_np(pos).astype(np.float64), rpos)
    spec = ctx.spectrum(rho_f, fx.grid)
    q = pair.quats[:1]
    flush_print("full size: volume")
    vol = to_np(ctx.score_volume_nfft(spec, fx.grid, pos, c, q, width=6))[0].astype(np.float64)
    gpos = to_np(pos).astype(np.float64)
    gc = to_np(c).astype(np.complex128)
    ref = onf.score_volume_trig(to_np(rho_f).astype(np.complex128), gpos, gc, q[0], False, w=6)
    err = np.abs(vol - ref).max() / np.abs(ref).max()
    flush_print("full size: err vs algorithm", err)
    assert err <= 2e-5
    out = ctx.score_rotations_nfft(spec, fx.grid, pos, c, q, width=6)
    assert abs(float(to_np(out["score"])[0]) - ref.max()) <= 2e-5 * np.abs(ref).max()
