"""The alternative phi-kernels of sdf_build_phi (inverse-square, radial basis,
double skin layer) against the oracle (oracle/phi.py), through the C ABI:
ragged grids, planar and 3D parts, the 256-sample tile edges, a two-sided
radial shell (eps < 1), and sampled nodes of the full 128^3 mechanical part."""

import numpy as np
import pytest

from helpers import flush_print
from oracle import phi as ophi
from oracle import sdf as osdf
from workloads import configs as C
from workloads import shapes

pytestmark = pytest.mark.gpu

KINDS = ["inverse_square", "radial", "dsl"]


@pytest.fixture(scope="module")
def ctxs():
    from paper_1712_00238_amd.api import Context
    c32, c64 = Context(0, "f32"), Context(0, "f64")
    yield {"f32": c32, "f64": c64}
    c32.close()
    c64.close()


def decision_free(kind, samples, pts, params, radius, band):
    """Nodes where the FP64 oracle sits within `band` of a discrete decision the
    kernel takes with other rounding: the nearest sample tied across the
    boundary or on the floor (inverse-square, DSL), the contact ball's edge
    (inverse-square), a Gaussian truncation edge (DSL: of xi / R -+ 1; radial:
    of |p - s| / R - 1 for some offset point)."""
    _, diag = osdf.sdf_points(samples, pts, params, diagnostics=True, band_rel=band)
    xi = diag["xi"]
    free = diag["pmc_gap"] <= band * np.maximum(np.abs(xi), 1.0)
    if kind == "inverse_square":
        free |= diag["trunc_margin"] <= band
        free |= np.abs(np.abs(xi) - params.xi_floor) <= band * np.maximum(np.abs(xi), 1.0)
    elif kind == "dsl":
        for sgn in (-1.0, 1.0):
            free |= np.abs(np.abs(xi / radius + sgn) - params.eps) <= band * max(1.0, params.eps)
    else:
        free[:] = False
        for off in (radius * samples.n, -radius * samples.n):
            s = samples.q + off
            for a in range(0, len(pts), 512):
                e = np.sqrt(((pts[a:a + 512, None, :] - s[None, :, :]) ** 2).sum(-1))
                m = np.abs(np.abs(e / radius - 1.0) - params.eps).min(axis=1)
                free[a:a + 512] |= m <= band * max(1.0, params.eps)
    return free


def compare(kind, got, samples, pts, params, radius, dtype):
    ref = ophi.phi_points(samples, pts, params, kind, radius)
    # the kernels take every discrete decision in FP64 in both precisions, so
    # the band only covers FP64 rounding; FP32 changes the sum itself
    rel = 1e-10 if dtype == "f64" else 2e-5
    free = decision_free(kind, samples, pts, params, radius, 1e-9)
    scale = np.abs(ref).max()
    err = np.abs(np.asarray(got).reshape(-1) - ref)
    bad = (err > rel * scale) & ~free
    rep = {"max_err": float(err[~free].max()) if (~free).any() else 0.0, "scale": float(scale),
           "n_free": int(free.sum()), "n": len(ref), "n_bad": int(bad.sum())}
    flush_print(kind, dtype, rep)
    assert scale > 0
    assert not bad.any(), rep
    assert free.mean() <= 0.01, rep


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind", KINDS)
def test_phi_small_3d_ragged(ctxs, dtype, kind):
    pair = C.small_3d(seed=1, n=16, n_m=6)
    s = pair.fixed.samples
    grid = C.GridSpec((15, 13, 11), (-7.3, -6.1, -5.2), 1.0)
    radius = 1.37
    got = ctxs[dtype].sdf_build(s.q, s.n, s.w, grid, pair.params, phi=kind, radius=radius).cpu().numpy()
    compare(kind, got, s, grid.node_positions(), pair.params, radius, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind", KINDS)
def test_phi_planar_pair(ctxs, dtype, kind):
    pair = C.peg_in_hole_2d(seed=0)
    radius = 2.11
    for part in (pair.fixed, pair.moving):
        s = part.samples
        got = ctxs[dtype].sdf_build(s.q, s.n, s.w, part.grid, pair.params, phi=kind, radius=radius).cpu().numpy()
        compare(kind, got, s, part.grid.node_positions(), pair.params, radius, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("count", [1, 256, 257, 700])
def test_phi_sample_tile_edges(ctxs, dtype, kind, count):
    rng = np.random.default_rng(count)
    v = rng.normal(size=(count, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    s = shapes.PointSamples(4.0 * v + 0.3, v.copy(), np.full(count, 4.0 * np.pi * 16.0 / count))
    grid = C.GridSpec((14, 13, 12), (-6.5, -6.0, -5.5), 1.0)
    params = C.SDFParams(xi_floor=0.25)
    radius = 1.73
    got = ctxs[dtype].sdf_build(s.q, s.n, s.w, grid, params, phi=kind, radius=radius).cpu().numpy()
    compare(kind, got, s, grid.node_positions(), params, radius, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_radial_two_sided_shell(ctxs, dtype):
    """eps < 1: the shell R (1 - eps) <= |p - s| <= R (1 + eps) has an inner edge,
    and bricks whose tiles lie inside it skip them."""
    pair = C.small_3d(seed=2, n=16, n_m=6)
    s = pair.fixed.samples
    params = C.SDFParams(sigma=0.2, eps=0.6)
    grid = C.GridSpec((16, 15, 13), (-7.7, -7.1, -6.3), 0.9)
    got = ctxs[dtype].sdf_build(s.q, s.n, s.w, grid, params, phi="radial", radius=2.9).cpu().numpy()
    compare("radial", got, s, grid.node_positions(), params, 2.9, dtype)


@pytest.mark.parametrize("kind", ["radial", "dsl"])
def test_phi_rejects_bad_radius(ctxs, kind):
    from paper_1712_00238_amd._lib import SDF_EINVAL, SdfError
    pair = C.small_3d(seed=1, n=16, n_m=6)
    s = pair.fixed.samples
    for r in (0.0, -1.0, float("nan")):
        with pytest.raises(SdfError) as ei:
            ctxs["f32"].sdf_build(s.q, s.n, s.w, pair.fixed.grid, pair.params, phi=kind, radius=r)
        assert ei.value.code == SDF_EINVAL


@pytest.mark.parametrize("kind", KINDS)
def test_phi_mechanical_full_grid_sampled_nodes(ctxs, kind):
    """The 128^3 mechanical receptor (15.7k samples), FP32, 2000 sampled nodes."""
    pair = C.mechanical_3d(seed=0)
    part = pair.fixed
    radius = 2.37
    flush_print("phi full grid", kind)
    rho = ctxs["f32"].sdf_build(part.samples.q, part.samples.n, part.samples.w, part.grid, pair.params, phi=kind,
                                radius=radius)
    rng = np.random.default_rng(7)
    flat = rng.choice(part.grid.size, size=2000, replace=False)
    got = rho.reshape(-1).cpu().numpy()[flat]
    compare(kind, got, part.samples, part.grid.node_positions()[flat], pair.params, radius, "f32")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dsl_search_planar_matches_oracle(ctxs, dtype):
    """The whole search on DSL affinities (probe radius 2) of the planar
    peg-in-hole pair: GPU-built fields, 36 rotations, peaks against the oracle's
    fields and FFT correlation."""
    from oracle import correlate as oc
    from oracle import peak as op
    from oracle import pipeline
    import torch
    pair = C.peg_in_hole_2d(seed=0)
    fx, mv = pair.fixed, pair.moving
    ctx = ctxs[dtype]
    rf = ctx.sdf_build(fx.samples.q, fx.samples.n, fx.samples.w, fx.grid, pair.params, phi="dsl", radius=2.0)
    rm = ctx.sdf_build(mv.samples.q, mv.samples.n, mv.samples.w, mv.grid, pair.params, phi="dsl", radius=2.0)
    w = torch.ones(rm.shape, dtype=ctx.real, device=rm.device)
    out = ctx.score_rotations(ctx.spectrum(rf, fx.grid), fx.grid, rm, w, mv.grid, pair.quats)
    s, t = out["score"].cpu().numpy(), out["t"].cpu().numpy()
    ref_f = ophi.phi_grid(fx.samples, fx.grid, pair.params, "dsl", 2.0)
    ref_m = ophi.phi_grid(mv.samples, mv.grid, pair.params, "dsl", 2.0)
    c = oc.moving_coefficients(ref_m, pipeline.body_weights(mv.grid))
    tol = 1e-9 if dtype == "f64" else 1e-4
    best = []
    for r, q in enumerate(pair.quats):
        vol = oc.score_volume(ref_f, c, q, mv.grid.n[0], True)
        s0, _, t0 = op.peak(vol)
        best.append(s0)
        scale = np.abs(vol).max()
        assert abs(s[r] - s0) <= tol * scale, (r, s[r], s0)
        if tuple(t[r]) != t0:
            assert abs(vol[t[r][2], t[r][1], t[r][0]] - s0) <= tol * scale
    assert int(np.argmax(s)) == int(np.argmax(best))
