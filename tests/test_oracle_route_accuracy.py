"""Why the nonequispaced route and the B-spline window score differently
(Implementation section).  Both meet the fixed field between its nodes: the
route's transform through the field's trigonometric interpolant, the search
through a local cubic B-spline.  The windowless reference (the turned part's
SDF built from its turned samples) needs neither, so each route's distance
from it is how well it reproduces the fixed SDF between nodes.

  * On a band-limited field the trigonometric interpolant is exact and the
    B-spline (a smoother, not an interpolant) is not.
  * The SDF is not band-limited: it has a steep layer at the boundary (the
    kernel of eq. 15 peaks there, the floor and the truncation of eq. 17t cut
    it).  The interpolant rings at that layer and, being global, carries the
    ringing cells away from it; the B-spline's error stays at the layer.
  * A placement's score sums the fixed field at the turned samples, so these
    errors enter every score: on the planar peg-in-hole pair the route's
    peaks sit farther from the reference's than the window's.  Where the best
    rotations of a pair lie within that error of each other, the route can
    pick another best rotation than the reference.

Everything here runs the oracle only."""

import numpy as np
import pytest

from oracle import correlate as oc
from oracle import direct as od
from oracle import nfft as onf
from oracle import peak as op
from oracle import pipeline
from oracle import sdf as osdf
from oracle import spread as osp
from workloads import configs as C


def bspline_smooth(rho2d, p):
    """sum_n rho(n) beta3(p - n) at planar points p (m, >= 2), periodic."""
    n = rho2d.shape[0]
    fl = np.floor(p[:, :2]).astype(int)
    out = np.zeros(len(p), dtype=np.complex128)
    for dy in range(-1, 3):
        for dx in range(-1, 3):
            nx, ny = fl[:, 0] + dx, fl[:, 1] + dy
            out += osp.bspline3(p[:, 0] - nx) * osp.bspline3(p[:, 1] - ny) * rho2d[ny % n, nx % n]
    return out


def test_trig_interpolant_exact_on_band_limited_field():
    n = 64
    rng = np.random.default_rng(11)
    modes = [(int(rng.integers(-8, 9)), int(rng.integers(-8, 9)), rng.normal() + 1j * rng.normal()) for _ in range(12)]

    def field(x, y):
        return sum(a * np.exp(2j * np.pi * (kx * x + ky * y) / n) for kx, ky, a in modes)

    yy, xx = np.mgrid[0:n, 0:n]
    rho = field(xx, yy)[None]
    p = np.concatenate([rng.uniform(0, n, (400, 2)), np.zeros((400, 1))], axis=1)
    exact = field(p[:, 0], p[:, 1])
    scale = np.abs(rho).max()
    e_trig = np.abs(onf.trig_interpolant(rho, p, planar=True) - exact).max() / scale
    e_bs = np.median(np.abs(bspline_smooth(rho[0], p) - exact)) / scale
    assert e_trig < 1e-10
    assert e_bs > 1e-3  # the B-spline smooths a band-limited field


@pytest.fixture(scope="module")
def peg():
    pair = C.peg_in_hole_2d(seed=0)
    return pair, pipeline.build_fields(pair)


def test_sdf_layer_rings_through_the_trig_interpolant(peg):
    pair, f = peg
    fx = pair.fixed
    s, g = fx.samples, fx.grid
    rng = np.random.default_rng(1)
    m = 3000
    idx = rng.choice(len(s.q), m)
    xi = rng.uniform(-3.0, 3.0, m)  # signed offset along the normal, in cells
    pw = s.q[idx] + xi[:, None] * s.n[idx] * g.h + rng.normal(scale=0.3 * g.h, size=(m, 3))
    pw[:, 2] = s.q[idx, 2]
    p = (pw - np.asarray(g.origin)) / g.h
    exact = osdf.sdf_points(s, pw, pair.params)
    trig = onf.trig_interpolant(f.rho_f, p, planar=True)
    bs = bspline_smooth(f.rho_f[0], p)
    scale = np.abs(f.rho_f).max()
    for lo, hi, ratio in ((1.0, 3.0, 5.0), (-3.0, -1.0, 2.0)):
        sel = (xi >= lo) & (xi < hi)
        e_trig = np.median(np.abs(trig - exact)[sel]) / scale
        e_bs = np.median(np.abs(bs - exact)[sel]) / scale
        assert e_trig > ratio * e_bs, (lo, hi, e_trig, e_bs)
    # one to three cells outside the layer the window is accurate to 1%
    sel = xi >= 1.0
    assert np.median(np.abs(bs - exact)[sel]) / scale < 1e-2


def test_route_peaks_farther_from_reference_than_window(peg):
    pair, f = peg
    mv = pair.moving
    w_node = float(mv.grid.h ** 2)
    pos = osp.body_positions(f.n_m, True)
    win, trig, ref = [], [], []
    for q in pair.quats:
        win.append(op.peak(oc.score_volume(f.rho_f, f.c, q, f.n_m, True))[0])
        trig.append(op.peak(onf.score_volume_trig(f.rho_f, pos, f.c, q, True))[0])
        ref.append(op.peak(od.direct_volume(f.rho_f, mv.samples, mv.grid, pair.params, q, w_node, True))[0])
    win, trig, ref = np.array(win), np.array(trig), np.array(ref)
    scale = np.abs(ref).max()
    d_win = np.median(np.abs(win - ref)) / scale
    d_trig = np.median(np.abs(trig - ref)) / scale
    assert d_trig > 1.5 * d_win, (d_trig, d_win)
    # the seated pose wins by > 40% here, far beyond either error
    assert int(np.argmax(win)) == int(np.argmax(ref)) == int(np.argmax(trig))
