"""Pins of the FP64 oracle's skeletal density function to facts that do not
come from the oracle itself: closed forms derived from eq. 13 / 15 / 16c,
the sign pattern of Table 1, rigid covariance (eq. 8 remark and the
contact-region congruence of the Formulation section), the inverse-square
scaling law behind Proposition 1, and the truncation error bound of
Proposition 2 (eq. 18b)."""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import sdf as osdf
from workloads import shapes
from workloads.configs import SDFParams

P = SDFParams()  # lambda1 = 1, lambda2 = 3, sigma = 0.5, eps = 1.5 (validation section)


def circle_samples(a, n, centre=(0.0, 0.0)):
    th = (np.arange(n) + 0.5) * 2 * math.pi / n
    q = np.stack([centre[0] + a * np.cos(th), centre[1] + a * np.sin(th), np.zeros(n)], axis=1)
    nrm = np.stack([np.cos(th), np.sin(th), np.zeros(n)], axis=1)
    return shapes.PointSamples(q, nrm, np.full(n, 2 * math.pi * a / n))


def flat_patch(half, spacing, z=0.0, normal=1.0):
    m = int(round(2 * half / spacing))
    c = -half + (np.arange(m) + 0.5) * spacing
    x, y = np.meshgrid(c, c, indexing="ij")
    q = np.stack([x.ravel(), y.ravel(), np.full(x.size, z)], axis=1)
    nrm = np.zeros_like(q)
    nrm[:, 2] = normal
    return shapes.PointSamples(q, nrm, np.full(len(q), spacing * spacing))


def plane_closed_form(params, exterior=True):
    """Flat face at height h: with s = h sqrt(r^2 - 1), eta = h r,
    cos theta = +-1/r and ds = 2 pi s ds = 2 pi h^2 r dr, the sum of eq. 13
    over the contact disk becomes (lambda / sigma) int_1^{1+eps} G(r)
    (1 -+ i r)^2 / (1 + r^2)^2 dr, with no dependence on h."""
    s = params.sigma
    g = lambda r: math.exp(-0.5 * ((r - 1.0) / s) ** 2)
    sgn = -1.0 if exterior else 1.0
    re = integrate.quad(lambda r: g(r) * ((1 - r * r)) / (1 + r * r) ** 2, 1.0, 1.0 + params.eps, epsabs=1e-13)[0]
    im = integrate.quad(lambda r: g(r) * (sgn * 2 * r) / (1 + r * r) ** 2, 1.0, 1.0 + params.eps, epsabs=1e-13)[0]
    lam = params.lambda1 if exterior else params.lambda2
    return lam / s * (re + 1j * im)


def test_sphere_centre_closed_form():
    # Interior centre of a sphere of radius a: every sample has eta = |xi| = a,
    # cos theta = -1, so rho = i lambda2 sum(w) / (4 pi sigma a^2) = i lambda2 / sigma.
    for a in (3.0, 7.5):
        s = shapes.sphere_samples((1.0, -2.0, 0.5), a, density=6.0)
        rho = osdf.sdf_points(s, [(1.0, -2.0, 0.5)], P)[0]
        assert abs(rho - 1j * P.lambda2 / P.sigma) < 1e-12
        rho_np = osdf.sdf_points_numpy(s, [(1.0, -2.0, 0.5)], P)[0]
        assert abs(rho_np - 1j * P.lambda2 / P.sigma) < 1e-12


def test_circle_centre_closed_form():
    # Planar version: sum(w) = 2 pi a gives i lambda2 / (2 sigma a).
    for a, n in ((4.0, 200), (10.0, 513)):
        s = circle_samples(a, n, centre=(0.3, 0.7))
        rho = osdf.sdf_points(s, [(0.3, 0.7, 0.0)], P)[0]
        assert abs(rho - 1j * P.lambda2 / (2 * P.sigma * a)) < 1e-12


@pytest.mark.parametrize("h", [0.5, 1.0, 2.0])
def test_flat_plane_closed_form_and_height_independence(h):
    ext = plane_closed_form(P, exterior=True)
    inn = plane_closed_form(P, exterior=False)
    # interior value is (lambda2 / lambda1) conj(exterior value)
    assert abs(inn - P.lambda2 / P.lambda1 * np.conj(ext)) < 1e-12
    patch = flat_patch(half=3.2 * h, spacing=0.025 * h)
    rho_out = osdf.sdf_points(patch, [(0.0, 0.0, h)], P)[0]
    rho_in = osdf.sdf_points(patch, [(0.0, 0.0, -h)], P)[0]
    assert abs(rho_out - ext) < 2e-3 * abs(ext)
    assert abs(rho_in - inn) < 2e-3 * abs(inn)


def test_table1_signs_at_medial_points():
    # Exterior medial point: centre of the slot of the planar hole part.
    # Interior medial point: centre of the peg.
    hole = shapes.sample_polygon(shapes.HOLE_PART_2D, 4096, None)
    peg = shapes.sample_polygon(shapes.PEG_2D, 4096, None)
    r_ext = osdf.sdf_points(hole, [(0.0, 20.0, 0.0)], P)[0]
    r_int = osdf.sdf_points(peg, [(0.0, 0.0, 0.0)], P)[0]
    assert r_ext.imag < 0 < r_int.imag
    assert abs(r_ext.imag) > abs(r_ext.real) and abs(r_int.imag) > abs(r_int.real)
    # Table 1: ext-int overlap rewards, int-int and ext-ext overlaps penalise,
    # and the collision penalty dominates the separation penalty.
    assert (r_ext * r_int).real > 0
    assert (r_int * r_int).real < 0 and (r_ext * r_ext).real < 0
    assert abs((r_int * r_int).real) > abs((r_ext * r_ext).real)


def test_rigid_covariance():
    rng = np.random.default_rng(3)
    s = shapes.PointSamples.concat(shapes.sample_box_faces((-3, -2, -1.5), (3, 2, 1.5), 9.0, rng))
    pts = rng.uniform(-5, 5, size=(300, 3))
    a = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    if np.linalg.det(a) < 0:
        a[:, 0] *= -1
    b = rng.normal(size=3) * 4
    moved = shapes.PointSamples(s.q @ a.T + b, s.n @ a.T, s.w)
    r0 = osdf.sdf_points(s, pts, P)
    r1 = osdf.sdf_points(moved, pts @ a.T + b, P)
    assert np.max(np.abs(r0 - r1)) < 1e-9 * max(1.0, np.max(np.abs(r0)))


def test_inverse_square_scaling():
    # phi(alpha zeta) = alpha^-2 phi(zeta) for alpha > 0: scaling a 3D solid,
    # its area weights (alpha^2) and the query point leaves rho unchanged; in
    # 2D (arc weights scale by alpha) rho scales by 1/alpha.
    rng = np.random.default_rng(5)
    s = shapes.PointSamples.concat(shapes.sample_box_faces((-2, -1, -1), (2, 1, 1), 16.0, rng))
    pts = rng.uniform(-3, 3, size=(100, 3))
    alpha = 2.5
    big = shapes.PointSamples(s.q * alpha, s.n, s.w * alpha ** 2)
    p2 = SDFParams(xi_floor=P.xi_floor * alpha)
    r0 = osdf.sdf_points(s, pts, P)
    r1 = osdf.sdf_points(big, pts * alpha, p2)
    assert np.max(np.abs(r0 - r1)) < 1e-10 * np.max(np.abs(r0))
    c = circle_samples(3.0, 300)
    cb = circle_samples(3.0 * alpha, 300)
    pp = np.array([[0.5, -0.2, 0.0], [4.0, 1.0, 0.0]])
    assert np.max(np.abs(osdf.sdf_points(c, pp, P) / alpha - osdf.sdf_points(cb, pp * alpha, p2))) < 1e-12


def test_truncation_error_bound():
    # Proposition 2: the dropped tail obeys |E| <= |lambda| / (2 pi sigma)
    # exp(-eps^2 / (2 sigma^2)) * (unsigned observed solid angle).  The solid
    # angle carries the 4 pi that the printed 1D forms drop, i.e.
    # sum_j w_j |cos theta_j| / eta_j^2 over the samples.
    rng = np.random.default_rng(9)
    s = shapes.PointSamples.concat(shapes.sample_box_faces((-3, -2, -1.5), (3, 2, 1.5), 9.0, rng))
    pts = rng.uniform(-6, 6, size=(200, 3))
    full = SDFParams(eps=1e6)
    for eps in (0.5, 1.0, 1.5, 2.5):
        pe = SDFParams(eps=eps)
        err = np.abs(osdf.sdf_points(s, pts, full) - osdf.sdf_points(s, pts, pe))
        d = pts[:, None, :] - s.q[None]
        eta = np.linalg.norm(d, axis=-1)
        omega = (s.w * np.abs((d * s.n[None]).sum(-1)) / eta ** 3).sum(axis=1)
        # the larger |lambda| = lambda2 bounds both sides
        bound = P.lambda2 / (2 * math.pi * P.sigma) * math.exp(-eps ** 2 / (2 * P.sigma ** 2)) * omega
        assert np.all(err <= bound * (1 + 1e-9) + 1e-15), eps
    # and the tail vanishes as eps grows
    e1 = np.abs(osdf.sdf_points(s, pts, full) - osdf.sdf_points(s, pts, SDFParams(eps=4.3 * P.sigma)))
    e0 = np.abs(osdf.sdf_points(s, pts, full) - osdf.sdf_points(s, pts, SDFParams(eps=1.0 * P.sigma)))
    assert e1.max() < e0.max()


def test_boundary_floor_and_membership():
    c = circle_samples(5.0, 64)
    # exactly on a sample: pmc = 0 -> rho = 0; within the floor: 0
    on = c.q[3]
    near = c.q[3] * (1 + 0.2 / 5.0)
    rho = osdf.sdf_points(c, [on, near], P)
    assert rho[0] == 0 and rho[1] == 0
    # diagnostics: signed distance is negative inside, positive outside
    _, diag = osdf.sdf_points(c, [(0, 0, 0), (9, 0, 0)], P, diagnostics=True)
    assert diag["xi"][0] < 0 < diag["xi"][1]
    assert abs(diag["xi"][0] + 5.0) < 1e-9


def test_numpy_and_c_agree():
    rng = np.random.default_rng(11)
    s = shapes.sample_polygon(shapes.PEG_2D, 300, rng)
    pts = np.concatenate([rng.uniform(-25, 25, size=(400, 2)), np.zeros((400, 1))], axis=1)
    a = osdf.sdf_points(s, pts, P)
    b = osdf.sdf_points_numpy(s, pts, P)
    assert np.max(np.abs(a - b)) < 1e-10 * np.max(np.abs(a))


def tie_pair(order, near_tie):
    """Two samples on either side of the origin, facing +x, so the origin is
    inside for the sample at +x and outside for the one at -x.  Exact tie:
    both at squared distance 4.  Near tie: the +x sample is pushed off the
    axis by 2^-25, squared distance 4 + 2^-50 (exact in FP64) whose square
    root still rounds to 2."""
    qa = np.array([2.0, 2.0 ** -25 if near_tie else 0.0, 0.0])
    qb = np.array([-2.0, 0.0, 0.0])
    q = np.stack([qa, qb] if order == 0 else [qb, qa])
    w = np.array([1.0, 0.25]) if order == 0 else np.array([0.25, 1.0])
    return shapes.PointSamples(q, np.tile([1.0, 0.0, 0.0], (2, 1)), w)


@pytest.mark.parametrize("order", [0, 1])
def test_nearest_sample_tie_rule(order):
    """Reading of eq. 10A for sampled boundaries: the nearest sample is the
    exact-distance minimiser, lowest index among exact ties.  At an exact tie
    the lowest index decides the membership sign (a highest-index rule flips
    it); at a near tie whose distances round to the same square root, the
    strictly nearer sample decides (an argmin over rounded distances would
    take the lower index instead)."""
    origin = [(0.0, 0.0, 0.0)]
    exact = tie_pair(order, False)
    rho, diag = osdf.sdf_points(exact, origin, P, diagnostics=True)
    assert diag["nearest"][0] == 0
    assert diag["xi"][0] == (-2.0 if order == 0 else 2.0)  # +x sample first -> inside
    near = tie_pair(order, True)
    assert math.sqrt(float(np.sum(near.q[0 if order == 0 else 1] ** 2))) == 2.0
    rho_n, diag_n = osdf.sdf_points(near, origin, P, diagnostics=True)
    assert diag_n["nearest"][0] == (1 if order == 0 else 0)   # the -x sample, strictly nearer
    assert diag_n["xi"][0] == 2.0                             # outside
    # both branches give different affinities, and NumPy follows the same rule
    assert abs(rho[0] - rho_n[0]) > 1e-3 if order == 0 else abs(rho[0] - rho_n[0]) < 1e-12
    for s, r in ((exact, rho[0]), (near, rho_n[0])):
        assert abs(osdf.sdf_points_numpy(s, origin, P)[0] - r) <= 1e-12 * abs(r)
