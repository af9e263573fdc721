"""Pins of the oracle's alternative phi-kernels (oracle/phi.py) to facts that
do not come from the oracle: closed forms of each kernel on a sphere and on a
flat face, the skin / core reward pattern the paper states for the radial and
double-skin-layer affinities (Our Approach section), the inverse-square scaling
law behind Proposition 1, and rigid covariance."""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import phi as ophi
from oracle import sdf as osdf
from workloads import shapes
from workloads.configs import SDFParams

P = SDFParams()  # lambda1 = 1, lambda2 = 3, sigma = 0.5, eps = 1.5


def flat_patch(half, spacing, normal=1.0):
    m = int(round(2 * half / spacing))
    c = -half + (np.arange(m) + 0.5) * spacing
    x, y = np.meshgrid(c, c, indexing="ij")
    q = np.stack([x.ravel(), y.ravel(), np.zeros(x.size)], axis=1)
    nrm = np.zeros_like(q)
    nrm[:, 2] = normal
    return shapes.PointSamples(q, nrm, np.full(len(q), spacing * spacing))


def g(x, s=P.sigma):
    return math.exp(-0.5 * (x / s) ** 2) / (math.sqrt(2 * math.pi) * s)


def gb(x, s=P.sigma, eps=P.eps):
    return g(x, s) if abs(x) <= eps else 0.0


# ----------------------------------------------------------------------------- inverse square

def test_inverse_square_sphere_centre():
    # every sample at eta = |xi| = a (r = 1, the medial Gaussian's peak), cos theta = -1:
    # the value equals the skeletal kernel's, i lambda2 / sigma for sum(w) = 4 pi a^2
    for a in (3.0, 7.5):
        s = shapes.sphere_samples((1.0, -2.0, 0.5), a, density=6.0)
        rho = ophi.phi_points(s, [(1.0, -2.0, 0.5)], P, "inverse_square")[0]
        assert abs(rho - 1j * P.lambda2 / P.sigma) < 1e-12


@pytest.mark.parametrize("h", [0.5, 1.0, 2.0])
def test_inverse_square_flat_face_closed_form(h):
    # With s = h sqrt(r^2 - 1), eta = h r, cos theta = +-1/r, ds = 2 pi h^2 r dr and
    # zeta = h(+-1 + i r), the contact disk gives (lambda1 / sigma) int_1^{1+eps} dr / (1 + i r)^2
    # outside and (lambda2 / sigma) int_1^{1+eps} dr / (1 - i r)^2 inside, whose antiderivatives are
    # i / (1 + i r) and -i / (1 - i r): no dependence on h.
    r1 = 1.0 + P.eps
    ext = P.lambda1 / P.sigma * (1j / (1 + 1j * r1) - 1j / (1 + 1j))
    inn = P.lambda2 / P.sigma * (-1j / (1 - 1j * r1) + 1j / (1 - 1j))
    patch = flat_patch(half=3.2 * h, spacing=0.025 * h)
    r_out, r_in = ophi.phi_points(patch, [(0.0, 0.0, h), (0.0, 0.0, -h)], P, "inverse_square")
    assert abs(r_out - ext) < 2e-3 * abs(ext)
    assert abs(r_in - inn) < 2e-3 * abs(inn)
    # Table 1's signs survive without the medial component
    assert r_out.imag < 0 < r_in.imag


def test_inverse_square_scale_invariance():
    # phi(alpha zeta) = alpha^-2 phi(zeta): scaling a 3D solid, its area weights and the
    # query points leaves rho unchanged (Proposition 1's premise)
    rng = np.random.default_rng(5)
    s = shapes.PointSamples.concat(shapes.sample_box_faces((-2, -1, -1), (2, 1, 1), 16.0, rng))
    pts = rng.uniform(-3, 3, size=(100, 3))
    alpha = 2.5
    big = shapes.PointSamples(s.q * alpha, s.n, s.w * alpha ** 2)
    r0 = ophi.phi_points(s, pts, P, "inverse_square")
    r1 = ophi.phi_points(big, pts * alpha, SDFParams(xi_floor=P.xi_floor * alpha), "inverse_square")
    assert np.max(np.abs(r0 - r1)) < 1e-10 * np.max(np.abs(r0))


# ----------------------------------------------------------------------------- radial basis

@pytest.mark.parametrize("a,R", [(2.5, 2.0), (3.0, 1.5), (1.0, 4.0)])
def test_radial_sphere_centre(a, R):
    # skin points at distance a + R from the centre, core points at |a - R|, so for sum(w) = 4 pi a^2:
    # rho = 4 pi a^2 [lambda1 gb(a / R) + i lambda2 gb(|a - R| / R - 1)]
    s = shapes.sphere_samples((0.3, -1.0, 2.0), a, density=8.0)
    rho = ophi.phi_points(s, [(0.3, -1.0, 2.0)], P, "radial", R)[0]
    want = 4 * math.pi * a * a * (P.lambda1 * gb(a / R) + 1j * P.lambda2 * gb(abs(a - R) / R - 1))
    assert abs(rho - want) < 1e-12 * max(1.0, abs(want))
    assert abs(want) > 0


def radial_plane(d, R):
    """Point at signed height d over an infinite face (normal +z): the skin offset lies at z = R and
    the core offset at z = -R; a plane at distance c contributes 2 pi int_c^inf eta gb(eta / R - 1) d eta."""
    def shell(c):
        lo, hi = max(c, R * max(0.0, 1 - P.eps)), R * (1 + P.eps)
        if lo >= hi:
            return 0.0
        return 2 * math.pi * integrate.quad(lambda e: e * g(e / R - 1), lo, hi, epsabs=1e-13, epsrel=1e-12)[0]
    return P.lambda1 * shell(abs(d - R)) + 1j * P.lambda2 * shell(abs(d + R))


@pytest.mark.parametrize("d", [0.5, 1.0, 2.5, -0.7, -2.0])
def test_radial_flat_face(d):
    R = 1.0
    patch = flat_patch(half=3.5, spacing=0.02)
    rho = ophi.phi_points(patch, [(0.01, -0.013, d)], P, "radial", R)[0]
    want = radial_plane(d, R)
    assert abs(rho - want) < 2e-3 * abs(want), (rho, want)


# ----------------------------------------------------------------------------- double skin layer

@pytest.mark.parametrize("h", [0.5, 1.5, 2.0, 3.0])
def test_dsl_on_signed_distance_of_a_face(h):
    # directly over (under) a sample of a face the nearest-sample distance is exactly h and the
    # membership +1 (-1): rho = lambda1 gb(+-h / R - 1) + i lambda2 gb(+-h / R + 1)
    R = 2.0
    patch = flat_patch(half=4.0, spacing=0.25)
    x, y = patch.q[137, 0], patch.q[137, 1]
    out, inn = ophi.phi_points(patch, [(x, y, h), (x, y, -h)], P, "dsl", R)
    assert abs(out - (P.lambda1 * gb(h / R - 1) + 1j * P.lambda2 * gb(h / R + 1))) < 1e-14
    assert abs(inn - (P.lambda1 * gb(-h / R - 1) + 1j * P.lambda2 * gb(-h / R + 1))) < 1e-14


def test_dsl_sphere_centre_and_boundary():
    a, R = 3.0, 2.5
    s = shapes.sphere_samples((0.0, 0.0, 0.0), a, density=4.0)
    c, on = ophi.phi_points(s, [(0.0, 0.0, 0.0), tuple(s.q[5])], P, "dsl", R)
    assert abs(c - (P.lambda1 * gb(-a / R - 1) + 1j * P.lambda2 * gb(1 - a / R))) < 1e-14
    # on a sample xi = 0: both layers meet there, no singularity and no floor
    assert abs(on - (P.lambda1 + 1j * P.lambda2) * g(1.0)) < 1e-14


@pytest.mark.parametrize("kind", ["dsl", "radial"])
def test_skin_core_reward_pattern(kind):
    # Our Approach section: skin (real, lambda1) overlaps reward, core (imaginary, lambda2)
    # collisions penalise, Re f = Re(rho1 rho2).  Outside a face at the skin's peak distance the
    # affinity is real and positive, inside at the core's peak it is imaginary.
    R = 1.0
    patch = flat_patch(half=3.5, spacing=0.05)
    skin = 2.0 * R if kind == "radial" else R
    ext, core = ophi.phi_points(patch, [(0.0, 0.0, skin), (0.0, 0.0, -skin)], P, kind, R)
    assert ext.real > 0 and abs(ext.imag) < 1e-3 * ext.real
    assert core.imag > 0 and abs(core.real) < 1e-3 * core.imag
    assert (ext * ext).real > 0 > (core * core).real
    assert abs((ext * core).real) < 1e-3 * abs(ext * core)


# ----------------------------------------------------------------------------- all kernels

@pytest.mark.parametrize("kind", ophi.KINDS)
def test_rigid_covariance_all_kernels(kind):
    rng = np.random.default_rng(3)
    s = shapes.PointSamples.concat(shapes.sample_box_faces((-3, -2, -1.5), (3, 2, 1.5), 9.0, rng))
    pts = rng.uniform(-5, 5, size=(200, 3))
    a = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    if np.linalg.det(a) < 0:
        a[:, 0] *= -1
    b = rng.normal(size=3) * 4
    moved = shapes.PointSamples(s.q @ a.T + b, s.n @ a.T, s.w)
    r0 = ophi.phi_points(s, pts, P, kind, 1.2)
    r1 = ophi.phi_points(moved, pts @ a.T + b, P, kind, 1.2)
    assert np.max(np.abs(r0 - r1)) < 1e-9 * max(1.0, np.max(np.abs(r0)))


def test_skeletal_kind_is_the_sdf():
    rng = np.random.default_rng(1)
    s = shapes.PointSamples.concat(shapes.sample_box_faces((-3, -2, -1.5), (3, 2, 1.5), 9.0, rng))
    pts = rng.uniform(-5, 5, size=(50, 3))
    assert np.array_equal(ophi.phi_points(s, pts, P, "skeletal"), osdf.sdf_points(s, pts, P))


def best_pose_and_shape(pair, kind, radius):
    from oracle import correlate as oc
    from oracle import peak as op
    from oracle import pipeline
    fx, mv = pair.fixed, pair.moving
    rf = ophi.phi_grid(fx.samples, fx.grid, pair.params, kind, radius)
    rm = ophi.phi_grid(mv.samples, mv.grid, pair.params, kind, radius)
    c = oc.moving_coefficients(rm, pipeline.body_weights(mv.grid))
    best = None
    for r, q in enumerate(pair.quats):
        vol = oc.score_volume(rf, c, q, mv.grid.n[0], True)
        s, _, t = op.peak(vol)
        if best is None or s > best[0]:
            best = (s, r, t, vol[0])
    s, r, t, v = best
    support = float((np.abs(v) > 1e-3 * np.abs(v).max()).mean())
    step = max(np.abs(np.roll(v, -1, a) - v).max() for a in (0, 1)) / v.max()
    return r, t, support, step


def test_validation_dsl_against_skeletal_on_the_planar_pair():
    """The Validation section's comparison, on the planar peg-in-hole pair:
    the skeletal affinity seats the peg in the slot (0 or 180 degrees), with a
    score that is nonzero everywhere and varies smoothly; the DSL affinity
    (probe radius 2) has a narrower support and sharper steps, and prefers a
    single flat contact outside the slot (the Our Approach section's
    criticism that skin overlap does not reward multiple contact)."""
    from workloads import configs as C
    pair = C.peg_in_hole_2d(seed=0)
    r, t, sup_s, step_s = best_pose_and_shape(pair, "skeletal", 0.0)
    assert (r, t[:2]) in ((0, (64, 84)), (18, (63, 83)))
    rd, td, sup_d, step_d = best_pose_and_shape(pair, "dsl", 2.0)
    assert (rd, td[:2]) not in ((0, (64, 84)), (18, (63, 83)))
    assert sup_s > sup_d and step_d > 2 * step_s
