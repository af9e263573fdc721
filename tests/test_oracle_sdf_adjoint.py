"""Pins of the SDF adjoint (oracle/sdf_adjoint.py) against central finite
differences of the oracle's own SDF (sdf.py), which share no derivative code
with it.  Every perturbed parameter is checked for a change of the discrete
choices (nearest sample, membership, contact-ball set) between the two
evaluations; such parameters are skipped, and the test requires that almost
none are.  The weight gradient is also pinned exactly: L is linear in w."""

import numpy as np
import pytest

from oracle import sdf as osdf
from oracle import sdf_adjoint as oadj
from workloads import configs as C
from workloads import shapes


def _case(seed):
    rng = np.random.default_rng(seed)
    m = 40
    v = rng.normal(size=(m, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    rad = 3.0 + 0.3 * rng.normal(size=m)
    q = rad[:, None] * v
    nrm = v + 0.2 * rng.normal(size=(m, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    w = rng.uniform(0.5, 1.5, size=m)
    pts = rng.uniform(-7.0, 7.0, size=(60, 3))
    cot = rng.normal(size=60) + 1j * rng.normal(size=60)
    return shapes.PointSamples(q, nrm, w), pts, cot, C.SDFParams(xi_floor=0.25)


def _structure(s, pts, params):
    d = pts[:, None, :] - s.q[None, :, :]
    eta2 = np.einsum("pjk,pjk->pj", d, d)
    js = np.argmin(eta2, axis=1)
    xi2 = eta2[np.arange(len(pts)), js]
    dot = np.einsum("pk,pk->p", d[np.arange(len(pts)), js], s.n[js])
    ball = eta2 <= (1 + params.eps) ** 2 * xi2[:, None]
    live = (np.sign(dot) != 0) & (np.sqrt(xi2) >= params.xi_floor)
    return js, np.sign(dot), ball, live


def _L(s, pts, params, cot):
    return float(np.real(np.sum(cot * osdf.sdf_points(s, pts, params))))


@pytest.mark.parametrize("seed", [0, 1])
def test_adjoint_matches_central_differences(seed):
    s, pts, cot, params = _case(seed)
    gq, gn, gw = oadj.sdf_adjoint_points(s, pts, params, cot)
    h = 1e-6
    base = _structure(s, pts, params)
    checked = skipped = 0
    worst = 0.0
    scale = max(np.abs(gq).max(), np.abs(gn).max(), np.abs(gw).max())
    for what, arr, grad in (("q", s.q, gq), ("n", s.n, gn), ("w", s.w, gw)):
        for idx in np.ndindex(arr.shape):
            vals = []
            stable = True
            for sign in (1.0, -1.0):
                a = arr.copy()
                a[idx] += sign * h
                s2 = shapes.PointSamples(a if what == "q" else s.q, a if what == "n" else s.n,
                                         a if what == "w" else s.w)
                st = _structure(s2, pts, params)
                if not all(np.array_equal(x, y) for x, y in zip(st, base)):
                    stable = False
                vals.append(_L(s2, pts, params, cot))
            if not stable:
                skipped += 1
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            worst = max(worst, abs(fd - grad[idx]) / scale)
            checked += 1
    assert skipped <= 0.05 * (checked + skipped), (skipped, checked)
    assert worst <= 1e-6, worst


def test_weight_gradient_is_exact_by_linearity():
    s, pts, cot, params = _case(3)
    _, _, gw = oadj.sdf_adjoint_points(s, pts, params, cot)
    for j in (0, 7, 21):
        e = np.zeros(len(s.w))
        e[j] = s.w[j]
        # rho is linear in w with the discrete choices fixed (they do not depend on w)
        lj = _L(shapes.PointSamples(s.q, s.n, e), pts, params, cot)
        assert abs(gw[j] * s.w[j] - lj) <= 1e-12 * max(1.0, abs(lj))


def test_fixed_cotangent_is_the_adjoint_of_the_gather():
    """sum_b s_b f_b evaluated by gathering Phi at the moved samples equals
    Re sum_p rho_F(p) G(p) with G the spread cotangent (the gather and the
    spread are transposes)."""
    from oracle import grad as og
    from oracle import spread as osp
    from workloads import rotations as wr
    rng = np.random.default_rng(5)
    n, nm = 12, 5
    rho_f = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    c = rng.normal(size=nm ** 3) + 1j * rng.normal(size=nm ** 3)
    xb = osp.body_positions(nm)
    B = 4
    poses = np.concatenate([rng.uniform(-n, 2 * n, size=(B, 3)), wr.uniform_quaternions(B, 3)], axis=1)
    s = rng.normal(size=B)
    gather = sum(s[b] * og.pose_value(rho_f, c, xb, poses[b, :3], poses[b, 3:]) for b in range(B))
    g = og.fixed_cotangent(c, xb, poses, s, rho_f.shape)
    assert abs(gather - np.real(np.sum(rho_f * g))) <= 1e-10 * max(1.0, abs(gather))
