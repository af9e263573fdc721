"""Pins of the windowless reference search (oracle/direct.py) against what
eq. 8 and the affinity's covariance fix, independent of its code:
  * covariance: the affinity of the turned samples at a node equals the
    affinity of the unturned samples at the node turned back (R^T about the
    body centre), evaluated pointwise by the oracle's SDF;
  * identity: with R = I the turned box SDF is the plain box SDF;
  * placement: the FFT route equals the brute-force sum
    f(t) = sum_k w rho_R(x_k) rho_F((x_k + t) mod N) on a tiny grid."""

import numpy as np
import pytest

from oracle import direct as od
from oracle import rotation as orot
from oracle import sdf as osdf
from workloads import configs as C
from workloads import rotations as wr


def _pair():
    return C.small_3d(seed=1, n=16, n_m=6)


@pytest.mark.parametrize("qi", [0, 1, 2])
def test_turned_sdf_is_covariant(qi):
    pair = _pair()
    mv = pair.moving
    q = wr.uniform_quaternions(3, 5)[qi]
    rho_r = od.turned_box_sdf(mv.samples, mv.grid, pair.params, q).ravel()
    c = od.body_centre(mv.grid)
    x = mv.grid.node_positions() - c
    r = orot.quat_to_matrix(q)
    back = c + x @ r  # c + R^T x, row form
    rho_b, diag = osdf.sdf_points(mv.samples, back, pair.params, diagnostics=True)
    scale = np.abs(rho_b).max()
    # nodes whose classification sits within rounding of a tie may differ
    amb = (diag["trunc_margin"] <= 1e-9) | (diag["pmc_gap"] <= 1e-9 * np.maximum(np.abs(diag["xi"]), 1.0))
    err = np.abs(rho_r - rho_b)
    assert np.all(err[~amb] <= 1e-9 * scale), float(err[~amb].max() / scale)
    assert amb.mean() < 0.02


def test_identity_turn_is_the_box_sdf():
    pair = _pair()
    mv = pair.moving
    rho_i = od.turned_box_sdf(mv.samples, mv.grid, pair.params, np.array([1.0, 0.0, 0.0, 0.0]))
    rho_0 = osdf.sdf_grid(mv.samples, mv.grid, pair.params)
    assert np.allclose(rho_i, rho_0, rtol=0, atol=1e-12 * np.abs(rho_0).max())


def test_direct_volume_is_the_brute_force_sum():
    pair = _pair()
    fx, mv = pair.fixed, pair.moving
    rng = np.random.default_rng(3)
    n = 8
    rho_f = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    q = wr.uniform_quaternions(1, 9)[0]
    w_node = 0.7
    vol = od.direct_volume(rho_f, mv.samples, mv.grid, pair.params, q, w_node)
    rho_r = od.turned_box_sdf(mv.samples, mv.grid, pair.params, q)
    nm = mv.grid.n[0]
    for t in [(0, 0, 0), (1, 2, 3), (7, 0, 5), (4, 4, 4)]:
        f = 0j
        for kz in range(nm):
            for ky in range(nm):
                for kx in range(nm):
                    x = np.array([kx, ky, kz]) - nm // 2
                    p = np.mod(x + np.array(t), n)
                    f += w_node * rho_r[kz, ky, kx] * rho_f[p[2], p[1], p[0]]
        assert abs(vol[t[2], t[1], t[0]] - f.real) <= 1e-10 * max(1.0, abs(f)), t


def test_odd_body_box_is_refused():
    with pytest.raises(ValueError):
        od.placed_grid(np.zeros((5, 5, 5)), 5, (8, 8, 8), 1.0)
