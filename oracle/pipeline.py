"""ORACLE - TEST INFRASTRUCTURE ONLY.  End-to-end FP64 scoring of a pair.

Follows the paper's flow: affinities of both parts on their grids once
(SDFs precomputed and reused, validation section), then per rotation one
correlation over all translations (Implementation section), then the peak.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import correlate, peak, sdf


@dataclass
class PairFields:
    rho_f: np.ndarray   # complex128 (nz, ny, nx)
    rho_m: np.ndarray   # complex128 (n_m, n_m, n_m) or (1, n_m, n_m)
    w_m: np.ndarray     # float64, same shape as rho_m
    c: np.ndarray       # complex128 flat
    n_m: int
    planar: bool


def body_weights(grid) -> np.ndarray:
    """Volume element per body node: h^3 in 3D, h^2 in the plane."""
    nx, ny, nz = grid.n
    hv = grid.h ** (2 if nz == 1 else 3)
    return np.full((nz, ny, nx), hv)


def build_fields(pair) -> PairFields:
    rho_f = sdf.sdf_grid(pair.fixed.samples, pair.fixed.grid, pair.params)
    rho_m = sdf.sdf_grid(pair.moving.samples, pair.moving.grid, pair.params)
    w_m = body_weights(pair.moving.grid)
    return PairFields(rho_f, rho_m, w_m, correlate.moving_coefficients(rho_m, w_m), pair.moving.grid.n[0],
                      pair.fixed.grid.n[2] == 1)


def score_rotation(fields: PairFields, quat):
    """-> (score, (tx, ty, tz), nbhd27, refined t) for one rotation."""
    vol = correlate.score_volume(fields.rho_f, fields.c, quat, fields.n_m, fields.planar)
    s, _, t = peak.peak(vol)
    nb = peak.neighbourhood(vol, t)
    return s, t, nb, peak.subvoxel(nb, t)


def score_rotations(fields: PairFields, quats):
    out = [score_rotation(fields, q) for q in np.asarray(quats).reshape(-1, 4)]
    scores = np.array([o[0] for o in out])
    ts = np.array([o[1] for o in out], dtype=np.int64)
    nbs = np.array([o[2] for o in out])
    refined = np.array([o[3] for o in out])
    return scores, ts, nbs, refined
