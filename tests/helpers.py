"""Shared test plumbing: oracle evaluation of whole pairs and comparison
helpers.  Nothing here computes the method itself; the oracle does."""

from __future__ import annotations

import numpy as np

from oracle import correlate as oc
from oracle import pipeline
from oracle import sdf as osdf


def flush_print(*a):
    print(*a, flush=True)


def oracle_fields(pair):
    return pipeline.build_fields(pair)


def body_weights(pair):
    return pipeline.body_weights(pair.moving.grid)


def sdf_compare(gpu_rho, samples, grid, params, rel_tol, band_rel, max_ambiguous_frac=0.01):
    """Compare a GPU SDF grid with the oracle node by node.

    Nodes where the oracle's own FP64 evaluation sits within ``band_rel`` of
    a discrete decision (a sample on the truncation sphere, the nearest sample
    nearly tied with an opposite-side one, the distance on the floor) may
    differ by the magnitude of the terms that decision moves; every other
    node must agree within rel_tol * max|rho|.  Returns a report dict."""
    pts = grid.node_positions()
    rho, diag = osdf.sdf_points(samples, pts, params, diagnostics=True, band_rel=band_rel)
    g = np.asarray(gpu_rho).reshape(-1)
    scale = np.abs(rho).max()
    err = np.abs(g - rho)
    tol = rel_tol * scale
    xi_abs = np.abs(diag["xi"])
    amb_trunc = diag["trunc_margin"] <= band_rel
    amb_pmc = diag["pmc_gap"] <= band_rel * np.maximum(xi_abs, 1.0)
    amb_floor = np.abs(xi_abs - params.xi_floor) <= band_rel * np.maximum(xi_abs, 1.0)
    allowed = np.where(amb_trunc, tol + 1.01 * diag["band_mag"], tol)
    free = amb_pmc | amb_floor
    bad = (err > allowed) & ~free
    return {"max_err": float(err.max()), "scale": float(scale), "n_bad": int(bad.sum()),
            "n_amb": int((amb_trunc | free).sum()), "n": len(rho),
            "ok": (not bad.any()) and (amb_trunc | free).mean() <= max_ambiguous_frac,
            "worst": int(np.argmax(np.where(free, 0, err - allowed)))}


def oracle_peaks(fields, quats):
    return pipeline.score_rotations(fields, quats)


def score_rel_err(s_gpu, s_ref):
    """Per-rotation relative error with a floor at 1e-3 of the largest score."""
    s_gpu = np.asarray(s_gpu, dtype=np.float64)
    s_ref = np.asarray(s_ref, dtype=np.float64)
    den = np.maximum(np.abs(s_ref), 1e-3 * np.abs(s_ref).max())
    return np.abs(s_gpu - s_ref) / den


def check_peak_identity(t_gpu, t_ref, s_gpu_at_ref_or_none=None):
    return np.all(np.asarray(t_gpu) == np.asarray(t_ref), axis=1)


def volume_at(vol, t):
    tx, ty, tz = (int(v) for v in t)
    return vol[tz, ty, tx]


def oracle_volume(fields, quat):
    return oc.score_volume(fields.rho_f, fields.c, quat, fields.n_m, fields.planar)
