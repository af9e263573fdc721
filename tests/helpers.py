"""Shared test plumbing: oracle evaluation of whole pairs and comparison
helpers.  Nothing here computes the method itself; the oracle does."""

from __future__ import annotations

import os

import numpy as np
import pytest

from oracle import correlate as oc
from oracle import pipeline
from oracle import sdf as osdf


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def load_peaks(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    a = np.loadtxt(path)
    return {"q": a[:, 1:5], "score": a[:, 5], "t": a[:, 6:9].astype(int), "refined": a[:, 9:12], "nbhd": a[:, 12:39]}


def check_against_golden(gold, s, t, refined, tag, tol=1e-4, refined_tol=1e-3):
    s = np.asarray(s, dtype=np.float64)
    ref = gold["score"]
    den = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    rel = np.abs(s - ref) / den
    flush_print(tag, "max rel err", rel.max(), "median", np.median(rel))
    assert rel.max() <= tol, (tag, int(np.argmax(rel)), rel.max())
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    n_tie = 0
    for r in range(len(s)):
        if np.array_equal(t[r], gold["t"][r]):
            continue
        d = tuple(int(v) for v in (t[r] - gold["t"][r]))
        assert d in offs, (tag, r, t[r], gold["t"][r])
        v = gold["nbhd"][r][offs.index(d)]
        assert abs(v - ref[r]) <= tol * den[r], (tag, r, v, ref[r])
        n_tie += 1
    flush_print(tag, "near-tie translations", n_tie, "of", len(s))
    if refined is not None:
        # FP64 sub-voxel refinement at the rotations whose integer peak matches
        same = np.all(np.asarray(t) == gold["t"], axis=1)
        d_ref = np.abs(np.asarray(refined, dtype=np.float64)[same] - gold["refined"][same]).max()
        flush_print(tag, "refined t max abs diff", d_ref, "over", int(same.sum()), "rotations")
        assert d_ref <= refined_tol, (tag, d_ref)
    b_gpu, b_ref = int(np.argmax(s)), int(np.argmax(ref))
    assert b_gpu == b_ref or abs(ref[b_gpu] - ref[b_ref]) <= tol * abs(ref[b_ref]), (tag, b_gpu, b_ref)
