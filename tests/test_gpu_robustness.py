"""Failure and caching behaviour of the library, through the C ABI: the
workspace cap, graph capture and re-capture, and the autotuner's parity
probe rejecting a candidate.  Every condition is forced from the host; every
kernel runs to completion."""

import numpy as np
import pytest

from helpers import flush_print
from oracle import correlate as oc
from oracle import peak as op
from workloads import configs as C
from workloads import rotations as wr

pytestmark = pytest.mark.gpu


def rand_case(n, nm, seed):
    rng = np.random.default_rng(seed)
    gf = C.GridSpec((n, n, n), (0, 0, 0), 1.0)
    gm = C.GridSpec((nm, nm, nm), (0, 0, 0), 1.0)
    rho_f = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    rho_m = rng.normal(size=(nm, nm, nm)) + 1j * rng.normal(size=(nm, nm, nm))
    return gf, gm, rho_f, rho_m, rng.uniform(0.5, 1.5, size=(nm, nm, nm))


def test_workspace_cap_gives_enomem_and_leaves_inputs_untouched():
    import torch
    from paper_1712_00238_amd._lib import SDF_ENOMEM, SdfError
    from paper_1712_00238_amd.api import Context
    gf, gm, rho_f, rho_m, w = rand_case(64, 24, 1)
    with Context(0, "f32") as big:
        spec = big.spectrum(rho_f, gf)
    with Context(0, "f32", workspace_cap=1 << 20) as ctx:
        rm = torch.as_tensor(rho_m, dtype=torch.complex64, device="cuda")
        wt = torch.as_tensor(w, dtype=torch.float32, device="cuda")
        before = [t.clone() for t in (spec, rm, wt)]
        flush_print("workspace cap 1 MiB, search at 64^3")
        with pytest.raises(SdfError) as ei:
            ctx.score_rotations(spec, gf, rm, wt, gm, wr.uniform_quaternions(4, 2))
        assert ei.value.code == SDF_ENOMEM and "cap" in str(ei.value)
        # a build whose Morton workspace exceeds the cap fails the same way
        s = np.random.default_rng(2).normal(size=(40000, 3))
        nrm = s / np.linalg.norm(s, axis=1, keepdims=True)
        with pytest.raises(SdfError) as ei:
            ctx.sdf_build(s * 5, nrm, np.ones(40000), C.GridSpec((8, 8, 8), (-4, -4, -4), 1.0), C.SDFParams())
        assert ei.value.code == SDF_ENOMEM
        torch.cuda.synchronize()
        for a, b in zip(before, (spec, rm, wt)):
            assert torch.equal(a, b)
        # small work still fits under the cap afterwards
        g8 = C.GridSpec((8, 8, 8), (-3.5, -3.5, -3.5), 1.0)
        ctx.sdf_build(s[:50] * 2, nrm[:50], np.ones(50), g8, C.SDFParams(xi_floor=0.25))
        torch.cuda.synchronize()


def test_graph_captured_once_per_shape_and_replays_match_eager():
    """With "graph" = 1 the search is captured on its first call and replayed
    while buffers and shapes stay; a call with another rotation count is
    captured anew (one graph is cached, so returning to the first shape
    captures again).  Every replay, with eager work in between, equals the
    eager result bit for bit."""
    import torch
    from paper_1712_00238_amd.api import Context
    gf, gm, rho_f, rho_m, w = rand_case(32, 14, 3)
    qa, qb = wr.uniform_quaternions(6, 4), wr.uniform_quaternions(4, 5)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream), Context(0, "f32") as ctx:
        spec = ctx.spectrum(rho_f, gf)
        ctx.set_option("graph", 0)
        ref_a = ctx.score_rotations(spec, gf, rho_m, w, gm, qa)
        ref_b = ctx.score_rotations(spec, gf, rho_m, w, gm, qb)
        ctx.set_option("graph", 1)
        c0 = ctx.get_option("graph_captures")
        out_a = None
        seen = []
        for it in range(3):
            out_a = ctx.score_rotations(spec, gf, rho_m, w, gm, qa, out=out_a)
            seen.append(ctx.get_option("graph_captures") - c0)
            torch.cuda.synchronize()
            for k in ("score", "t", "nbhd", "refined"):
                assert torch.equal(out_a[k], ref_a[k]), (it, k)
            junk = torch.randn(1 << 20, device="cuda") * 2  # eager work between replays
            del junk
            out_a["score"].zero_()
        assert seen == [1, 1, 1]
        out_b = ctx.score_rotations(spec, gf, rho_m, w, gm, qb)
        assert ctx.get_option("graph_captures") - c0 == 2
        torch.cuda.synchronize()
        assert torch.equal(out_b["score"], ref_b["score"]) and torch.equal(out_b["t"], ref_b["t"])
        ctx.score_rotations(spec, gf, rho_m, w, gm, qa, out=out_a)
        assert ctx.get_option("graph_captures") - c0 == 3
        torch.cuda.synchronize()
        assert torch.equal(out_a["score"], ref_a["score"])
    # the eager reference itself against the oracle
    c = oc.moving_coefficients(rho_m, w)
    for r, q in enumerate(qa):
        vol = oc.score_volume(rho_f, c, q, 14, False)
        assert abs(float(ref_a["score"][r]) - vol.max()) <= 2e-5 * np.abs(vol).max()


def test_autotune_skips_a_candidate_that_fails_its_probe():
    """The "autotune_reject" option makes the probe fail for chosen candidates:
    the tuner then reports them without parity and picks another plan; with
    every candidate rejected it fails cleanly and the search still runs."""
    from paper_1712_00238_amd._lib import SdfError
    from paper_1712_00238_amd.api import Context
    gf, gm, rho_f, rho_m, w = rand_case(32, 14, 9)
    with Context(0, "f32") as ctx:
        flush_print("autotune 32^3 / 14^3 twice")
        rep = ctx.autotune(gf, gm)
        cands = rep["candidates"]
        key = lambda c: (c["batch"], c["group"], c["radix"])
        first = key(rep["chosen"])
        idx = [key(c) for c in cands].index(first)
        ctx.set_option("autotune_reject", 1 << idx)
        rep2 = ctx.autotune(gf, gm)
        assert not rep2["candidates"][idx]["parity"]
        assert key(rep2["chosen"]) != first
        assert all(c["parity"] for i, c in enumerate(rep2["candidates"]) if i != idx)
        ctx.set_option("autotune_reject", (1 << len(cands)) - 1)
        with pytest.raises(SdfError, match="no candidate"):
            ctx.autotune(gf, gm)
        ctx.set_option("autotune_reject", 0)
        quats = wr.uniform_quaternions(5, 6)
        out = ctx.score_rotations(ctx.spectrum(rho_f, gf), gf, rho_m, w, gm, quats)
        c = oc.moving_coefficients(rho_m, w)
        for r, q in enumerate(quats):
            vol = oc.score_volume(rho_f, c, q, 14, False)
            assert abs(float(out["score"][r]) - vol.max()) <= 2e-5 * np.abs(vol).max()
