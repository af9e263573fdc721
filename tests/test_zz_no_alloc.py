"""The allocation-free pose-gradient entry point (score_grad_noalloc), through
the C ABI, against score_grad on the same inputs: two calls in a row, the
second smaller, in both precisions, and the size limit."""

import numpy as np
import pytest

from helpers import flush_print
from workloads import configs as C
from workloads import rotations as wr

pytestmark = pytest.mark.gpu


def case(n, nm, planar, B, seed):
    rng = np.random.default_rng(seed)
    if planar:
        gf, gm = C.GridSpec((n, n, 1), (0, 0, 0), 1.0), C.GridSpec((nm, nm, 1), (0, 0, 0), 1.0)
        sf, sm = (1, n, n), (1, nm, nm)
        q = wr.planar_rotations(360.0 / B, B)
    else:
        gf, gm = C.GridSpec((n, n, n), (0, 0, 0), 1.0), C.GridSpec((nm, nm, nm), (0, 0, 0), 1.0)
        sf, sm = (n, n, n), (nm, nm, nm)
        q = wr.uniform_quaternions(B, seed + 1)
    rho_f = rng.normal(size=sf) + 1j * rng.normal(size=sf)
    rho_m = rng.normal(size=sm) + 1j * rng.normal(size=sm)
    w = rng.uniform(0.5, 1.5, size=sm)
    t = rng.uniform(0, n, size=(B, 3))
    if planar:
        t[:, 2] = 0.0
    return gf, gm, rho_f, rho_m, w, np.concatenate([t, q], axis=1)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_matches_score_grad_twice(dtype):
    import torch
    from paper_1712_00238_amd.api import Context
    tol = 2e-6 if dtype == "f32" else 1e-12
    with Context(0, dtype) as ctx:
        # first call the larger problem, then a smaller one (fewer poses, smaller box, planar in FP64)
        cases = [(64, 24, False, 200, 5, True), (64, 16, dtype == "f64", 37, 6, False)]
        for n, nm, planar, B, seed, want_w in cases:
            gf, gm, rho_f, rho_m, w, poses = case(n, nm, planar, B, seed)
            flush_print("score_grad_noalloc", dtype, n, nm, planar, B, want_w)
            rf, rm = ctx._dev(rho_f, ctx.cplx), ctx._dev(rho_m, ctx.cplx)
            wm, pd = ctx._dev(w, ctx.real), ctx._dev(poses, torch.float64)
            scale = ctx._dev(np.linspace(0.5, 1.5, B), torch.float64)
            ref_s, ref_g, ref_w = ctx.score_grad(rf, gf, rm, wm, gm, pd, want_pose=True, want_w=want_w,
                                                 grad_scale=scale)
            score = torch.full((B,), float("nan"), dtype=ctx.real, device=ctx.device)
            gpose = torch.full((B, 7), float("nan"), dtype=torch.float64, device=ctx.device)
            gw = torch.full(wm.shape, float("nan"), dtype=ctx.real, device=ctx.device) if want_w else None
            ctx.score_grad_noalloc(rf, gf, rm, wm, gm, pd, score, gpose, gw, scale)
            torch.cuda.synchronize()
            for got, ref in ((score, ref_s), (gpose, ref_g), (gw, ref_w)):
                if ref is None:
                    continue
                got, ref = got.cpu().numpy().astype(np.float64), ref.cpu().numpy().astype(np.float64)
                assert np.all(np.isfinite(got))
                assert np.max(np.abs(got - ref)) <= tol * max(1.0, np.abs(ref).max())


def test_noalloc_rejects_problems_beyond_its_scratch():
    import torch
    from paper_1712_00238_amd._lib import SDF_ENOMEM, SdfError
    from paper_1712_00238_amd.api import Context
    with Context(0, "f32") as ctx:
        n, nm, B = 128, 64, 2048  # 2048 poses of a 64^3 box with weight sums: about 185 MiB
        gf, gm = C.GridSpec((n, n, n), (0, 0, 0), 1.0), C.GridSpec((nm, nm, nm), (0, 0, 0), 1.0)
        rf = torch.zeros((n, n, n), dtype=torch.complex64, device=ctx.device)
        rm = torch.zeros((nm, nm, nm), dtype=torch.complex64, device=ctx.device)
        wm = torch.ones((nm, nm, nm), dtype=torch.float32, device=ctx.device)
        poses = torch.zeros((B, 7), dtype=torch.float64, device=ctx.device)
        poses[:, 3] = 1.0
        score = torch.full((B,), 7.0, dtype=torch.float32, device=ctx.device)
        gw = torch.full(wm.shape, 7.0, dtype=torch.float32, device=ctx.device)
        with pytest.raises(SdfError) as ei:
            ctx.score_grad_noalloc(rf, gf, rm, wm, gm, poses, score, None, gw)
        assert ei.value.code == SDF_ENOMEM and "scratch" in str(ei.value)
        torch.cuda.synchronize()
        assert bool((score == 7.0).all()) and bool((gw == 7.0).all())  # nothing was enqueued
