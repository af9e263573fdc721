#!/usr/bin/env python
"""Benchmark of the scoring hot path on one MI355X.

Workload (default): the 3D mechanical pair - a 60 x 60 x 30 box with a
cylindrical hole (fixed) and a 30 x 30 x 10 plate with a cylindrical peg
(moving), surfaces sampled at 1 point per unit area, fixed grid 128^3 at unit
spacing, moving body box 64^3, 576 rotations of the level-1 Hopf grid, FP32.

A step is one score_rotations call over all 576 rotations (rotation matrices
in FP64, fused spread + 3D FFT + spectral product + inverse FFT + peak,
27-neighbourhood, FP64 sub-voxel refinement), inputs resident in HBM.  The
one-time SDF construction and spectrum, the plain FP64 path, pose-gradient
evaluations and per-kernel roofline figures are measured around it and
reported in the same JSON line, as are the reference search without the
spreading window (the top rotations rescored), the same rotations through
octree-adaptive samples and the nonequispaced transform, shape gradients,
the protein-like pair, gradient refinement and a queue of uneven pairs.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1712_00238_amd/csrc/kernels_fused.hip", "paper_1712_00238_amd/csrc/fft.hpp",
                  "paper_1712_00238_amd/csrc/common.hpp"]


def sources_sha() -> str:
    """Hash of the kernel sources' code: line comments and blank space are
    dropped first, so an edit of a comment keeps the stored counters valid
    while any change to the code itself invalidates them."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            for line in f:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=64, help="rotations per fused launch sequence")
    ap.add_argument("--pencil-group", type=int, default=2)
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--autotune", type=int, default=1, help="tune batch, pencil group and radix schedule first")
    ap.add_argument("--fp64-rotations", type=int, default=64, help="rotations timed on the plain FP64 path")
    ap.add_argument("--direct-rotations", type=int, default=32,
                    help="top rotations rescored by the windowless reference search")
    ap.add_argument("--nfft-rotations", type=int, default=32,
                    help="of the directly rescored rotations, how many the nonequispaced route scores (0: skip)")
    ap.add_argument("--nfft-width", type=int, default=6, help="ES kernel width of the nonequispaced route")
    ap.add_argument("--nfft-tols", default="0,0.003,0.01,0.03", help="octree tolerances (0: every node)")
    ap.add_argument("--grad-poses", type=int, default=1024)
    ap.add_argument("--refine-poses", type=int, default=1024,
                    help="protein-like refinement: poses perturbed from the top peaks (0 skips)")
    ap.add_argument("--refine-steps", type=int, default=50)
    ap.add_argument("--refine-lr", type=float, default=0.05)
    ap.add_argument("--grad-steps", type=int, default=5)
    ap.add_argument("--cpu-rotations", type=int, default=2,
                    help="oracle rotations per host worker in the CPU baseline")
    ap.add_argument("--protein-rotations", type=int, default=3600,
                    help="rotations of the protein-like pair scored 64 per launch (0: skip)")
    ap.add_argument("--uneven-pairs", type=int, default=256,
                    help="pairs in the multi-pair queue figure, 512 rotations each (0: skip)")
    ap.add_argument("--uneven-e2e", type=int, default=1,
                    help="also run the uneven batch end to end on its own pairs with per-pair SDF builds (0: skip)")
    ap.add_argument("--phi-kernels", type=int, default=1,
                    help="compare the alternative kernels of eq. 13 on the planar and mechanical pairs (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["bench", "copy"], default="bench",
                    help="copy: launch one device copy of known size (counter calibration)")
    return ap.parse_args()


def copy_mode():
    import torch
    n = 256 * 1024 * 1024 // 4  # 256 MiB of floats read, 256 MiB written
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))


def reach_fraction(quats, n_m: int, N: int) -> float:
    """Mean fraction of the N slab heights that a rotated n_m^3 body box and
    its B-spline support can reach (the bound the rotation descriptors carry):
    the other slabs are identically zero and are neither written nor read."""
    import numpy as np
    q = np.asarray(quats, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    row_z = np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], axis=1)
    a = -row_z
    lo, hi = -0.5 * n_m, 0.5 * n_m - 1.0
    zmin = np.minimum(a * lo, a * hi).sum(axis=1)
    zmax = np.maximum(a * lo, a * hi).sum(axis=1)
    zl = np.maximum(np.floor(zmin - 2.0 - 1e-3), -N // 2)
    zh = np.minimum(np.ceil(zmax + 2.0 + 1e-3), N // 2 - 1)
    return float(np.mean(zh - zl + 1) / N)


def algorithmic_bytes(kernel: str, nb: int, N: int, n_m: int, planar: bool, reach: float = 1.0) -> float:
    """Bytes a kernel must move per launch of nb rotations (complex64 = 8 B):
    spread_slab reads each rotation's coefficients once and writes the slabs
    its body box reaches (fraction `reach`); pencil reads those slabs, the
    spectrum once, and writes the folded grid of each rotation pair;
    islab_peak reads the folded grids."""
    nz = 1 if planar else N
    G = N * N * nz
    K = n_m * n_m * (1 if planar else n_m)
    pairs = (nb + 1) // 2
    if kernel == "spread_slab":
        return nb * (8.0 * K + 8.0 * G * reach)
    if kernel == "pencil":
        return nb * 8.0 * G * reach + 8.0 * G + pairs * 8.0 * G
    if kernel == "islab_peak":
        return pairs * 8.0 * G
    if kernel == "finish":
        return nb * 3 * 8.0 * N * N
    if kernel == "finish_rot":
        return nb * (27 * 8.0 + 27 * 4.0 + 3 * 8.0)
    raise KeyError(kernel)


def load_traffic(kernel: str, sha: str, rotations: int):
    """HBM bytes of one launch of `kernel` over `rotations` rotations, from the
    counter summary under profiles/ (FETCH_SIZE + WRITE_SIZE per rotation,
    calibrated against a plain copy); None when the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    k = rec.get("kernels", {}).get(kernel)
    if not k or rec.get("source_sha") != sha:
        return None
    return k["hbm_bytes_per_rotation"] * rotations


def _oracle_rotations(args):
    """Worker: score rotations qs with the oracle on seeded fields (fork)."""
    import numpy as np

    from oracle import correlate as oc
    from oracle import peak as op

    qs, n, nm = args
    rng = np.random.default_rng(0)
    rho_f = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    c = rng.normal(size=nm ** 3) + 1j * rng.normal(size=nm ** 3)
    t0 = time.perf_counter()
    for q in qs:
        vol = oc.score_volume(rho_f, c, q, nm, False)
        _, _, t = op.peak(vol)
        op.subvoxel(op.neighbourhood(vol, t), t)
    return time.perf_counter() - t0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pair, per_worker: int):
    """The FP64 oracle's per-rotation scoring on the host (spread, numpy FFT
    pair, peak, sub-voxel) on seeded random complex fields of the workload's
    shapes (values do not change the work): rotation-parallel over the cores
    this process may use (at most 16), `per_worker` rotations per worker,
    plus one worker alone for the single-core rate."""
    import concurrent.futures as cf
    import multiprocessing as mp

    n = pair.fixed.grid.n[0]
    nm = pair.moving.grid.n[0]
    avail = len(os.sched_getaffinity(0))
    workers = max(1, min(16, avail))
    qs = pair.quats
    t0 = time.perf_counter()
    single = _oracle_rotations((qs[:per_worker], n, nm))
    single_rate = per_worker / single
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        chunks = [(qs[(i * per_worker) % len(qs):][:per_worker], n, nm) for i in range(workers)]
        list(ex.map(_oracle_rotations, chunks))
    wall = time.perf_counter() - t0
    total = workers * per_worker
    return {"value": total / wall, "unit": "rotations/s", "cores": workers, "kind": "oracle",
            "sample": f"{total} of {len(qs)} rotations at {n}^3 / {nm}^3 (FP64 spread, numpy FFT pair, peak, "
                      f"sub-voxel), {workers} processes x {per_worker} rotations, {wall:.1f} s wall; "
                      f"host: {cpu_model()}, {avail} cores available",
            "single_core_value": single_rate}


def cpu_extras(pair):
    """Oracle SDF build pairs/s (C, OpenMP) and pose-gradient evaluations/s
    (numpy, one process) on bounded samples of the workload."""
    import numpy as np

    from oracle import grad as og
    from oracle import sdf as osdf
    from oracle import spread as osp

    fx = pair.fixed
    rng = np.random.default_rng(1)
    nodes = fx.grid.node_positions()[rng.choice(fx.grid.size, size=20000, replace=False)]
    t0 = time.perf_counter()
    osdf.sdf_points(fx.samples, nodes, pair.params)
    dt = time.perf_counter() - t0
    pairs_per_s = len(nodes) * fx.samples.count / dt
    n, nm = fx.grid.n[0], pair.moving.grid.n[0]
    rho_f = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    rho_m = rng.normal(size=(nm, nm, nm)) + 1j * rng.normal(size=(nm, nm, nm))
    c = rho_m.reshape(-1)
    xb = osp.body_positions(nm)
    t0 = time.perf_counter()
    for b in range(2):
        og.pose_value_and_grad(rho_f, c, rho_m, xb, np.array([3.3, -2.1, 0.7]) * (b + 1), pair.quats[b])
    g = 2 / (time.perf_counter() - t0)
    return {"sdf_build_pairs_per_s": pairs_per_s, "sdf_build_threads": int(os.environ.get("OMP_NUM_THREADS", "0")) or
            len(os.sched_getaffinity(0)), "sdf_sample": f"20000 nodes x {fx.samples.count} samples",
            "grad_evals_per_s": g, "grad_sample": "2 poses, one process"}


def volume_shape(vol):
    """Support (fraction of translations with |f| > 1e-3 max |f|) and the
    largest step between neighbouring translations relative to the peak, of
    one rotation's score volume (the shape the Validation section compares)."""
    import numpy as np
    v = np.asarray(vol, dtype=np.float64)
    peak = float(v.max())
    steps = [np.abs(np.roll(v, -1, axis=a) - v).max() for a in range(v.ndim) if v.shape[a] > 1]
    return {"support": round(float((np.abs(v) > 1e-3 * np.abs(v).max()).mean()), 4),
            "max_step_over_peak": round(float(max(steps)) / peak, 4) if peak > 0 else None}


PHI_KERNELS = (("skeletal", 0.0), ("inverse_square", 0.0), ("dsl", 2.0), ("radial", 2.0))


def phi_kernel_section(dev):
    """Alternative kernels of eq. 13 on the planar peg-in-hole pair (FP64) and
    the mechanical pair (FP32): each part's affinity built on the GPU with
    the kernel, every rotation searched, and the best pose's score volume."""
    import numpy as np
    import torch

    from paper_1712_00238_amd.api import Context
    from workloads import configs as C

    out = {}
    for name, pair, dtype in (("peg_in_hole_2d", C.peg_in_hole_2d(seed=0), "f64"),
                              ("mechanical_3d", C.mechanical_3d(seed=0), "f32")):
        fx, mv = pair.fixed, pair.moving
        rows = []
        with Context(0, dtype) as c:
            for kind, R in PHI_KERNELS:
                c.sdf_build(mv.samples.q, mv.samples.n, mv.samples.w, mv.grid, pair.params, phi=kind, radius=R)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rf = c.sdf_build(fx.samples.q, fx.samples.n, fx.samples.w, fx.grid, pair.params, phi=kind, radius=R)
                torch.cuda.synchronize()
                build_ms = 1e3 * (time.perf_counter() - t0)
                rm = c.sdf_build(mv.samples.q, mv.samples.n, mv.samples.w, mv.grid, pair.params, phi=kind, radius=R)
                spec = c.spectrum(rf, fx.grid)
                w = torch.ones(rm.shape, dtype=c.real, device=dev)
                o = c.score_rotations(spec, fx.grid, rm, w, mv.grid, pair.quats)
                s = o["score"].cpu().numpy().astype(np.float64)
                b = int(np.argmax(s))
                t = [int(v) for v in o["t"][b].cpu().numpy()]
                vol = c.score_volume(spec, fx.grid, rm, w, mv.grid, pair.quats[b:b + 1])[0].cpu().numpy()
                row = {"kernel": kind, "radius": R or None, "fixed_build_ms": round(build_ms, 2),
                       "best_rotation": b, "best_t": t, "best_score": float(s[b])}
                if name == "peg_in_hole_2d":
                    row["seated"] = (b, t[:2]) in ((0, [64, 84]), (18, [63, 83]))
                row.update(volume_shape(vol))
                rows.append(row)
                del rf, rm, spec, w, o
        out[name] = rows
    return out


def sdf_build_counts(ctx, part, params, build_ms):
    """Node-sample pairs of one sdf_build, counted by the library's counting
    variant (a separate, untimed build): pass 1 (nearest sample), pass 2
    (kernel sum, samples of the visited tiles) and pairs inside the contact
    ball, with their rates over the timed build."""
    import torch
    ctx.set_option("sdf_stats", 1)
    ctx.sdf_build(part.samples.q, part.samples.n, part.samples.w, part.grid, params)
    torch.cuda.synchronize()
    c = {k: ctx.get_option("sdf_pairs_" + k) for k in ("nearest", "sum", "in_ball")}
    ctx.set_option("sdf_stats", 0)
    dense = float(part.samples.count) * part.grid.size
    sec = build_ms * 1e-3
    # VALU issue bound: the FP32 kernel's inner loops issue about 8 VALU
    # instructions per pass-1 pair (FP64 distance and compares), 9 per pass-2
    # pair (distance and ball test) and 18 more per pair inside the ball; the
    # chip issues 256 CUs x 64 lanes x 2.4 GHz lane instructions per second
    lanes_per_s = 256 * 64 * 2.4e9
    bound_ms = 1e3 * (8.0 * c["nearest"] + 9.0 * c["sum"] + 18.0 * c["in_ball"]) / lanes_per_s
    return {"build_ms": round(build_ms, 3), "samples": part.samples.count, "nodes": part.grid.size,
            "pairs_nearest": c["nearest"], "pairs_sum": c["sum"], "pairs_in_ball": c["in_ball"],
            "frac_of_dense": {k: round(v / dense, 4) for k, v in c.items()},
            "in_ball_pairs_per_s": c["in_ball"] / sec, "sum_pairs_per_s": c["sum"] / sec,
            "nearest_pairs_per_s": c["nearest"] / sec,
            "valu_bound_ms": round(bound_ms, 3), "frac_of_valu_bound": round(bound_ms / build_ms, 3)}


def uneven_end_to_end(ctx, dev, n_pairs, workers):
    """The uneven batch end to end: its own seeded pairs (sampled on the host
    by a process pool, outside the timing), then on the GPU both SDFs of every
    pair, the fixed spectra and one score_pairs queue of all pairs x 512
    rotations, timed with events on the current stream."""
    import torch

    from workloads import configs as C
    t0 = time.perf_counter()
    pairs = C.uneven_batch(n_pairs, 512, workers)
    gen_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream(dev)

    def run(sub):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        jobs = []
        for p in sub:
            fx, mv = p.fixed, p.moving
            rf = ctx.sdf_build(fx.samples.q, fx.samples.n, fx.samples.w, fx.grid, p.params)
            rm = ctx.sdf_build(mv.samples.q, mv.samples.n, mv.samples.w, mv.grid, p.params)
            jobs.append({"spec": ctx.spectrum(rf, fx.grid), "g_fixed": fx.grid, "rho_moving": rm,
                         "w_moving": torch.ones(rm.shape, dtype=torch.float32, device=dev), "g_moving": mv.grid,
                         "quats": p.quats})
            del rf
        ev[1].record(stream)
        ctx.score_pairs(jobs)
        ev[2].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])

    # warm-up on one pair of each grid class (workspace, autotuned plans)
    seen, warm = set(), []
    for p in pairs:
        if p.n_fixed not in seen:
            seen.add(p.n_fixed)
            warm.append(p)
    run(warm)
    build_ms, search_ms = run(pairs)
    rots = 512 * len(pairs)
    classes = {}
    for p in pairs:
        k = f"{p.n_fixed}^3/{p.n_moving}^3"
        classes[k] = classes.get(k, 0) + 1
    return {"pairs": len(pairs), "rotations": rots, "classes": classes,
            "samples_total": int(sum(p.fixed.samples.count + p.moving.samples.count for p in pairs)),
            "host_sampling_s": round(gen_s, 2), "host_workers": workers,
            "sdf_and_spectrum_ms": round(build_ms, 2), "search_ms": round(search_ms, 2),
            "end_to_end_ms": round(build_ms + search_ms, 2),
            "sdf_share": round(build_ms / (build_ms + search_ms), 4),
            "search_rotations_per_s": round(rots / (search_ms * 1e-3), 1),
            "end_to_end_rotations_per_s": round(rots / ((build_ms + search_ms) * 1e-3), 1)}


def copy_bandwidth(dev) -> float:
    """Device-to-device copy of 1 GiB, read + write bytes per second."""
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / 5
    del a, b
    return 2.0 * n * 4 / sec


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: every box here has one GPU and the multi-GPU path is a design "
              "note only (rotations shard across GPUs with a final top-k merge).", file=sys.stderr)
        sys.exit(2)
    if args.mode == "copy":
        copy_mode()
        return
    import numpy as np
    import torch

    from paper_1712_00238_amd.api import Context
    from paper_1712_00238_amd.autograd import sdf_score
    from workloads import configs as C
    from workloads import rotations as wr

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    pair = C.mechanical_3d(seed=0)
    fx, mv = pair.fixed, pair.moving
    N, n_m = fx.grid.n[0], mv.grid.n[0]
    n_rot = len(pair.quats)
    report = {}

    def ev():
        return torch.cuda.Event(enable_timing=True)

    with torch.cuda.stream(stream):
        ctx = Context(0, "f32")
        ctx.set_option("batch", args.batch)
        ctx.set_option("pencil_group", args.pencil_group)
        ctx.set_option("graph", args.graph)
        # --- a1 / a2 (one-time per pair), timed with events on this stream
        rho_m = ctx.sdf_build(mv.samples.q, mv.samples.n, mv.samples.w, mv.grid, pair.params)
        e0, e1 = ev(), ev()
        e0.record(stream)
        rho_f = ctx.sdf_build(fx.samples.q, fx.samples.n, fx.samples.w, fx.grid, pair.params)
        e1.record(stream)
        e2, e3 = ev(), ev()
        e2.record(stream)
        spec = ctx.spectrum(rho_f, fx.grid)
        e3.record(stream)
        torch.cuda.synchronize()
        report["sdf_build_fixed_ms"] = e0.elapsed_time(e1)
        report["sdf_build_fixed"] = sdf_build_counts(ctx, fx, pair.params, e0.elapsed_time(e1))
        report["spectrum_ms"] = e2.elapsed_time(e3)
        w = torch.ones(rho_m.shape, dtype=torch.float32, device=dev)  # h^3 = 1
        tuned = None
        if args.autotune:
            rep = ctx.autotune(fx.grid, mv.grid)
            tuned = rep["chosen"]
            args.batch, args.pencil_group = tuned["batch"], tuned["group"]

        out = None
        for _ in range(args.warmup):
            out = ctx.score_rotations(spec, fx.grid, rho_m, w, mv.grid, pair.quats, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = ctx.score_rotations(spec, fx.grid, rho_m, w, mv.grid, pair.quats, out=out)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        ms_per_step = elapsed * 1e3 / args.steps
        value = n_rot / (ms_per_step * 1e-3)
        report["graph_launches"] = ctx.get_option("graph_launches")
        s32 = out["score"].cpu().numpy().astype(np.float64)
        t32 = out["t"].cpu().numpy()

        # --- per-kernel durations with HIP events on this stream
        ctx.set_option("profile", 1)
        ctx.reset_stats()
        prof_steps = 3
        for _ in range(prof_steps):
            ctx.score_rotations(spec, fx.grid, rho_m, w, mv.grid, pair.quats, out=out)
        torch.cuda.synchronize()
        kernels = {}
        for k in ("spread_slab", "pencil", "islab_peak", "finish", "finish_rot"):
            ms, launches = ctx.kernel_stats(k)
            kernels[k] = {"avg_us": 1e3 * ms / max(launches, 1), "launches": launches,
                          "share": 0.0}
        ctx.set_option("profile", 0)
        tot = sum(v["avg_us"] * v["launches"] for v in kernels.values())
        # one call spreads its rotations evenly over ceil(n_rot / batch) launches
        # (even sizes, the last one takes the rest): bytes and durations are both
        # averaged over those launches
        n_launch = -(-n_rot // args.batch)
        per = min(args.batch, (-(-n_rot // n_launch) + 1) // 2 * 2) if n_launch > 1 else args.batch
        sizes = [min(per, n_rot - i) for i in range(0, n_rot, per)]
        rot_per_launch = n_rot / len(sizes)
        reach = reach_fraction(pair.quats, n_m, N)
        report["slab_reach"] = round(reach, 4)
        for k, v in kernels.items():
            v["share"] = v["avg_us"] * v["launches"] / tot
            v["algorithmic_bytes_per_launch"] = sum(algorithmic_bytes(k, nb, N, n_m, False, reach)
                                                    for nb in sizes) / len(sizes)
            v["achieved_GBs"] = v["algorithmic_bytes_per_launch"] / (v["avg_us"] * 1e-6) / 1e9
        dom = max(kernels, key=lambda k: kernels[k]["share"])
        sha = sources_sha()
        traffic = load_traffic(dom, sha, rot_per_launch)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(kernels[dom]["achieved_GBs"], 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(kernels[dom]["achieved_GBs"] / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "avg_launch_us": round(kernels[dom]["avg_us"], 2),
                    "algorithmic_bytes_per_launch": kernels[dom]["algorithmic_bytes_per_launch"],
                    "source_sha": sha}
        # whole correlation stage (all four kernels of a batch) against HBM
        stage_bytes = sum(v["algorithmic_bytes_per_launch"] for v in kernels.values())
        stage_us = sum(v["avg_us"] for v in kernels.values())
        report["stage_GBs"] = stage_bytes / (stage_us * 1e-6) / 1e9
        # whole correlation stage per rotation (spread, FFTs, product, peak) over the
        # timed calls, against the model of a minimal three-pass design (slab R + W,
        # pencil R + spectrum R + W, inverse slab R: 6 N^3 x 8 B), against the HBM
        # bytes the counters measured, and against a measured device copy
        sec_per_rot = ms_per_step * 1e-3 / n_rot
        model = 6.0 * N ** 3 * 8.0
        tr = [load_traffic(k, sha, 1.0) for k in ("spread_slab", "pencil", "islab_peak", "finish")]
        counter = sum(tr) if all(v is not None for v in tr) else None
        copy_bps = copy_bandwidth(dev)
        report["correlation_stage"] = {
            "model_bytes_per_rotation": model,
            "achieved_model_GBs": round(model / sec_per_rot / 1e9, 1),
            "frac_model": round(model / sec_per_rot / (HBM_PEAK_GBS * 1e9), 4),
            "counter_bytes_per_rotation": counter,
            "achieved_counter_GBs": None if counter is None else round(counter / sec_per_rot / 1e9, 1),
            "frac_counter": None if counter is None else round(counter / sec_per_rot / (HBM_PEAK_GBS * 1e9), 4),
            "copy_GBs": round(copy_bps / 1e9, 1),
            "frac_model_of_copy": round(model / sec_per_rot / copy_bps, 4)}
        report["kernels"] = {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                             for k, v in kernels.items()}

        # --- plain FP64 path on the same workload (SDFs, spectrum and search in FP64)
        ctx64 = Context(0, "f64")
        rho_m64 = ctx64.sdf_build(mv.samples.q, mv.samples.n, mv.samples.w, mv.grid, pair.params)
        rho_f64 = ctx64.sdf_build(fx.samples.q, fx.samples.n, fx.samples.w, fx.grid, pair.params)
        spec64 = ctx64.spectrum(rho_f64, fx.grid)
        w64 = torch.ones(rho_m64.shape, dtype=torch.float64, device=dev)
        q64 = pair.quats[:args.fp64_rotations]
        ctx64.score_rotations(spec64, fx.grid, rho_m64, w64, mv.grid, q64[:2])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o64 = ctx64.score_rotations(spec64, fx.grid, rho_m64, w64, mv.grid, q64)
        torch.cuda.synchronize()
        fp64_rps = len(q64) / (time.perf_counter() - t0)
        s64 = o64["score"].cpu().numpy()
        t64 = o64["t"].cpu().numpy()
        k = len(q64)
        den = np.maximum(np.abs(s64), 1e-3 * np.abs(s64).max())
        rel = np.abs(s32[:k] - s64) / den
        report["fp64_rotations_per_s"] = fp64_rps
        report["fp32_vs_fp64"] = {"rotations": int(k), "max_rel_err": float(rel.max()),
                                  "median_rel_err": float(np.median(rel)),
                                  "same_t_frac": float(np.mean(np.all(t32[:k] == t64, axis=1))),
                                  "same_best": bool(int(np.argmax(s32[:k])) == int(np.argmax(s64)))}

        # --- what the spreading window changes: the top rotations rescored by the
        # reference search that builds the turned part's SDF on the body box and
        # places it without a window (same FP32 context and spectrum)
        if args.direct_rotations:
            top = np.argsort(-s32, kind="stable")[:args.direct_rotations]
            qd = pair.quats[top]
            ctx.score_rotations_direct(spec, fx.grid, mv.samples.q, mv.samples.n, mv.samples.w, mv.grid,
                                       pair.params, qd[:1])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            od_ = ctx.score_rotations_direct(spec, fx.grid, mv.samples.q, mv.samples.n, mv.samples.w, mv.grid,
                                             pair.params, qd)
            torch.cuda.synchronize()
            d_rps = len(qd) / (time.perf_counter() - t0)
            sd = od_["score"].cpu().numpy().astype(np.float64)
            td = od_["t"].cpu().numpy()
            sw = s32[top]
            rank_w = np.argsort(np.argsort(-sw)); rank_d = np.argsort(np.argsort(-sd))
            spearman = 1.0 - 6.0 * float(np.sum((rank_w - rank_d) ** 2)) / (len(sw) * (len(sw) ** 2 - 1))
            dt = np.abs(t32[top].astype(np.int64) - td.astype(np.int64))
            dt = np.minimum(dt, 128 - dt)  # periodic
            report["window_effect"] = {
                "rotations": int(len(qd)), "direct_rotations_per_s": round(d_rps, 1),
                "median_rel_peak_diff": float(np.median(np.abs(sw - sd) / np.abs(sd))),
                "max_rel_peak_diff": float(np.max(np.abs(sw - sd) / np.abs(sd))),
                "same_t_frac": float(np.mean(np.all(dt == 0, axis=1))),
                "max_t_shift": int(dt.max()),
                "same_best": bool(int(np.argmax(sw)) == int(np.argmax(sd))),
                "spearman": round(spearman, 4)}

        # --- the nonequispaced route: octree-adaptive samples of the moving part
        # and the type-1 transform (ES spreading on the 2x grid, FFT,
        # deconvolution) for the same rotations as the direct reference
        if args.direct_rotations and args.nfft_rotations:
            qn = qd[:args.nfft_rotations]
            sdn, tdn = sd[:len(qn)], td[:len(qn)]
            rows, s_full = [], None
            ctx.octree_samples(rho_m, w, mv.grid, 0.0, 3)  # workspace allocation outside the timings
            for tol in [float(v) for v in args.nfft_tols.split(",")]:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pos, cc, lev = ctx.octree_samples(rho_m, w, mv.grid, tol, 3)  # reading the count synchronises
                t_oct = time.perf_counter() - t0
                ctx.score_rotations_nfft(spec, fx.grid, pos, cc, qn[:1], width=args.nfft_width)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                on = ctx.score_rotations_nfft(spec, fx.grid, pos, cc, qn, width=args.nfft_width)
                torch.cuda.synchronize()
                dt_n = time.perf_counter() - t0
                sn = on["score"].cpu().numpy().astype(np.float64)
                tn = on["t"].cpu().numpy()
                if s_full is None:
                    s_full = sn
                shift = np.abs(tn.astype(np.int64) - tdn.astype(np.int64))
                shift = np.minimum(shift, 128 - shift)
                rk_n = np.argsort(np.argsort(-sn)); rk_d = np.argsort(np.argsort(-sdn))
                nq = len(qn)
                rows.append({
                    "tol": tol, "samples": int(len(cc)), "sample_frac": round(len(cc) / float(rho_m.numel()), 4),
                    "levels": np.bincount(lev.cpu().numpy(), minlength=4).tolist(),
                    "octree_ms": round(1e3 * t_oct, 3), "rotations_per_s": round(nq / dt_n, 1),
                    "vs_direct_median_rel": float(np.median(np.abs(sn - sdn) / np.abs(sdn))),
                    "vs_direct_max_rel": float(np.max(np.abs(sn - sdn) / np.abs(sdn))),
                    "vs_direct_same_t_frac": float(np.mean(np.all(shift == 0, axis=1))),
                    "vs_direct_same_best": bool(int(np.argmax(sn)) == int(np.argmax(sdn))),
                    "vs_direct_spearman": round(1.0 - 6.0 * float(np.sum((rk_n - rk_d) ** 2)) / (nq * (nq * nq - 1)),
                                                4) if nq > 1 else None,
                    "vs_all_nodes_max_rel": float(np.max(np.abs(sn - s_full) / np.abs(s_full)))})
            report["nonequispaced"] = {"width": args.nfft_width, "oversampling": 2, "rotations": int(len(qn)),
                                       "octree_levels": 3, "per_tolerance": rows}

        # --- shape gradients: the cotangent of 32 refined poses' scores with
        # respect to the moving coefficients, then the SDF adjoint over the
        # moving part's boundary samples (both timed with events)
        sp = torch.tensor(np.concatenate([out["refined"][:32].cpu().numpy(), pair.quats[:32]], axis=1),
                          dtype=torch.float64, device=dev)
        ctx.score_grad_coef(rho_f, fx.grid, rho_m, w, mv.grid, sp)
        ctx.sdf_build_adjoint(mv.samples.q, mv.samples.n, mv.samples.w, mv.grid, pair.params, rho_m)
        torch.cuda.synchronize()
        a0, a1, a2 = ev(), ev(), ev()
        a0.record(stream)
        _, _, gco, _ = ctx.score_grad_coef(rho_f, fx.grid, rho_m, w, mv.grid, sp)
        a1.record(stream)
        ctx.sdf_build_adjoint(mv.samples.q, mv.samples.n, mv.samples.w, mv.grid, pair.params, w * gco)
        a2.record(stream)
        torch.cuda.synchronize()
        report["shape_grad"] = {"poses": 32, "moving_samples": mv.samples.count,
                                "cotangent_ms": round(a0.elapsed_time(a1), 3),
                                "sdf_adjoint_ms": round(a1.elapsed_time(a2), 3)}

        # --- pose-gradient evaluations: forward + backward through the adjoint kernel
        B = args.grad_poses
        top = ctx.topk(out["score"], min(n_rot, B)).long()
        base_t = out["refined"][top].cpu().numpy()
        base_q = pair.quats[top.cpu().numpy()]
        reps = int(math.ceil(B / len(base_t)))
        tt, qq = wr.perturb_poses(np.tile(base_t, (reps, 1))[:B], np.tile(base_q, (reps, 1))[:B], 2.0, 10.0, 7)
        poses = torch.tensor(np.concatenate([tt, qq], axis=1), dtype=torch.float64, device=dev, requires_grad=True)
        opt = torch.optim.SGD([poses], lr=1e-3)
        for it in range(args.grad_steps + 1):
            if it == 1:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            opt.zero_grad()
            sc = sdf_score(poses, w, ctx, rho_f, fx.grid, rho_m, mv.grid)
            (-sc.sum()).backward()
            opt.step()
        torch.cuda.synchronize()
        report["pose_grad_evals_per_s"] = B * args.grad_steps / (time.perf_counter() - t0)
        ctx64.close()

        # --- protein-like pair: SDFs from 241k / 57k samples, rotations 64 per launch (graph replay)
        if args.protein_rotations:
            pp = C.protein_like(seed=0, n_rot=args.protein_rotations)
            pf, pm = pp.fixed, pp.moving
            b0, b1, b2 = ev(), ev(), ev()
            b0.record(stream)
            rf = ctx.sdf_build(pf.samples.q, pf.samples.n, pf.samples.w, pf.grid, pp.params)
            b1.record(stream)
            rm = ctx.sdf_build(pm.samples.q, pm.samples.n, pm.samples.w, pm.grid, pp.params)
            b2.record(stream)
            psp = ctx.spectrum(rf, pf.grid)
            pw = torch.ones(rm.shape, dtype=torch.float32, device=dev)
            ctx.set_option("batch", 64)
            pout = ctx.score_rotations(psp, pf.grid, rm, pw, pm.grid, pp.quats)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                pout = ctx.score_rotations(psp, pf.grid, rm, pw, pm.grid, pp.quats, out=pout)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / 3
            build_ms = [b0.elapsed_time(b1), b1.elapsed_time(b2)]
            report["protein_like"] = {"rotations": len(pp.quats), "batch": 64, "graph": bool(args.graph),
                                      "rotations_per_s": round(len(pp.quats) / dt, 1),
                                      "samples": [pf.samples.count, pm.samples.count],
                                      "sdf_build_ms": [round(x, 2) for x in build_ms],
                                      "end_to_end_ms": round(sum(build_ms) + 1e3 * dt, 2),
                                      "receptor_build": sdf_build_counts(ctx, pf, pp.params, build_ms[0])}
            # --- differentiable refinement on the protein-like pair: poses from the
            # top peaks, perturbed by N(0, 2) grid units and N(0, 10 deg), then
            # gradient ascent on the score through the adjoint kernel
            if args.refine_poses:
                B = args.refine_poses
                topi = ctx.topk(pout["score"], min(len(pp.quats), B)).long()
                bt = pout["refined"][topi].cpu().numpy()
                bq = pp.quats[topi.cpu().numpy()]
                reps = int(math.ceil(B / len(bt)))
                tt, qq = wr.perturb_poses(np.tile(bt, (reps, 1))[:B], np.tile(bq, (reps, 1))[:B], 2.0, 10.0, 11)
                rposes = torch.tensor(np.concatenate([tt, qq], axis=1), dtype=torch.float64, device=dev,
                                      requires_grad=True)
                ropt = torch.optim.Adam([rposes], lr=args.refine_lr)
                s_start = None
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for it in range(args.refine_steps):
                    ropt.zero_grad()
                    sc = sdf_score(rposes, pw, ctx, rf, pf.grid, rm, pm.grid)
                    if it == 0:
                        s_start = sc.detach().double().clone()
                    (-sc.sum()).backward()
                    ropt.step()
                torch.cuda.synchronize()
                dt_r = time.perf_counter() - t0
                s_end = ctx.score_grad(rf, pf.grid, rm, pw, pm.grid, rposes.detach(), want_pose=False)[0].double()
                report["refinement"] = {
                    "pair": "protein_like", "poses": B, "steps": args.refine_steps, "optimizer": "adam",
                    "lr": args.refine_lr, "evals_per_s": round(B * args.refine_steps / dt_r, 1),
                    "mean_score_start": float(s_start.mean()), "mean_score_end": float(s_end.mean()),
                    "improved_frac": float((s_end > s_start).double().mean()),
                    "best_peak_score": float(pout["score"].max())}
                del rposes, ropt
            ctx.set_option("batch", args.batch)
            del rf, rm, psp, pw, pout

        # --- alternative kernels of eq. 13 (the Validation section's comparison of
        # the DSL and skeletal affinities): best poses and score-volume shapes
        if args.phi_kernels:
            report["phi_kernels"] = phi_kernel_section(dev)

        # --- uneven multi-pair queue: pairs cycle through the three grid classes
        # the uneven batch picks by extent (128^3 / 64^3, 96^3 / 48^3, 64^3 / 32^3);
        # seeded random fields, since the work does not depend on the values
        if args.uneven_pairs:
            from workloads import rotations as wrot
            classes = [(128, 64), (96, 48), (64, 32)]
            gen = torch.Generator(device=dev).manual_seed(11)
            jobs = []
            for i in range(args.uneven_pairs):
                n, nm = classes[i % 3]
                gfix = C.GridSpec((n, n, n), (0.0, 0.0, 0.0), 1.0)
                gmov = C.body_grid(nm, (0.0, 0.0, 0.0), 1.0)
                jobs.append({"spec": torch.randn((n, n, n), dtype=torch.complex64, device=dev, generator=gen) * 1e-3,
                             "g_fixed": gfix,
                             "rho_moving": torch.randn((nm, nm, nm), dtype=torch.complex64, device=dev, generator=gen),
                             "w_moving": torch.ones((nm, nm, nm), dtype=torch.float32, device=dev),
                             "g_moving": gmov, "quats": wrot.uniform_quaternions(512, 5000 + i)})
            ctx.set_option("autotune", 1)
            ctx.score_pairs(jobs)  # tunes the two smaller classes, captures the graph
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                ctx.score_pairs(jobs)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / 2
            total = 512 * len(jobs)
            report["uneven_batch"] = {"pairs": len(jobs), "rotations": total,
                                      "rotations_per_s": round(total / dt, 1),
                                      "classes": ["128^3/64^3", "96^3/48^3", "64^3/32^3"],
                                      "fields": "seeded random (the work does not depend on the values)"}
            del jobs
            if args.uneven_e2e:
                workers = max(1, min(16, len(os.sched_getaffinity(0))))
                report["uneven_end_to_end"] = uneven_end_to_end(ctx, dev, args.uneven_pairs, workers)
        ctx.close()

    line = {"metric": "rotations scored/sec at 128^3 (FP32 fused path); FP64 path and pose-gradient evals/sec "
                      "reported alongside",
            "value": round(value, 1), "unit": "rotations/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "mechanical_3d: box-with-hole (fixed, 15.7k samples) vs plate-with-peg (moving, "
                                   "4.1k samples), 128^3 grid h=1, 64^3 body box, 576 Hopf rotations",
                       "rotations": n_rot, "batch": args.batch, "rotations_per_launch": sizes,
                       "graph": bool(args.graph),
                       "pencil_group": args.pencil_group, "radix": (tuned or {}).get("radix", 0),
                       "autotuned": bool(args.autotune)},
            "roofline": roofline,
            "fp64_rotations_per_s": round(report["fp64_rotations_per_s"], 1),
            "pose_grad_evals_per_s": round(report["pose_grad_evals_per_s"], 1),
            "fp32_vs_fp64": report["fp32_vs_fp64"],
            "window_effect": report.get("window_effect"),
            "nonequispaced": report.get("nonequispaced"),
            "shape_grad": report.get("shape_grad"),
            "stage_GBs": round(report["stage_GBs"], 1),
            "correlation_stage": report["correlation_stage"],
            "slab_reach": report["slab_reach"],
            "sdf_build_fixed_ms": round(report["sdf_build_fixed_ms"], 3),
            "sdf_build_fixed": report["sdf_build_fixed"],
            "spectrum_ms": round(report["spectrum_ms"], 4),
            "protein_like": report.get("protein_like"),
            "refinement": report.get("refinement"),
            "uneven_batch": report.get("uneven_batch"),
            "uneven_end_to_end": report.get("uneven_end_to_end"),
            "phi_kernels": report.get("phi_kernels"),
            "kernels": report["kernels"]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(pair, args.cpu_rotations)
        line["cpu_oracle_extras"] = cpu_extras(pair)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
