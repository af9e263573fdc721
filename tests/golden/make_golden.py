"""Write the stored oracle results the full-size GPU tests compare against.

Every value here comes from the FP64 oracle (``oracle/``) applied to the
seeded workloads (``workloads/``); nothing is read from the GPU path.

  python tests/golden/make_golden.py peg      # planar peg-in-hole, 36 rotations
  python tests/golden/make_golden.py mech     # 3D mechanical pair, 576 Hopf rotations
  python tests/golden/make_golden.py protein  # protein-like pair, 64 seeded rotations
  python tests/golden/make_golden.py grad     # 32 perturbed poses of the protein-like pair
  python tests/golden/make_golden.py uneven   # 16 sampled pairs of the uneven batch, 8 rotations each

Files: <name>.txt with '#' header lines (workload, seed, parameters,
columns) and one whitespace-separated row per rotation / pose.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import correlate as oc  # noqa: E402
from oracle import grad as og  # noqa: E402
from oracle import peak as op  # noqa: E402
from oracle import pipeline  # noqa: E402
from oracle import spread as osp  # noqa: E402
from workloads import configs as C  # noqa: E402
from workloads import rotations as wr  # noqa: E402

_F = None


def _score_one(i):
    f = _F
    vol = oc.score_volume(f.rho_f, f.c, _QUATS[i], f.n_m, f.planar)
    s, _, t = op.peak(vol)
    nb = op.neighbourhood(vol, t)
    return i, s, t, nb, op.subvoxel(nb, t)


_QUATS = None


def score_parallel(fields, quats, workers):
    global _F, _QUATS
    _F, _QUATS = fields, quats
    rows = [None] * len(quats)
    ctx = __import__("multiprocessing").get_context("fork")
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        for i, s, t, nb, ref in ex.map(_score_one, range(len(quats)), chunksize=4):
            rows[i] = (s, t, nb, ref)
    return rows


def write_peaks(path, pair, quats, rows, note):
    with open(path, "w") as f:
        f.write(f"# oracle per-rotation peaks; workload {pair.name}; {note}\n")
        p = pair.params
        f.write(f"# params lambda1={p.lambda1} lambda2={p.lambda2} sigma={p.sigma} eps={p.eps} "
                f"xi_floor={p.xi_floor}\n")
        f.write("# written by tests/golden/make_golden.py from oracle/ only\n")
        f.write("# columns: rotation qw qx qy qz score tx ty tz refined_x refined_y refined_z nbhd[27] "
                "(offsets dz, dy, dx in -1..1, dx fastest)\n")
        for i, (q, (s, t, nb, ref)) in enumerate(zip(quats, rows)):
            f.write(f"{i} {q[0]:.17g} {q[1]:.17g} {q[2]:.17g} {q[3]:.17g} {s:.17g} {t[0]} {t[1]} {t[2]} "
                    f"{ref[0]:.17g} {ref[1]:.17g} {ref[2]:.17g} " + " ".join(f"{v:.17g}" for v in nb) + "\n")


UNEVEN_PAIRS = tuple(range(0, 256, 16))
UNEVEN_ROTATIONS = 8


def cached_fields(pair, name):
    """Oracle fields of a pair, kept between runs under SDF_GOLDEN_CACHE."""
    cache = os.path.join(os.environ.get("SDF_GOLDEN_CACHE", "/tmp/sdf_golden_cache"), name + "_fields.npz")
    if os.path.exists(cache):
        z = np.load(cache)
        return pipeline.PairFields(z["rho_f"], z["rho_m"], z["w_m"], z["c"], int(z["n_m"]), bool(z["planar"]))
    fields = pipeline.build_fields(pair)
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    np.savez(cache, rho_f=fields.rho_f, rho_m=fields.rho_m, w_m=fields.w_m, c=fields.c, n_m=fields.n_m,
             planar=fields.planar)
    return fields


def write_uneven(path, workers, t0):
    with open(path + ".tmp", "w") as f:
        f.write(f"# oracle per-rotation peaks; workload uneven batch (pairs {UNEVEN_PAIRS[0]}, "
                f"{UNEVEN_PAIRS[1]}, ..., {UNEVEN_PAIRS[-1]}), {UNEVEN_ROTATIONS} seeded rotations each "
                f"(uneven_pair(i, n_rot={UNEVEN_ROTATIONS}))\n")
        p = C.SDFParams()
        f.write(f"# params lambda1={p.lambda1} lambda2={p.lambda2} sigma={p.sigma} eps={p.eps} "
                f"xi_floor={p.xi_floor}\n")
        f.write("# written by tests/golden/make_golden.py from oracle/ only\n")
        f.write("# columns: pair N N_M rotation qw qx qy qz score tx ty tz refined_x refined_y refined_z nbhd[27] "
                "(offsets dz, dy, dx in -1..1, dx fastest)\n")
        for i in UNEVEN_PAIRS:
            pair = C.uneven_pair(i, n_rot=UNEVEN_ROTATIONS)
            fields = cached_fields(pair, pair.name)
            print("fields", pair.name, pair.n_fixed, pair.n_moving, time.time() - t0, flush=True)
            rows = score_parallel(fields, pair.quats, workers)
            for r, (q, (s, t, nb, ref)) in enumerate(zip(pair.quats, rows)):
                f.write(f"{i} {pair.n_fixed} {pair.n_moving} {r} {q[0]:.17g} {q[1]:.17g} {q[2]:.17g} {q[3]:.17g} "
                        f"{s:.17g} {t[0]} {t[1]} {t[2]} {ref[0]:.17g} {ref[1]:.17g} {ref[2]:.17g} " +
                        " ".join(f"{v:.17g}" for v in nb) + "\n")
            f.flush()
    os.replace(path + ".tmp", path)


def main(which, workers):
    t0 = time.time()
    if which == "peg":
        pair = C.peg_in_hole_2d(seed=0)
        fields = pipeline.build_fields(pair)
        rows = score_parallel(fields, pair.quats, workers)
        write_peaks(os.path.join(HERE, "peg_in_hole_2d_seed0.txt"), pair, pair.quats, rows, "seed 0, 36 rotations")
    elif which == "mech":
        pair = C.mechanical_3d(seed=0)
        fields = pipeline.build_fields(pair)
        print("fields", time.time() - t0, flush=True)
        rows = score_parallel(fields, pair.quats, workers)
        write_peaks(os.path.join(HERE, "mechanical_3d_seed0.txt"), pair, pair.quats, rows,
                    "seed 0, 576 Hopf rotations (level 1)")
    elif which == "uneven":
        write_uneven(os.path.join(HERE, "uneven_pairs_seed4000.txt"), workers, t0)
    elif which in ("protein", "grad"):
        pair = C.protein_like(seed=0, n_rot=64)
        cache = os.path.join(os.environ.get("SDF_GOLDEN_CACHE", "/tmp/sdf_golden_cache"), "protein_fields.npz")
        if os.path.exists(cache):
            z = np.load(cache)
            fields = pipeline.PairFields(z["rho_f"], z["rho_m"], z["w_m"], z["c"], int(z["n_m"]), False)
        else:
            fields = pipeline.build_fields(pair)
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            np.savez(cache, rho_f=fields.rho_f, rho_m=fields.rho_m, w_m=fields.w_m, c=fields.c, n_m=fields.n_m)
        print("fields", time.time() - t0, flush=True)
        if which == "protein":
            rows = score_parallel(fields, pair.quats, workers)
            write_peaks(os.path.join(HERE, "protein_like_seed0.txt"), pair, pair.quats, rows,
                        "seed 0, 64 seeded uniform rotations")
        else:
            peaks = np.loadtxt(os.path.join(HERE, "protein_like_seed0.txt"))
            order = op.top_k(peaks[:, 5], 8)
            base_t = np.repeat(peaks[order][:, 9:12], 4, axis=0)
            base_q = np.repeat(peaks[order][:, 1:5], 4, axis=0)
            t, q = wr.perturb_poses(base_t, base_q, 2.0, 10.0, 5)
            xb = osp.body_positions(fields.n_m)
            with open(os.path.join(HERE, "protein_like_grad_seed0.txt"), "w") as f:
                f.write("# oracle pose values and gradients; workload protein_like seed 0; 32 poses = top 8 oracle "
                        "peaks x 4, perturbed N(0, 2) per axis and N(0, 10 deg) about a random axis (seed 5)\n")
                f.write("# central finite differences with h = 1e-3 on the FP64 oracle value\n")
                f.write("# written by tests/golden/make_golden.py from oracle/ only\n")
                f.write("# columns: tx ty tz qw qx qy qz f g_tx g_ty g_tz g_qw g_qx g_qy g_qz "
                        "fd_tx fd_ty fd_tz fd_qw fd_qx fd_qy fd_qz\n")
                for b in range(len(t)):
                    val, dt, dq, _ = og.pose_value_and_grad(fields.rho_f, fields.c, fields.rho_m, xb, t[b], q[b])
                    x = np.concatenate([t[b], q[b]])
                    fd = og.fd_gradient(lambda v: og.pose_value(fields.rho_f, fields.c, xb, v[:3], v[3:]), x, 1e-3)
                    row = list(x) + [val] + list(dt) + list(dq) + list(fd)
                    f.write(" ".join(f"{v:.17g}" for v in row) + "\n")
                    print("pose", b, time.time() - t0, flush=True)
    print("done", which, time.time() - t0, flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else max(1, (os.cpu_count() or 2) - 1))
