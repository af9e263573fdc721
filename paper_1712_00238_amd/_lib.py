"""ctypes view of libsdfdock.so (the C ABI declared in include/sdfdock.h).

Loading never falls back to anything: a missing or unloadable library raises.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# SDF_LIB_PATH selects another build of the same library (the host-sanitized
# one of the CPU tests); there is no fallback if it is missing
LIB_PATH = os.environ.get("SDF_LIB_PATH") or os.path.join(HERE, "libsdfdock.so")

SDF_OK, SDF_EINVAL, SDF_EUNSUPPORTED, SDF_EHIP, SDF_ENOMEM = 0, -1, -2, -3, -4
SDF_F32, SDF_F64 = 0, 1

EXPORTS = ["sdf_ctx_create", "sdf_ctx_destroy", "sdf_last_error", "sdf_ctx_set_option", "sdf_ctx_get_option",
           "sdf_ctx_stats", "sdf_ctx_stats_reset",
           "sdf_build", "sdf_build_phi", "sdf_spectrum", "score_rotations", "score_pairs", "sdf_autotune", "score_volume",
           "sdf_spread", "sdf_fft", "sdf_topk", "score_grad", "score_rotations_direct", "sdf_build_adjoint",
           "score_grad_noalloc", "score_grad_coef", "score_grad_fixed", "score_grad_backward",
           "score_grad_pose_chain", "octree_samples", "score_rotations_nfft", "score_volume_nfft"]


class SdfGrid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("origin", ctypes.c_double * 3), ("h", ctypes.c_double)]


class SdfParams(ctypes.Structure):
    _fields_ = [("lambda1", ctypes.c_double), ("lambda2", ctypes.c_double), ("sigma", ctypes.c_double),
                ("eps", ctypes.c_double), ("xi_floor", ctypes.c_double)]


class SdfPhi(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("radius", ctypes.c_double)]


PHI_KINDS = {"skeletal": 0, "inverse_square": 1, "radial": 2, "dsl": 3}


class SdfPairJob(ctypes.Structure):
    _fields_ = [("spec_fixed", ctypes.c_void_p), ("g_fixed", SdfGrid), ("rho_moving", ctypes.c_void_p),
                ("w_moving", ctypes.c_void_p), ("g_moving", SdfGrid), ("quats", ctypes.c_void_p),
                ("n_rot", ctypes.c_int64), ("peak_score", ctypes.c_void_p), ("peak_t", ctypes.c_void_p),
                ("peak_nbhd", ctypes.c_void_p), ("refined_t", ctypes.c_void_p)]


class SdfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sdfdock error {code}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1712_00238_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32p, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    gp, pp = ctypes.POINTER(SdfGrid), ctypes.POINTER(SdfParams)
    sig = {
        "sdf_ctx_create": ([ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_size_t], ctypes.c_int),
        "sdf_ctx_destroy": ([vp], None),
        "sdf_last_error": ([vp], ctypes.c_char_p),
        "sdf_ctx_set_option": ([vp, ctypes.c_char_p, i64], ctypes.c_int),
        "sdf_ctx_get_option": ([vp, ctypes.c_char_p, ctypes.POINTER(i64)], ctypes.c_int),
        "sdf_ctx_stats": ([vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)], ctypes.c_int),
        "sdf_ctx_stats_reset": ([vp], ctypes.c_int),
        "sdf_build": ([vp, vp, vp, vp, i64, gp, pp, vp, vp], ctypes.c_int),
        "sdf_build_phi": ([vp, vp, vp, vp, i64, gp, pp, ctypes.POINTER(SdfPhi), vp, vp], ctypes.c_int),
        "sdf_build_adjoint": ([vp, vp, vp, vp, i64, gp, pp, vp, vp, vp, vp, vp], ctypes.c_int),
        "sdf_spectrum": ([vp, vp, gp, vp, vp], ctypes.c_int),
        "score_rotations": ([vp, vp, gp, vp, vp, gp, vp, i64, vp, vp, vp, vp, vp], ctypes.c_int),
        "score_rotations_direct": ([vp, vp, gp, vp, vp, vp, i64, gp, pp, ctypes.c_double, vp, i64, vp, vp, vp, vp,
                                    vp], ctypes.c_int),
        "score_pairs": ([vp, ctypes.POINTER(SdfPairJob), i64, vp], ctypes.c_int),
        "sdf_autotune": ([vp, gp, gp, ctypes.c_char_p, ctypes.c_size_t, vp], ctypes.c_int),
        "score_volume": ([vp, vp, gp, vp, vp, gp, vp, i64, vp, vp], ctypes.c_int),
        "sdf_spread": ([vp, gp, vp, vp, gp, vp, i64, vp, vp], ctypes.c_int),
        "sdf_fft": ([vp, vp, vp, gp, ctypes.c_int, vp], ctypes.c_int),
        "sdf_topk": ([vp, vp, i64, i64, vp, vp], ctypes.c_int),
        "score_grad": ([vp, vp, gp, vp, vp, gp, vp, i64, vp, vp, vp, vp, vp], ctypes.c_int),
        "score_grad_noalloc": ([vp, vp, gp, vp, vp, gp, vp, i64, vp, vp, vp, vp, vp], ctypes.c_int),
        "score_grad_coef": ([vp, vp, gp, vp, vp, gp, vp, i64, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "score_grad_fixed": ([vp, gp, vp, vp, gp, vp, i64, vp, vp, vp], ctypes.c_int),
        "score_grad_backward": ([vp, vp, gp, vp, vp, gp, vp, i64, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "score_grad_pose_chain": ([vp, vp, vp, i64, vp, vp], ctypes.c_int),
        "octree_samples": ([vp, vp, vp, gp, ctypes.c_double, ctypes.c_int, vp, vp, vp, vp, vp], ctypes.c_int),
        "score_rotations_nfft": ([vp, vp, gp, vp, vp, i64, ctypes.c_int, vp, i64, vp, vp, vp, vp, vp],
                                 ctypes.c_int),
        "score_volume_nfft": ([vp, vp, gp, vp, vp, i64, ctypes.c_int, vp, i64, vp, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    del i32p, dp
    _lib = lib
    return lib


def check(rc: int, ctx=None):
    if rc != SDF_OK:
        msg = load().sdf_last_error(ctx)
        raise SdfError(rc, msg.decode() if msg else "")


def make_grid(spec) -> SdfGrid:
    g = SdfGrid()
    for a in range(3):
        g.n[a] = int(spec.n[a])
        g.origin[a] = float(spec.origin[a])
    g.h = float(spec.h)
    return g


def make_params(p) -> SdfParams:
    return SdfParams(float(p.lambda1), float(p.lambda2), float(p.sigma), float(p.eps), float(p.xi_floor))


def make_phi(kind: str, radius: float = 0.0) -> SdfPhi:
    if kind not in PHI_KINDS:
        raise ValueError(f"unknown phi kernel {kind!r}; one of {sorted(PHI_KINDS)}")
    return SdfPhi(PHI_KINDS[kind], float(radius))
