"""MI355X (gfx950) skeletal-density-function shape-complementarity scoring.

The hot path (SDF construction, rotated spreading, 3D FFT correlation,
peak reduction, pose adjoint) runs in hand-written HIP kernels behind the C
ABI of include/sdfdock.h; this package holds the build script, the ctypes
binding (argument marshalling only) and the autograd wrapper.
"""

from . import _lib  # noqa: F401


def _lazy():
    from .api import Context  # noqa: F401
    from .autograd import SDFScore, sdf_score  # noqa: F401
    return Context, SDFScore, sdf_score


def __getattr__(name):
    if name in ("Context", "SDFScore", "sdf_score"):
        Context, SDFScore, sdf_score = _lazy()
        return {"Context": Context, "SDFScore": SDFScore, "sdf_score": sdf_score}[name]
    raise AttributeError(name)
