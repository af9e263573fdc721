"""Host-side checks of the C ABI: the library loads, exports every function
include/sdfdock.h declares, and rejects invalid arguments before touching a
device.  No compute call runs here."""

import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1712_00238_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sdfdock.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_expected_entry_points():
    names = declared_functions()
    assert sorted(_lib.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if " T " in line)
    for name in declared_functions():
        assert name in exported, name


def grid(n, origin=(0.0, 0.0, 0.0), h=1.0):
    g = _lib.SdfGrid()
    for a in range(3):
        g.n[a] = n[a]
        g.origin[a] = origin[a]
    g.h = h
    return g


def err_of(lib):
    return lib.sdf_last_error(None).decode()


def test_argument_validation_without_a_device():
    lib = _lib.load()
    null = ctypes.c_void_p(0)
    dummy = ctypes.c_void_p(4096)
    p = _lib.SdfParams(1.0, 3.0, 0.5, 1.5, 0.5)
    g = grid((16, 16, 16))
    # sdf_build: bad counts, grid, params
    assert lib.sdf_build(null, dummy, dummy, dummy, 0, ctypes.byref(g), ctypes.byref(p), dummy, null) == _lib.SDF_EINVAL
    assert "sample count" in err_of(lib)
    bad = grid((16, 0, 16))
    assert lib.sdf_build(null, dummy, dummy, dummy, 10, ctypes.byref(bad), ctypes.byref(p), dummy, null) == _lib.SDF_EINVAL
    pn = _lib.SdfParams(1.0, 3.0, float("nan"), 1.5, 0.5)
    assert lib.sdf_build(null, dummy, dummy, dummy, 10, ctypes.byref(g), ctypes.byref(pn), dummy, null) == _lib.SDF_EINVAL
    assert "non-finite" in err_of(lib)
    assert lib.sdf_build(null, dummy, dummy, dummy, 10, ctypes.byref(g), ctypes.byref(p), dummy, null) == _lib.SDF_EINVAL
    assert "ctx is NULL" in err_of(lib)
    # spectrum: unsupported FFT size, non-cubic grid, aliasing
    g20 = grid((20, 20, 20))
    assert lib.sdf_spectrum(null, dummy, ctypes.byref(g20), ctypes.c_void_p(8192), null) == _lib.SDF_EUNSUPPORTED
    g_nc = grid((16, 16, 8))
    assert lib.sdf_spectrum(null, dummy, ctypes.byref(g_nc), ctypes.c_void_p(8192), null) == _lib.SDF_EINVAL
    assert lib.sdf_spectrum(null, dummy, ctypes.byref(g), dummy, null) == _lib.SDF_EINVAL
    # score_rotations: body box too large for the torus, zero / NaN quaternions
    gm = grid((8, 8, 8))
    q = np.array([[1.0, 0, 0, 0]])
    qp = q.ctypes.data_as(ctypes.c_void_p)
    rc = lib.score_rotations(null, dummy, ctypes.byref(g), dummy, dummy, ctypes.byref(gm), qp, 1, dummy, dummy,
                             null, null, null)
    assert rc == _lib.SDF_EINVAL and "does not fit" in err_of(lib)
    gm6 = grid((6, 6, 6))
    qz = np.zeros((1, 4))
    rc = lib.score_rotations(null, dummy, ctypes.byref(g), dummy, dummy, ctypes.byref(gm6),
                             qz.ctypes.data_as(ctypes.c_void_p), 1, dummy, dummy, null, null, null)
    assert rc == _lib.SDF_EINVAL and "zero quaternion" in err_of(lib)
    qn = np.array([[math.nan, 0, 0, 1.0]])
    rc = lib.score_rotations(null, dummy, ctypes.byref(g), dummy, dummy, ctypes.byref(gm6),
                             qn.ctypes.data_as(ctypes.c_void_p), 1, dummy, dummy, null, null, null)
    assert rc == _lib.SDF_EINVAL and "non-finite" in err_of(lib)
    # mismatched spacing
    gm_h = grid((6, 6, 6), h=0.5)
    rc = lib.score_rotations(null, dummy, ctypes.byref(g), dummy, dummy, ctypes.byref(gm_h), qp, 1, dummy, dummy,
                             null, null, null)
    assert rc == _lib.SDF_EINVAL and "share h" in err_of(lib)
    # planar fixed grid needs a planar body box
    g2 = grid((32, 32, 1))
    rc = lib.score_rotations(null, dummy, ctypes.byref(g2), dummy, dummy, ctypes.byref(gm6), qp, 1, dummy, dummy,
                             null, null, null)
    assert rc == _lib.SDF_EINVAL
    # valid arguments but no context
    rc = lib.score_rotations(null, dummy, ctypes.byref(g), dummy, dummy, ctypes.byref(gm6), qp, 1, dummy, dummy,
                             null, null, null)
    assert rc == _lib.SDF_EINVAL and "ctx is NULL" in err_of(lib)
    # top-k and score_grad bounds
    assert lib.sdf_topk(null, dummy, 10, 0, dummy, null) == _lib.SDF_EINVAL
    assert lib.sdf_topk(null, dummy, 10, 11, dummy, null) == _lib.SDF_EINVAL
    assert lib.score_grad(null, dummy, ctypes.byref(g), dummy, dummy, ctypes.byref(gm6), dummy, 0, dummy, null, null,
                          null, null) == _lib.SDF_EINVAL
    # octree samples: N_M a multiple of 8, max_level <= 3, finite tol >= 0
    cnt = ctypes.c_void_p(8192)
    for n_m, lev, tol in ((12, 3, 0.1), (16, 4, 0.1), (16, -1, 0.1), (16, 3, -0.5), (16, 3, math.nan)):
        gmo = grid((n_m, n_m, n_m))
        assert lib.octree_samples(null, dummy, dummy, ctypes.byref(gmo), tol, lev, dummy, dummy, null, cnt,
                                  null) == _lib.SDF_EINVAL, (n_m, lev, tol)
    g16m = grid((16, 16, 16))
    assert lib.octree_samples(null, dummy, dummy, ctypes.byref(g16m), 0.1, 3, dummy, dummy, null, cnt,
                              null) == _lib.SDF_EINVAL and "ctx is NULL" in err_of(lib)
    # nonequispaced route: power-of-two N, width in [2, 8], sample count >= 0
    assert lib.score_volume_nfft(null, dummy, ctypes.byref(g), dummy, dummy, 10, 9, qp, 1, dummy,
                                 null) == _lib.SDF_EINVAL and "width" in err_of(lib)
    assert lib.score_volume_nfft(null, dummy, ctypes.byref(g), dummy, dummy, -1, 6, qp, 1, dummy,
                                 null) == _lib.SDF_EINVAL
    g48 = grid((48, 48, 48))  # no transform plan for 96-point lines
    assert lib.score_volume_nfft(null, dummy, ctypes.byref(g48), dummy, dummy, 10, 6, qp, 1, dummy,
                                 null) == _lib.SDF_EUNSUPPORTED
    assert lib.score_rotations_nfft(null, dummy, ctypes.byref(g), dummy, dummy, 10, 6, qz.ctypes.data_as(
        ctypes.c_void_p), 1, dummy, dummy, null, null, null) == _lib.SDF_EINVAL and "zero quaternion" in err_of(lib)
    assert lib.score_rotations_nfft(null, dummy, ctypes.byref(g), null, null, 0, 6, qp, 1, dummy, dummy, null, null,
                                    null) == _lib.SDF_EINVAL and "ctx is NULL" in err_of(lib)
    # options need a context
    assert lib.sdf_ctx_set_option(null, b"batch", 8) == _lib.SDF_EINVAL
    # context creation rejects bad dtypes and out pointers
    h = ctypes.c_void_p()
    assert lib.sdf_ctx_create(ctypes.byref(h), 0, 7, 0) == _lib.SDF_EINVAL
    assert lib.sdf_ctx_create(None, 0, 0, 0) == _lib.SDF_EINVAL


def test_context_creation_without_gpu_fails_cleanly():
    from conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is visible")
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.sdf_ctx_create(ctypes.byref(h), 0, 0, 0) == _lib.SDF_EHIP
    assert not h.value


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _lib.load()
