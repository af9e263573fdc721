"""Python binding of the sdfdock C ABI: argument marshalling only.

Every computation runs in the HIP library; these wrappers allocate output
tensors with PyTorch, pass raw device pointers and the current HIP stream,
and raise on any non-zero return code.  Grids and parameters are any
objects with the fields of ``workloads.configs.GridSpec`` / ``SDFParams``.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib

_REAL = {"f32": torch.float32, "f64": torch.float64}
_CPLX = {"f32": torch.complex64, "f64": torch.complex128}


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Context:
    """An sdfdock context on one GPU.  dtype "f32" or "f64"."""

    def __init__(self, device: int = 0, dtype: str = "f32", workspace_cap: int = 0):
        if dtype not in _REAL:
            raise ValueError("dtype must be 'f32' or 'f64'")
        self.lib = _lib.load()
        self.dtype = dtype
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        _lib.check(self.lib.sdf_ctx_create(ctypes.byref(h), device, _lib.SDF_F64 if dtype == "f64" else _lib.SDF_F32,
                                           workspace_cap))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.sdf_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def real(self):
        return _REAL[self.dtype]

    @property
    def cplx(self):
        return _CPLX[self.dtype]

    def _check(self, rc):
        _lib.check(rc, self.handle)

    def set_option(self, key: str, value: int):
        self._check(self.lib.sdf_ctx_set_option(self.handle, key.encode(), int(value)))

    def get_option(self, key: str) -> int:
        v = ctypes.c_int64()
        self._check(self.lib.sdf_ctx_get_option(self.handle, key.encode(), ctypes.byref(v)))
        return v.value

    def kernel_stats(self, kernel: str):
        """(total ms, launches) of one fused kernel since the last reset."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.sdf_ctx_stats(self.handle, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def reset_stats(self):
        self._check(self.lib.sdf_ctx_stats_reset(self.handle))

    def _dev(self, a, dtype):
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(a)
        return a.to(device=self.device, dtype=dtype).contiguous()

    # ------------------------------------------------------------------ SDF
    def sdf_build(self, q, n, w, grid, params, out=None, phi=None, radius=0.0):
        """Skeletal density function of one solid on ``grid`` -> complex (nz, ny, nx).
        ``phi`` selects another kernel of eq. 13 ("inverse_square", "radial",
        "dsl"; None or "skeletal" = eq. 15) with probe radius ``radius``."""
        q = self._dev(q, torch.float64)
        n = self._dev(n, torch.float64)
        w = self._dev(w, torch.float64)
        nx, ny, nz = grid.n
        if out is None:
            out = torch.empty((nz, ny, nx), dtype=self.cplx, device=self.device)
        g = _lib.make_grid(grid)
        p = _lib.make_params(params)
        if phi is None:
            self._check(self.lib.sdf_build(self.handle, _ptr(q), _ptr(n), _ptr(w), int(w.numel()), ctypes.byref(g),
                                           ctypes.byref(p), _ptr(out), _stream(self.device)))
        else:
            ph = _lib.make_phi(phi, radius)
            self._check(self.lib.sdf_build_phi(self.handle, _ptr(q), _ptr(n), _ptr(w), int(w.numel()),
                                               ctypes.byref(g), ctypes.byref(p), ctypes.byref(ph), _ptr(out),
                                               _stream(self.device)))
        return out

    def sdf_build_adjoint(self, q, n, w, grid, params, cot):
        """Shape gradients: (dL/dq (n, 3), dL/dn (n, 3), dL/dw (n,)) in FP64 for
        L = Re sum_p cot(p) rho(p), rho = sdf_build(q, n, w, grid, params)."""
        q = self._dev(q, torch.float64)
        n = self._dev(n, torch.float64)
        w = self._dev(w, torch.float64)
        cot = self._dev(cot, self.cplx)
        m = int(w.numel())
        gq = torch.empty((m, 3), dtype=torch.float64, device=self.device)
        gn = torch.empty((m, 3), dtype=torch.float64, device=self.device)
        gw = torch.empty(m, dtype=torch.float64, device=self.device)
        g = _lib.make_grid(grid)
        p = _lib.make_params(params)
        self._check(self.lib.sdf_build_adjoint(self.handle, _ptr(q), _ptr(n), _ptr(w), m, ctypes.byref(g),
                                               ctypes.byref(p), _ptr(cot), _ptr(gq), _ptr(gn), _ptr(gw),
                                               _stream(self.device)))
        return gq, gn, gw

    def spectrum(self, rho_fixed, grid, out=None):
        rho_fixed = self._dev(rho_fixed, self.cplx)
        if out is None:
            out = torch.empty_like(rho_fixed)
        g = _lib.make_grid(grid)
        self._check(self.lib.sdf_spectrum(self.handle, _ptr(rho_fixed), ctypes.byref(g), _ptr(out),
                                          _stream(self.device)))
        return out

    # ------------------------------------------------------------------ search
    def score_rotations(self, spec, g_fixed, rho_moving, w_moving, g_moving, quats, nbhd=True, refined=True,
                        out=None):
        """Per-rotation peaks.  Returns dict(score, t, nbhd, refined)."""
        q = np.ascontiguousarray(np.asarray(quats, dtype=np.float64).reshape(-1, 4))
        n_rot = len(q)
        spec = self._dev(spec, self.cplx)
        rm = self._dev(rho_moving, self.cplx)
        wm = self._dev(w_moving, self.real)
        if out is None:
            out = {"score": torch.empty(n_rot, dtype=self.real, device=self.device),
                   "t": torch.empty((n_rot, 3), dtype=torch.int32, device=self.device),
                   "nbhd": torch.empty((n_rot, 27), dtype=self.real, device=self.device) if nbhd else None,
                   "refined": torch.empty((n_rot, 3), dtype=torch.float64, device=self.device) if refined else None}
        gf, gm = _lib.make_grid(g_fixed), _lib.make_grid(g_moving)
        self._check(self.lib.score_rotations(self.handle, _ptr(spec), ctypes.byref(gf), _ptr(rm), _ptr(wm),
                                             ctypes.byref(gm), q.ctypes.data_as(ctypes.c_void_p), n_rot,
                                             _ptr(out["score"]), _ptr(out["t"]), _ptr(out["nbhd"]),
                                             _ptr(out["refined"]), _stream(self.device)))
        return out

    def score_rotations_direct(self, spec, g_fixed, q, n, w, g_moving, params, quats, w_node=None, nbhd=True,
                               refined=True):
        """Reference search without the spreading window: per rotation, the
        SDF of the moving part's turned boundary samples on its body box,
        placed on the fixed grid at integer offsets.  q, n: (n, 3), w: (n,)
        boundary samples (FP64); w_node defaults to h^3.  Returns dict(score,
        t, nbhd, refined) as score_rotations."""
        qq = np.ascontiguousarray(np.asarray(quats, dtype=np.float64).reshape(-1, 4))
        n_rot = len(qq)
        spec = self._dev(spec, self.cplx)
        qs = self._dev(q, torch.float64)
        ns = self._dev(n, torch.float64)
        ws = self._dev(w, torch.float64)
        out = {"score": torch.empty(n_rot, dtype=self.real, device=self.device),
               "t": torch.empty((n_rot, 3), dtype=torch.int32, device=self.device),
               "nbhd": torch.empty((n_rot, 27), dtype=self.real, device=self.device) if nbhd else None,
               "refined": torch.empty((n_rot, 3), dtype=torch.float64, device=self.device) if refined else None}
        gf, gm = _lib.make_grid(g_fixed), _lib.make_grid(g_moving)
        p = _lib.make_params(params)
        wn = float(g_moving.h ** 3) if w_node is None else float(w_node)
        self._check(self.lib.score_rotations_direct(self.handle, _ptr(spec), ctypes.byref(gf), _ptr(qs), _ptr(ns),
                                                    _ptr(ws), int(ws.numel()), ctypes.byref(gm), ctypes.byref(p), wn,
                                                    qq.ctypes.data_as(ctypes.c_void_p), n_rot, _ptr(out["score"]),
                                                    _ptr(out["t"]), _ptr(out["nbhd"]), _ptr(out["refined"]),
                                                    _stream(self.device)))
        return out

    def score_pairs(self, jobs, nbhd=True, refined=True):
        """Many pairs in one call.  ``jobs``: sequence of dicts with keys spec,
        g_fixed, rho_moving, w_moving, g_moving, quats.  Returns one output
        dict per job (score, t, nbhd, refined)."""
        arr = (_lib.SdfPairJob * len(jobs))()
        keep, outs = [], []
        for i, j in enumerate(jobs):
            q = np.ascontiguousarray(np.asarray(j["quats"], dtype=np.float64).reshape(-1, 4))
            spec = self._dev(j["spec"], self.cplx)
            rm = self._dev(j["rho_moving"], self.cplx)
            wm = self._dev(j["w_moving"], self.real)
            n = len(q)
            out = {"score": torch.empty(n, dtype=self.real, device=self.device),
                   "t": torch.empty((n, 3), dtype=torch.int32, device=self.device),
                   "nbhd": torch.empty((n, 27), dtype=self.real, device=self.device) if nbhd else None,
                   "refined": torch.empty((n, 3), dtype=torch.float64, device=self.device) if refined else None}
            keep += [q, spec, rm, wm]
            outs.append(out)
            a = arr[i]
            a.spec_fixed, a.rho_moving, a.w_moving = spec.data_ptr(), rm.data_ptr(), wm.data_ptr()
            a.g_fixed, a.g_moving = _lib.make_grid(j["g_fixed"]), _lib.make_grid(j["g_moving"])
            a.quats, a.n_rot = q.ctypes.data, n
            a.peak_score, a.peak_t = out["score"].data_ptr(), out["t"].data_ptr()
            a.peak_nbhd = out["nbhd"].data_ptr() if nbhd else None
            a.refined_t = out["refined"].data_ptr() if refined else None
        self._check(self.lib.score_pairs(self.handle, arr, len(jobs), _stream(self.device)))
        del keep
        return outs

    def autotune(self, g_fixed, g_moving) -> dict:
        """Tune the fused search for this grid-size class; returns the report."""
        import json
        buf = ctypes.create_string_buffer(1 << 16)
        gf, gm = _lib.make_grid(g_fixed), _lib.make_grid(g_moving)
        self._check(self.lib.sdf_autotune(self.handle, ctypes.byref(gf), ctypes.byref(gm), buf, len(buf),
                                          _stream(self.device)))
        return json.loads(buf.value.decode())

    def score_volume(self, spec, g_fixed, rho_moving, w_moving, g_moving, quats):
        q = np.ascontiguousarray(np.asarray(quats, dtype=np.float64).reshape(-1, 4))
        spec = self._dev(spec, self.cplx)
        rm = self._dev(rho_moving, self.cplx)
        wm = self._dev(w_moving, self.real)
        nx, ny, nz = g_fixed.n
        out = torch.empty((len(q), nz, ny, nx), dtype=self.real, device=self.device)
        gf, gm = _lib.make_grid(g_fixed), _lib.make_grid(g_moving)
        self._check(self.lib.score_volume(self.handle, _ptr(spec), ctypes.byref(gf), _ptr(rm), _ptr(wm),
                                          ctypes.byref(gm), q.ctypes.data_as(ctypes.c_void_p), len(q), _ptr(out),
                                          _stream(self.device)))
        return out

    def octree_samples(self, rho_moving, w_moving, g_moving, tol, max_level=3):
        """Octree-adaptive samples of the moving part: (pos (m', 3) real, c
        (m',) complex, level (m',) int32), device tensors trimmed to the leaf
        count (reading the count synchronises the stream)."""
        rm = self._dev(rho_moving, self.cplx)
        wm = self._dev(w_moving, self.real)
        cap = int(rm.numel())
        pos = torch.empty((cap, 3), dtype=self.real, device=self.device)
        c = torch.empty(cap, dtype=self.cplx, device=self.device)
        lev = torch.empty(cap, dtype=torch.int32, device=self.device)
        cnt = torch.zeros(1, dtype=torch.int64, device=self.device)
        gm = _lib.make_grid(g_moving)
        self._check(self.lib.octree_samples(self.handle, _ptr(rm), _ptr(wm), ctypes.byref(gm), float(tol),
                                            int(max_level), _ptr(pos), _ptr(c), _ptr(lev), _ptr(cnt),
                                            _stream(self.device)))
        m = int(cnt.item())
        return pos[:m], c[:m], lev[:m]

    def score_rotations_nfft(self, spec, g_fixed, pos, c, quats, width=6, nbhd=True, refined=True):
        """Search through the nonequispaced transform of samples (pos, c);
        returns dict(score, t, nbhd, refined) as score_rotations."""
        q = np.ascontiguousarray(np.asarray(quats, dtype=np.float64).reshape(-1, 4))
        n_rot = len(q)
        spec = self._dev(spec, self.cplx)
        ps = self._dev(pos, self.real).reshape(-1, 3)
        cs = self._dev(c, self.cplx).reshape(-1)
        out = {"score": torch.empty(n_rot, dtype=self.real, device=self.device),
               "t": torch.empty((n_rot, 3), dtype=torch.int32, device=self.device),
               "nbhd": torch.empty((n_rot, 27), dtype=self.real, device=self.device) if nbhd else None,
               "refined": torch.empty((n_rot, 3), dtype=torch.float64, device=self.device) if refined else None}
        gf = _lib.make_grid(g_fixed)
        self._check(self.lib.score_rotations_nfft(self.handle, _ptr(spec), ctypes.byref(gf), _ptr(ps), _ptr(cs),
                                                  int(cs.numel()), int(width), q.ctypes.data_as(ctypes.c_void_p),
                                                  n_rot, _ptr(out["score"]), _ptr(out["t"]), _ptr(out["nbhd"]),
                                                  _ptr(out["refined"]), _stream(self.device)))
        return out

    def score_volume_nfft(self, spec, g_fixed, pos, c, quats, width=6):
        """Volumes Re f(R, t) of the nonequispaced route, (n_rot, nz, ny, nx)."""
        q = np.ascontiguousarray(np.asarray(quats, dtype=np.float64).reshape(-1, 4))
        spec = self._dev(spec, self.cplx)
        ps = self._dev(pos, self.real).reshape(-1, 3)
        cs = self._dev(c, self.cplx).reshape(-1)
        nx, ny, nz = g_fixed.n
        out = torch.empty((len(q), nz, ny, nx), dtype=self.real, device=self.device)
        gf = _lib.make_grid(g_fixed)
        self._check(self.lib.score_volume_nfft(self.handle, _ptr(spec), ctypes.byref(gf), _ptr(ps), _ptr(cs),
                                               int(cs.numel()), int(width), q.ctypes.data_as(ctypes.c_void_p), len(q),
                                               _ptr(out), _stream(self.device)))
        return out

    def spread(self, g_fixed, rho_moving, w_moving, g_moving, quats):
        q = np.ascontiguousarray(np.asarray(quats, dtype=np.float64).reshape(-1, 4))
        rm = self._dev(rho_moving, self.cplx)
        wm = self._dev(w_moving, self.real)
        nx, ny, nz = g_fixed.n
        out = torch.empty((len(q), nz, ny, nx), dtype=self.cplx, device=self.device)
        gf, gm = _lib.make_grid(g_fixed), _lib.make_grid(g_moving)
        self._check(self.lib.sdf_spread(self.handle, ctypes.byref(gf), _ptr(rm), _ptr(wm), ctypes.byref(gm),
                                        q.ctypes.data_as(ctypes.c_void_p), len(q), _ptr(out), _stream(self.device)))
        return out

    def fft(self, x, grid, direction: int = -1):
        x = self._dev(x, self.cplx)
        out = torch.empty_like(x)
        g = _lib.make_grid(grid)
        self._check(self.lib.sdf_fft(self.handle, _ptr(x), _ptr(out), ctypes.byref(g), int(direction),
                                     _stream(self.device)))
        return out

    def topk(self, scores, k: int):
        scores = self._dev(scores, self.real)
        out = torch.empty(k, dtype=torch.int32, device=self.device)
        self._check(self.lib.sdf_topk(self.handle, _ptr(scores), int(scores.numel()), int(k), _ptr(out),
                                      _stream(self.device)))
        return out

    # ------------------------------------------------------------------ refinement
    def score_grad_coef(self, rho_fixed, g_fixed, rho_moving, w_moving, g_moving, poses, want_pose=False,
                        want_w=False, grad_scale=None):
        """score_grad with the cotangent of sum_b s_b f_b with respect to the
        moving coefficients c_k = w_k rho_M(x_k): grad_c[k] = sum_b s_b
        Phi_b(y_k), complex, shaped like rho_moving.  Returns (score, grad_pose
        or None, grad_c, grad_w or None)."""
        poses = self._dev(poses, torch.float64).reshape(-1, 7)
        B = poses.shape[0]
        rf = self._dev(rho_fixed, self.cplx)
        rm = self._dev(rho_moving, self.cplx)
        wm = self._dev(w_moving, self.real)
        score = torch.empty(B, dtype=self.real, device=self.device)
        gp = torch.empty((B, 7), dtype=torch.float64, device=self.device) if want_pose else None
        gc = torch.empty(rm.shape, dtype=self.cplx, device=self.device)
        gw = torch.empty(wm.shape, dtype=self.real, device=self.device) if want_w else None
        gs = None if grad_scale is None else self._dev(grad_scale, torch.float64)
        gf, gm = _lib.make_grid(g_fixed), _lib.make_grid(g_moving)
        self._check(self.lib.score_grad_coef(self.handle, _ptr(rf), ctypes.byref(gf), _ptr(rm), _ptr(wm),
                                             ctypes.byref(gm), _ptr(poses), B, _ptr(score), _ptr(gp), _ptr(gc),
                                             _ptr(gw), _ptr(gs), _stream(self.device)))
        return score, gp, gc, gw

    def score_grad_backward(self, rho_fixed, g_fixed, rho_moving, w_moving, g_moving, poses, grad_score,
                            want_pose=True, want_w=False, want_rho=False, want_fixed=False):
        """Backward of the scores for an incoming gradient grad_score (B,):
        (grad_pose (B, 7) FP64, grad_w, grad_rho_moving (cotangent w_k sum_b
        g_b Phi_b), grad_rho_fixed (cotangent of the fixed field)), each None
        unless asked for."""
        poses = self._dev(poses, torch.float64).reshape(-1, 7)
        B = poses.shape[0]
        rm = self._dev(rho_moving, self.cplx)
        wm = self._dev(w_moving, self.real)
        gs = self._dev(grad_score, torch.float64)
        side = want_pose or want_w or want_rho
        rf = self._dev(rho_fixed, self.cplx) if side else None
        gp = torch.empty((B, 7), dtype=torch.float64, device=self.device) if want_pose else None
        gw = torch.empty(wm.shape, dtype=self.real, device=self.device) if want_w else None
        gr = torch.empty(rm.shape, dtype=self.cplx, device=self.device) if want_rho else None
        nx, ny, nz = g_fixed.n
        gf = torch.empty((nz, ny, nx), dtype=self.cplx, device=self.device) if want_fixed else None
        g1, g2 = _lib.make_grid(g_fixed), _lib.make_grid(g_moving)
        self._check(self.lib.score_grad_backward(self.handle, _ptr(rf), ctypes.byref(g1), _ptr(rm), _ptr(wm),
                                                 ctypes.byref(g2), _ptr(poses), B, _ptr(gs), _ptr(gp), _ptr(gw),
                                                 _ptr(gr), _ptr(gf), _stream(self.device)))
        return gp, gw, gr, gf

    def score_grad_pose_chain(self, grad_pose, grad_score):
        """grad_pose[b] * grad_score[b] (FP64, (B, 7)), computed in the library."""
        gp = self._dev(grad_pose, torch.float64).reshape(-1, 7)
        gs = self._dev(grad_score, torch.float64)
        out = torch.empty_like(gp)
        self._check(self.lib.score_grad_pose_chain(self.handle, _ptr(gp), _ptr(gs), gp.shape[0], _ptr(out),
                                                   _stream(self.device)))
        return out

    def score_grad_fixed(self, g_fixed, rho_moving, w_moving, g_moving, poses, grad_scale=None):
        """Cotangent of sum_b s_b f_b with respect to rho_F: the periodic
        spread sum_b s_b sum_k c_k B3(p - y_kb), complex, shaped like the fixed
        grid (nz, ny, nx)."""
        poses = self._dev(poses, torch.float64).reshape(-1, 7)
        B = poses.shape[0]
        rm = self._dev(rho_moving, self.cplx)
        wm = self._dev(w_moving, self.real)
        nx, ny, nz = g_fixed.n
        out = torch.empty((nz, ny, nx), dtype=self.cplx, device=self.device)
        gs = None if grad_scale is None else self._dev(grad_scale, torch.float64)
        gf, gm = _lib.make_grid(g_fixed), _lib.make_grid(g_moving)
        self._check(self.lib.score_grad_fixed(self.handle, ctypes.byref(gf), _ptr(rm), _ptr(wm), ctypes.byref(gm),
                                              _ptr(poses), B, _ptr(gs), _ptr(out), _stream(self.device)))
        return out

    def score_grad_noalloc(self, rho_fixed, g_fixed, rho_moving, w_moving, g_moving, poses, score, grad_pose=None,
                           grad_w=None, grad_scale=None):
        """score_grad through the allocation-free entry point: every argument is
        a device tensor of the context's device and dtype that the caller has
        allocated (outputs score (B,), grad_pose (B, 7) FP64 or None, grad_w
        shaped like w_moving or None); nothing is converted or copied here."""
        B = int(poses.shape[0])
        for t in (rho_fixed, rho_moving, w_moving, poses, score, grad_pose, grad_w, grad_scale):
            if t is not None and (t.device != self.device or not t.is_contiguous()):
                raise ValueError("score_grad_noalloc takes contiguous tensors on the context's device")
        gf, gm = _lib.make_grid(g_fixed), _lib.make_grid(g_moving)
        self._check(self.lib.score_grad_noalloc(self.handle, _ptr(rho_fixed), ctypes.byref(gf), _ptr(rho_moving),
                                                _ptr(w_moving), ctypes.byref(gm), _ptr(poses), B, _ptr(score),
                                                _ptr(grad_pose), _ptr(grad_w), _ptr(grad_scale),
                                                _stream(self.device)))
        return score, grad_pose, grad_w

    def score_grad(self, rho_fixed, g_fixed, rho_moving, w_moving, g_moving, poses, want_pose=True,
                   want_w=False, grad_scale=None):
        poses = self._dev(poses, torch.float64).reshape(-1, 7)
        B = poses.shape[0]
        rf = self._dev(rho_fixed, self.cplx)
        rm = self._dev(rho_moving, self.cplx)
        wm = self._dev(w_moving, self.real)
        score = torch.empty(B, dtype=self.real, device=self.device)
        gp = torch.empty((B, 7), dtype=torch.float64, device=self.device) if want_pose else None
        gw = torch.empty(wm.shape, dtype=self.real, device=self.device) if want_w else None
        gs = None if grad_scale is None else self._dev(grad_scale, torch.float64)
        gf, gm = _lib.make_grid(g_fixed), _lib.make_grid(g_moving)
        self._check(self.lib.score_grad(self.handle, _ptr(rf), ctypes.byref(gf), _ptr(rm), _ptr(wm), ctypes.byref(gm),
                                        _ptr(poses), B, _ptr(score), _ptr(gp), _ptr(gw), _ptr(gs),
                                        _stream(self.device)))
        return score, gp, gw
