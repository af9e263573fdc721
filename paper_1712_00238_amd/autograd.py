"""torch.autograd.Functions over the adjoint kernels.

SDFScore: forward(poses, w, rho_moving) -> scores.  When the poses need a
gradient and nothing else does (pose refinement), forward runs the
value-and-gradient kernel once and keeps the B x 7 pose derivatives (FP64)
for backward, which only scales them by the incoming gradient.  When the
weights or the moving field need a gradient, backward re-runs the kernel with
the incoming gradient as per-pose scale and takes the cotangent of the moving
coefficients c_k = w_k rho_M(x_k), G_k = sum_b g_b Phi_b(y_k): then
d(loss)/d(w_k) = Re(rho_M(x_k) G_k) and the moving field's cotangent is
w_k G_k.  The fixed field's cotangent is the spread sum_b g_b sum_k c_k
B3(p - y_kb) (score_grad_fixed).  The B-spline stencils are recomputed in every call; no spread grid
is stored.

SDFBuild: forward(q, n, w) -> rho (sdf_build); backward through
sdf_build_adjoint, giving shape gradients with respect to the boundary
samples.

Complex tensors follow torch's convention: for a real loss L of a complex z
the incoming gradient is dL/d(Re z) + i dL/d(Im z), the conjugate of the
cotangent g in L = Re sum g z that the kernels take.
"""

from __future__ import annotations

import torch


class SDFScore(torch.autograd.Function):
    @staticmethod
    def forward(ctx, poses, w, sctx, rho_fixed, g_fixed, rho_moving, g_moving):
        pose_only = bool(ctx.needs_input_grad[0]) and not (bool(ctx.needs_input_grad[1]) or
                                                             bool(ctx.needs_input_grad[5]))
        score, gp, _ = sctx.score_grad(rho_fixed.detach(), g_fixed, rho_moving.detach(), w.detach(), g_moving,
                                       poses.detach(), want_pose=pose_only, want_w=False)
        ctx.save_for_backward(poses, w, rho_moving)
        ctx.aux = (sctx, rho_fixed, g_fixed, g_moving)
        ctx.gp = gp
        return score

    @staticmethod
    def backward(ctx, grad_score):
        poses, w, rho_moving = ctx.saved_tensors
        gs = grad_score.detach().to(torch.float64).contiguous()
        want_w, want_rho = bool(ctx.needs_input_grad[1]), bool(ctx.needs_input_grad[5])
        want_fixed = bool(ctx.needs_input_grad[3])
        sctx, rho_fixed, g_fixed, g_moving = ctx.aux
        grad_fixed = None
        if want_fixed:
            grad_fixed = torch.conj(sctx.score_grad_fixed(g_fixed, rho_moving.detach(), w.detach(), g_moving,
                                                          poses.detach(), grad_scale=gs))
        if ctx.gp is not None and not (want_w or want_rho):
            return ctx.gp * gs[:, None], None, None, grad_fixed, None, None, None
        want_pose = bool(ctx.needs_input_grad[0])
        if not (want_pose or want_w or want_rho):
            return None, None, None, grad_fixed, None, None, None
        _, gp, gc, gw = sctx.score_grad_coef(rho_fixed, g_fixed, rho_moving.detach(), w.detach(), g_moving,
                                             poses.detach(), want_pose=want_pose, want_w=want_w, grad_scale=gs)
        grad_poses = gp * gs[:, None] if want_pose else None
        grad_rho = torch.conj(w.detach().to(gc.real.dtype) * gc) if want_rho else None
        return grad_poses, (gw if want_w else None), None, grad_fixed, None, grad_rho, None


def sdf_score(poses, w, sctx, rho_fixed, g_fixed, rho_moving, g_moving):
    """Differentiable score of B poses (B x 7 FP64: t in grid units, q w-first)."""
    return SDFScore.apply(poses, w, sctx, rho_fixed, g_fixed, rho_moving, g_moving)


class SDFBuild(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, n, w, sctx, grid, params):
        rho = sctx.sdf_build(q.detach(), n.detach(), w.detach(), grid, params)
        ctx.save_for_backward(q, n, w)
        ctx.aux = (sctx, grid, params)
        return rho

    @staticmethod
    def backward(ctx, grad_rho):
        q, n, w = ctx.saved_tensors
        sctx, grid, params = ctx.aux
        gq, gn, gw = sctx.sdf_build_adjoint(q.detach(), n.detach(), w.detach(), grid, params,
                                           torch.conj(grad_rho.detach()))
        return (gq.to(q.dtype) if ctx.needs_input_grad[0] else None,
                gn.to(n.dtype) if ctx.needs_input_grad[1] else None,
                gw.to(w.dtype) if ctx.needs_input_grad[2] else None, None, None, None)


def sdf_field(q, n, w, sctx, grid, params):
    """Differentiable sdf_build: rho from boundary samples (q, n: (m, 3), w: (m,), FP64 tensors)."""
    return SDFBuild.apply(q, n, w, sctx, grid, params)
