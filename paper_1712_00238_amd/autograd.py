"""torch.autograd.Functions over the adjoint kernels.

SDFScore: forward(poses, w, rho_moving) -> scores.  When the poses need a
gradient and nothing else does (pose refinement), forward runs the
value-and-gradient kernel once and keeps the B x 7 pose derivatives (FP64);
backward scales them by the incoming gradient in the library
(score_grad_pose_chain).  Otherwise backward calls score_grad_backward, which
re-runs the kernel with the incoming gradient g_b as per-pose scale and
returns the scaled pose gradient, d(loss)/d(w_k) = Re(rho_M(x_k) G_k) with
G_k = sum_b g_b Phi_b(y_k), the moving field's cotangent w_k G_k and the
fixed field's cotangent sum_b g_b sum_k c_k B3(p - y_kb).  The B-spline
stencils are recomputed in every call; no spread grid is stored.

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
        # every product of the chain rule runs in the library; this only routes
        # tensors and converts complex cotangents to torch's conjugate convention
        poses, w, rho_moving = ctx.saved_tensors
        gs = grad_score.detach().to(torch.float64).contiguous()
        want_pose, want_w = bool(ctx.needs_input_grad[0]), bool(ctx.needs_input_grad[1])
        want_fixed, want_rho = bool(ctx.needs_input_grad[3]), bool(ctx.needs_input_grad[5])
        sctx, rho_fixed, g_fixed, g_moving = ctx.aux
        grad_poses = None
        if want_pose and ctx.gp is not None:
            grad_poses = sctx.score_grad_pose_chain(ctx.gp, gs)
        pose_here = want_pose and ctx.gp is None
        gw = grad_rho = grad_fixed = None
        if pose_here or want_w or want_rho or want_fixed:
            gp, gw, gr, gf = sctx.score_grad_backward(rho_fixed.detach(), g_fixed, rho_moving.detach(), w.detach(),
                                                      g_moving, poses.detach(), gs, want_pose=pose_here,
                                                      want_w=want_w, want_rho=want_rho, want_fixed=want_fixed)
            if pose_here:
                grad_poses = gp
            grad_rho = torch.conj(gr) if want_rho else None
            grad_fixed = torch.conj(gf) if want_fixed else None
        return grad_poses, gw, None, grad_fixed, None, grad_rho, None


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
