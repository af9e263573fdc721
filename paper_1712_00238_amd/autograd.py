"""torch.autograd.Function over the score_grad adjoint kernel.

forward(poses, w) -> scores.  When the poses need a gradient and the body
weights do not (pose refinement), forward runs the value-and-gradient kernel
once and keeps the B x 7 pose derivatives (FP64) for backward, which only
scales them by the incoming gradient.  When the weights need a gradient,
backward re-runs the value-and-gradient kernel with the incoming gradient as
per-pose scale, since d(loss)/d(w) = sum_b g_b Re(rho_M(x_k) Phi_b(y_k))
depends on it.  The B-spline stencils are recomputed in every call; no
spread grid is stored.
"""

from __future__ import annotations

import torch


class SDFScore(torch.autograd.Function):
    @staticmethod
    def forward(ctx, poses, w, sctx, rho_fixed, g_fixed, rho_moving, g_moving):
        pose_only = bool(ctx.needs_input_grad[0]) and not bool(ctx.needs_input_grad[1])
        score, gp, _ = sctx.score_grad(rho_fixed, g_fixed, rho_moving, w.detach(), g_moving, poses.detach(),
                                       want_pose=pose_only, want_w=False)
        ctx.save_for_backward(poses, w)
        ctx.aux = (sctx, rho_fixed, g_fixed, rho_moving, g_moving)
        ctx.gp = gp
        return score

    @staticmethod
    def backward(ctx, grad_score):
        poses, w = ctx.saved_tensors
        gs = grad_score.detach().to(torch.float64).contiguous()
        want_w = bool(ctx.needs_input_grad[1])
        if ctx.gp is not None and not want_w:
            return ctx.gp * gs[:, None], None, None, None, None, None, None
        sctx, rho_fixed, g_fixed, rho_moving, g_moving = ctx.aux
        _, gp, gw = sctx.score_grad(rho_fixed, g_fixed, rho_moving, w.detach(), g_moving, poses.detach(),
                                    want_pose=True, want_w=want_w, grad_scale=gs)
        grad_poses = gp * gs[:, None] if ctx.needs_input_grad[0] else None
        return grad_poses, (gw if want_w else None), None, None, None, None, None


def sdf_score(poses, w, sctx, rho_fixed, g_fixed, rho_moving, g_moving):
    """Differentiable score of B poses (B x 7 FP64: t in grid units, q w-first)."""
    return SDFScore.apply(poses, w, sctx, rho_fixed, g_fixed, rho_moving, g_moving)
