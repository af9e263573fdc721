"""torch.autograd.Function over the score_grad adjoint kernel.

forward(poses, w) -> scores runs the value-only kernel; backward recomputes
the B-spline stencils in the value-and-gradient kernel (nothing from the
forward pass is stored) and returns d(loss)/d(poses) (FP64) and, when
requested, d(loss)/d(w) = sum_b g_b Re(rho_M(x_k) Phi_b(y_k)).
"""

from __future__ import annotations

import torch


class SDFScore(torch.autograd.Function):
    @staticmethod
    def forward(ctx, poses, w, sctx, rho_fixed, g_fixed, rho_moving, g_moving):
        score, _, _ = sctx.score_grad(rho_fixed, g_fixed, rho_moving, w, g_moving, poses.detach(),
                                      want_pose=False, want_w=False)
        ctx.save_for_backward(poses, w)
        ctx.aux = (sctx, rho_fixed, g_fixed, rho_moving, g_moving)
        return score

    @staticmethod
    def backward(ctx, grad_score):
        poses, w = ctx.saved_tensors
        sctx, rho_fixed, g_fixed, rho_moving, g_moving = ctx.aux
        gs = grad_score.detach().to(torch.float64).contiguous()
        want_w = bool(ctx.needs_input_grad[1])
        _, gp, gw = sctx.score_grad(rho_fixed, g_fixed, rho_moving, w.detach(), g_moving, poses.detach(),
                                    want_pose=True, want_w=want_w, grad_scale=gs)
        grad_poses = gp * gs[:, None] if ctx.needs_input_grad[0] else None
        return grad_poses, (gw if want_w else None), None, None, None, None, None


def sdf_score(poses, w, sctx, rho_fixed, g_fixed, rho_moving, g_moving):
    """Differentiable score of B poses (B x 7 FP64: t in grid units, q w-first)."""
    return SDFScore.apply(poses, w, sctx, rho_fixed, g_fixed, rho_moving, g_moving)
