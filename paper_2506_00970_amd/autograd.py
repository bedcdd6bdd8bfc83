"""``torch.autograd.Function`` over the HIP rasterizer.

``render(rast, params, tau, pose_ref, camera)`` renders surfels ``params`` [15, N]
at the pose Exp(tau) pose_ref and returns (rgb, depth, normal, alpha).  Its
backward runs the library's reverse mode: gradients to every surfel parameter
(when ``params`` requires grad) and to ``tau`` through the left perturbation of
the paper's manifold derivative (Sec. "Camera Pose Optimization",
eq:derivatives), pulled back by the SE(3) left Jacobian J_l(tau)^T (the
identity at tau = 0).  All arithmetic runs in libgs2d.so; this module only
routes tensors.

A rasterizer context keeps the state of its last forward only: run each forward's
backward before the next forward on the same ``Rasterizer``.
"""

from __future__ import annotations

import torch


class RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, tau, pose_ref, rast, camera):
        ctx.set_materialize_grads(False)
        pose = rast.pose_exp(tau.detach().contiguous(), pose_ref.detach().reshape(12).contiguous())
        out = rast.render(params.detach().contiguous(), camera, pose)
        ctx.rast = rast
        ctx.generation = out.generation
        ctx.save_for_backward(tau)
        return out.rgb, out.depth, out.normal, out.alpha

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_normal, g_alpha):
        (tau,) = ctx.saved_tensors
        rast = ctx.rast
        c = lambda g: None if g is None else g.contiguous()
        need_params = ctx.needs_input_grad[0]
        d_params, d_pose = rast.backward(ctx.generation, c(g_rgb), c(g_depth), c(g_normal), c(g_alpha),
                                         params_grad=need_params)
        d_tau = rast.pose_tau_grad(tau.detach().contiguous(), d_pose) if ctx.needs_input_grad[1] else None
        return d_params, d_tau, None, None, None


def render(rast, params, tau, pose_ref, camera):
    """Differentiable render at Exp(tau) pose_ref; returns (rgb, depth, normal, alpha)."""
    return RenderFunction.apply(params, tau, pose_ref, rast, camera)
