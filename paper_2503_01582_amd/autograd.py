"""The rendering path as a torch.autograd.Function (Sec. III-B: the loss is
back-propagated to the NeRF parameters).  Forward and backward both run in
libprenom's kernels; autograd only supplies the upstream gradients of
(rgb, depth, opacity), so any loss written in torch can drive the
hand-written adjoint.

recompute=False keeps the forward's per-sample features in a workspace until
backward; recompute=True runs both passes chunk by chunk over the rays in a
workspace of one chunk, keeps nothing between them and has the backward
rebuild each chunk's features (far less memory, one extra encode + MLP
forward)."""
from __future__ import annotations

import torch

from . import api


class PrenomRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, model, samp, bg, recompute):
        if params.data_ptr() != model.params.data_ptr():
            raise ValueError("params must be the model's parameter tensor")
        n, S = samp.t.shape
        ws = api.Workspace(params.device).get(model.arch, n, S, recompute)
        out = api.prenom_render_fwd(model, samp, None, ws, bg=bg, want_loss=False, recompute=recompute)
        ctx.model, ctx.samp, ctx.bg, ctx.recompute = model, samp, bg, recompute
        ctx.ws = None if recompute else ws
        return out["rgb"], out["depth"], out["opacity"]

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_opacity):
        model, samp = ctx.model, ctx.samp
        n, S = samp.t.shape
        dev = model.params.device
        g_rgb = torch.zeros((n, 3), device=dev) if g_rgb is None else g_rgb.contiguous().float()
        g_depth = None if g_depth is None else g_depth.contiguous().float()
        g_opacity = None if g_opacity is None else g_opacity.contiguous().float()
        ws = ctx.ws if ctx.ws is not None else api.Workspace(dev).get(model.arch, n, S, True)
        grads = torch.zeros_like(model.params)
        api.prenom_render_bwd(model, samp, None, ws, bg=ctx.bg, d_rgb=g_rgb, d_depth=g_depth,
                              d_opacity=g_opacity, grads=grads, recompute=ctx.recompute)
        ctx.ws = None
        return grads, None, None, None, None


def render(model: api.Model, samp: api.SampleOut, bg=None, recompute=False):
    """(rgb, depth, opacity) of the sampled rays, differentiable w.r.t.
    model.params (which must have requires_grad set)."""
    return PrenomRender.apply(model.params, model, samp, bg, recompute)
