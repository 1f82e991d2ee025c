"""torch.autograd.Function wrappers over the libdvgo kernels.

The backward of each Function is the hand-written HIP backward; nothing is traced by
PyTorch.  The render Function recomputes every ray from per-chunk checkpoints in its
backward instead of saving per-sample intermediates.
"""
from __future__ import annotations

import torch

from . import ops


class RenderFn(torch.autograd.Function):
    """(density [nx,ny,nz,cs], colour) -> (rgb [R,3], T_final [R], dist [R]).

    colour is either a colour grid [nx,ny,nz,cs>=3] (``grid_color=True``) or per-sample
    rgb [S,3].  Gradients flow to the density grid and to the colour input.
    """

    @staticmethod
    def forward(ctx, density, colour, batch, box, grid_color, act_shift, halt_T, bg, want_dist):
        lo, hi = box
        dg = ops.DeviceGrid(density, lo, hi)
        cg = ops.DeviceGrid(colour, lo, hi, channels=3) if grid_color else None
        rgb, T, dist, state = ops.render_forward(batch, dg, cg, None if grid_color else colour, act_shift_=act_shift,
                                                 halt_T=halt_T, bg=bg, want_dist=want_dist)
        ctx.save_for_backward(density, colour, T, state)
        ctx.meta = (batch, box, grid_color, act_shift, halt_T, bg, want_dist)
        if dist is None:
            dist = torch.zeros_like(T)
        return rgb, T, dist

    @staticmethod
    def backward(ctx, g_rgb, g_T, g_dist):
        density, colour, T, state = ctx.saved_tensors
        batch, (lo, hi), grid_color, act_shift, halt_T, bg, want_dist = ctx.meta
        g_rgb = torch.zeros_like(T).unsqueeze(-1).expand(-1, 3).contiguous() if g_rgb is None else g_rgb.contiguous()
        g_T = None if g_T is None else g_T.contiguous()
        g_dist = None if (g_dist is None or not want_dist) else g_dist.contiguous()
        gden = torch.zeros_like(density)
        dg = ops.DeviceGrid(density, lo, hi, grad=gden)
        if grid_color:
            gcol = torch.zeros_like(colour)
            cg = ops.DeviceGrid(colour, lo, hi, grad=gcol, channels=3)
            ops.render_backward(batch, dg, cg, None, T, state, g_rgb, g_dist, g_T, act_shift_=act_shift, halt_T=halt_T,
                                bg=bg, want_dist=want_dist)
            return gden, gcol, None, None, None, None, None, None, None
        gs = ops.render_backward(batch, dg, None, colour, T, state, g_rgb, g_dist, g_T, act_shift_=act_shift,
                                 halt_T=halt_T, bg=bg, want_dist=want_dist)
        return gden, gs, None, None, None, None, None, None, None


def render(density, colour, batch, box, *, grid_color, act_shift, halt_T=0.0, bg=(1.0, 1.0, 1.0), want_dist=True):
    return RenderFn.apply(density, colour, batch, box, grid_color, act_shift, halt_T, tuple(bg), want_dist)


class DistortionFn(torch.autograd.Function):
    """Per-ray distortion loss (Eq. 1) of weights w [S] on a ragged layout."""

    @staticmethod
    def forward(ctx, w, ray_offsets, s_mid, s_len):
        loss, _ = ops.distortion_loss(ray_offsets, w.contiguous(), s_mid, s_len)
        ctx.save_for_backward(w, ray_offsets, s_mid, s_len)
        return loss

    @staticmethod
    def backward(ctx, g):
        w, offs, sm, sl = ctx.saved_tensors
        _, gw = ops.distortion_loss(offs, w.contiguous(), sm, sl, grad_loss=g.contiguous())
        return gw, None, None, None


def distortion(w, ray_offsets, s_mid, s_len):
    return DistortionFn.apply(w, ray_offsets, s_mid, s_len)


class GatherFn(torch.autograd.Function):
    """Trilinear gather of a channel-last grid at points xyz [S,3] -> [S,C]."""

    @staticmethod
    def forward(ctx, grid, xyz, box):
        lo, hi = box
        out = ops.grid_gather(ops.DeviceGrid(grid, lo, hi), xyz)
        ctx.save_for_backward(grid, xyz)
        ctx.box = box
        return out

    @staticmethod
    def backward(ctx, g):
        grid, xyz = ctx.saved_tensors
        lo, hi = ctx.box
        gg = torch.zeros_like(grid)
        ops.grid_scatter(ops.DeviceGrid(grid, lo, hi, grad=gg), xyz, g.contiguous())
        return gg, None, None


def gather(grid, xyz, box):
    return GatherFn.apply(grid, xyz, box)


class ColorMLPFn(torch.autograd.Function):
    """Colour MLP on FP32 matrix cores: feat [S,C] (+ view encoding of dirs) -> rgb [S,3]."""

    @staticmethod
    def forward(ctx, feat, W1, b1, W2, b2, W3, b3, ray_offsets, dirs, n_freq):
        mlp = ops.MLPParams([W1, W2, W3], [b1, b2, b3], in_feat=feat.shape[1], n_freq=n_freq)
        rgb = ops.mlp_forward(mlp, ray_offsets, dirs, feat)
        ctx.save_for_backward(feat, W1, b1, W2, b2, W3, b3, ray_offsets, dirs)
        ctx.n_freq = n_freq
        return rgb

    @staticmethod
    def backward(ctx, g):
        feat, W1, b1, W2, b2, W3, b3, offs, dirs = ctx.saved_tensors
        gW = [torch.zeros_like(W1), torch.zeros_like(W2), torch.zeros_like(W3)]
        gb = [torch.zeros_like(b1), torch.zeros_like(b2), torch.zeros_like(b3)]
        mlp = ops.MLPParams([W1, W2, W3], [b1, b2, b3], gW, gb, in_feat=feat.shape[1], n_freq=ctx.n_freq)
        gf = ops.mlp_backward(mlp, offs, dirs, feat, g.contiguous())
        return gf, gW[0], gb[0], gW[1], gb[1], gW[2], gb[2], None, None, None


def color_mlp(feat, W, b, ray_offsets, dirs, n_freq=4):
    return ColorMLPFn.apply(feat, W[0], b[0], W[1], b[1], W[2], b[2], ray_offsets, dirs, n_freq)
