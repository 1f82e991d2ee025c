"""Learned proposal stage: where to put the fine samples of a ray.

Pipeline per batch of rays (every stage a libdvgo kernel):
    proposal_coarse (64 uniform density-only samples -> weights -> ln(1 + w/eps))
    -> proposal_forward (64-64-64-64-64 MLP on BF16 matrix cores: logits, softmax, entropy)
    -> resample_offsets + resample (48 fine samples by inverse CDF; rays whose entropy
       exceeds tau fall back to 256 uniform samples), or resample_guarded_offsets +
       resample_guarded (coarse bins with weight nearby cut at plain spacing plus extra samples
       by the predicted probabilities; empty and occluded bins skipped)
    -> the usual gather / colour MLP / render on the fine ragged batch.
Training targets are the 64-bin histograms of the weights of a plain 256-sample render
(density-only render_forward with per-sample weights -> histogram), the loss is the
cross-entropy, and the FP32 master weights take an Adam step (grid_adam_step, no skip).
"""
from __future__ import annotations

import torch

from . import ops

N_BINS = 64


class ProposalNet:
    def __init__(self, W, b, lr=1e-3, betas=(0.9, 0.99), eps=1e-8, device="cuda"):
        """W, b: lists of 4 float arrays [64,64] / [64] (numpy or torch)."""
        def dev(a):
            return torch.as_tensor(a).to(device=device, dtype=torch.float32).contiguous()
        Ws, bs = [dev(w) for w in W], [dev(v) for v in b]
        self.flat = torch.cat([w.reshape(-1) for w in Ws] + [v.reshape(-1) for v in bs])
        self.grad = torch.zeros_like(self.flat)
        self.m = torch.zeros_like(self.flat)
        self.v = torch.zeros_like(self.flat)
        self.t_dev = torch.zeros(1, dtype=torch.int32, device=device)
        views, gviews, o = [], [], 0
        for t in Ws + bs:
            views.append(self.flat[o:o + t.numel()].view(t.shape))
            gviews.append(self.grad[o:o + t.numel()].view(t.shape))
            o += t.numel()
        self.params = ops.ProposalParams(views[:4], views[4:], gviews[:4], gviews[4:])
        self.lr, self.betas, self.eps = lr, betas, eps
        self.ws = None

    def forward(self, feat):
        return ops.proposal_forward(self.params, feat)

    def train_step(self, feat, target, loss=None):
        """One cross-entropy step on (feat [R,64], target [R,64]); returns the loss tensor."""
        R = feat.shape[0]
        need = ops.proposal_workspace_size(self.params, R)
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=feat.device)
        loss = ops.proposal_backward(self.params, feat, target, loss=loss, ws=self.ws)
        ops.counter_add(self.t_dev, 1)
        ops.grid_adam_step(self.flat, self.grad, self.m, self.v, lr=self.lr, beta1=self.betas[0],
                           beta2=self.betas[1], eps=self.eps, step_dev=self.t_dev, skip_zero_grad=False,
                           zero_grad_after=True)
        return loss


def coarse(rays: ops.RayBatch, density: ops.DeviceGrid, voxel: float, act_shift: float, eps: float = 1e-4):
    """Coarse pass: returns (feat [R,64], w_coarse [R,64])."""
    R = rays.n_rays
    w = torch.empty(R, N_BINS, device=rays.t_near.device)
    feat, _ = ops.proposal_coarse(rays, density, act_shift_=act_shift, voxel=voxel, eps=eps, w_coarse=w)
    return feat, w


def plain_targets(batch: ops.SampleBatch, density: ops.DeviceGrid, act_shift: float, min_mass=1e-4):
    """Histograms of the weights of a density-only render of `batch` (e.g. 256 uniform samples)."""
    w = torch.empty(batch.n_samples, device=batch.xyz.device)
    ops.render_forward(batch, density, None, None, act_shift_=act_shift, want_dist=False, sample_w=w,
                       density_only=True)
    return ops.histogram(batch.ray_offsets, w, batch.s_mid, N_BINS, min_mass)


def fine_batch(rays: ops.RayBatch, prob, entropy, tau, voxel, n_fine=48, n_plain=256):
    """Ragged fine batch from proposal probabilities (one host read of the sample count)."""
    offs = ops.resample_offsets(rays, entropy, tau, n_fine, n_plain)
    S = int(offs[-1].item())
    return ops.resample(rays, prob, entropy, tau, offs, S, voxel, n_fine, n_plain)


def guarded_batch(rays: ops.RayBatch, prob, w_coarse, entropy, tau, voxel, n_base=4, n_extra=32, w_min=1e-4):
    """Ragged fine batch by guarded resampling: the coarse bins with weight nearby get n_base
    sub-intervals plus a share of n_extra by the predicted probabilities, empty or occluded bins
    none (one host read of the sample count)."""
    offs, counts = ops.resample_guarded_offsets(rays, prob, w_coarse, entropy, tau, n_base, n_extra, w_min)
    S = int(offs[-1].item())
    return ops.resample_guarded(rays, offs, counts, S, voxel)
