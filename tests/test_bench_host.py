"""Host-side pieces of bench.py (no GPU): the stored-intermediates baseline of the config-4
memory measurement computes the same loss as the method (FP64, against the oracle's compositing
and distortion), and autograd through it gives the oracle's gradients, so the measurement
compares two ways of computing one thing."""
import numpy as np
import torch

import bench
import oracle
import synth


def test_stored_composite_matches_oracle():
    wl = synth.config4(R=48, N=64, n=24)
    smp = wl.samples
    R, S = smp.n_rays, smp.n_samples
    lens = np.diff(smp.ray_offsets)
    N = int(lens.max())
    assert np.all((lens == 0) | (lens == N)) and (lens == 0).any() and (lens == N).any()
    Rh = S // N
    hit = torch.as_tensor(np.flatnonzero(lens))
    shift = oracle.act_shift()
    rng = np.random.default_rng(3)
    srgb = rng.random((S, 3))
    d64 = lambda a: torch.tensor(np.asarray(a, np.float64))
    raw = d64(oracle.gather(wl.density, smp.xyz)[:, 0]).requires_grad_(True)
    srgb_t = d64(srgb).requires_grad_(True)
    rgb, D = bench.stored_composite(raw, d64(smp.delta), srgb_t, d64(smp.s_mid).view(Rh, N),
                                    d64(smp.s_len).view(Rh, N), shift, hit, R)
    o = oracle.render_forward(smp, wl.density, srgb=srgb, shift=shift)
    np.testing.assert_allclose(rgb.detach().numpy(), o["rgb"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(D.detach().numpy(), o["D"], rtol=1e-10, atol=1e-14 * np.abs(o["D"]).max())
    G_C, G_D = rng.standard_normal((R, 3)), rng.standard_normal(R)
    ((rgb * d64(G_C)).sum() + (D * d64(G_D)).sum()).backward()
    og = oracle.render_backward(smp, wl.density, G_C, G_D, None, srgb=srgb, shift=shift)
    np.testing.assert_allclose(srgb_t.grad.numpy(), og["grad_srgb"], rtol=1e-9, atol=1e-12)
    gd = oracle.scatter(wl.density, smp.xyz, raw.grad.numpy()[:, None])
    np.testing.assert_allclose(gd, og["grad_density"], rtol=1e-8, atol=1e-10 * np.abs(og["grad_density"]).max())
