"""Pins of the oracle's colour MLP, Adam step and proposal network.

The MLP reduces to torch float64 Linear/ReLU/Sigmoid (a library routine) and its
backward to torch autograd; Adam with all-non-zero gradients reduces to
torch.optim.Adam in float64; the proposal network reduces to torch float64 with
bfloat16 rounding applied by torch's own conversion, and its resampler to closed forms.
"""
import numpy as np
import pytest
import torch

import synth

torch.set_num_threads(4)


def _pe(d, F):
    d = torch.as_tensor(d, dtype=torch.float64)
    fr = [d * (2.0 ** q) for q in range(F)]
    return torch.cat([d] + [torch.sin(v) for v in fr] + [torch.cos(v) for v in fr], dim=-1)


def _torch_mlp(mlp, feat, dirs_per_sample, F=4):
    W = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in mlp.W]
    b = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in mlp.b]
    f = torch.tensor(feat, dtype=torch.float64, requires_grad=True)
    x = torch.cat([f, _pe(dirs_per_sample, F)], dim=-1)
    h = torch.relu(torch.nn.functional.linear(x, W[0], b[0]))
    h = torch.relu(torch.nn.functional.linear(h, W[1], b[1]))
    rgb = torch.sigmoid(torch.nn.functional.linear(h, W[2], b[2]))
    return rgb, f, W, b


def test_mlp_matches_torch(orc):
    rng = np.random.default_rng(40)
    mlp = synth.mlp_weights(rng, bias_std=0.3)
    offs = np.array([0, 5, 5, 17, 30], np.int32)
    S = int(offs[-1])
    dirs = synth.scenes._unit(rng.standard_normal((4, 3))).astype(np.float32)
    feat = rng.standard_normal((S, 12))
    rgb = orc.mlp_forward(mlp, offs, dirs, feat)
    ray_of = np.repeat(np.arange(4), np.diff(offs))
    trgb, f, W, b = _torch_mlp(mlp, feat, dirs[ray_of].astype(np.float64))
    np.testing.assert_allclose(rgb, trgb.detach().numpy(), rtol=1e-12, atol=1e-14)
    g = rng.standard_normal((S, 3))
    (trgb * torch.tensor(g)).sum().backward()
    gf, gW, gb = orc.mlp_backward(mlp, offs, dirs, feat, g)
    np.testing.assert_allclose(gf, f.grad.numpy(), rtol=1e-10, atol=1e-13)
    for a, t in zip(gW + gb, W + b):
        np.testing.assert_allclose(a, t.grad.numpy(), rtol=1e-10, atol=1e-13)


def _h(t):
    """FP16 significand rounding by numpy's float64 -> float16 conversion (scale into [1, 2),
    convert, scale back).  numpy converts directly; torch's float64 -> half path rounds through
    float32 first (double rounding near ties), so it cannot serve as the reference."""
    t = np.asarray(t.detach().numpy() if isinstance(t, torch.Tensor) else t, dtype=np.float64)
    m, e = np.frexp(t)
    return torch.as_tensor(np.ldexp((2.0 * m).astype(np.float16).astype(np.float64), e - 1))


def test_r16_matches_torch_half(orc):
    rng = np.random.default_rng(44)
    x = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-12, 12, 2000),
                        [0.0, 1.0, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, -(1 + 2.0 ** -10 + 2.0 ** -11)]])
    np.testing.assert_array_equal(orc.r16_round(x), _h(x).numpy())
    # ties go to even: 1 + 2^-11 -> 1, 1 + 3 * 2^-11 -> 1 + 2^-9
    assert orc.r16_round([1 + 2.0 ** -11])[0] == 1.0 and orc.r16_round([1 + 3 * 2.0 ** -11])[0] == 1 + 2.0 ** -9


def _torch_mlp_half(mlp, feat, dirs_per_sample, F=4):
    """The cheaper colour head in torch float64: every matrix-product operand rounded to an FP16
    significand (weights and activations in the forward, the back-propagated gradients at the
    product outputs), biases, the output layer and activations exact."""
    class RoundGrad(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t):
            return t.clone()

        @staticmethod
        def backward(ctx, g):
            return _h(g)

    def rnd(t):  # rounded value, identity gradient
        return t + (_h(t.detach()) - t.detach())
    W = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in mlp.W]
    b = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in mlp.b]
    f = torch.tensor(feat, dtype=torch.float64, requires_grad=True)
    x = torch.cat([f, _pe(dirs_per_sample, F)], dim=-1)
    m1 = RoundGrad.apply(rnd(x) @ rnd(W[0]).T)
    h1 = torch.relu(m1 + b[0])
    m2 = RoundGrad.apply(rnd(h1) @ rnd(W[1]).T)
    h2 = torch.relu(m2 + b[1])
    rgb = torch.sigmoid(torch.nn.functional.linear(h2, W[2], b[2]))
    return rgb, f, W, b


def test_half_mlp_matches_torch(orc):
    rng = np.random.default_rng(43)
    mlp = synth.mlp_weights(rng, bias_std=0.3)
    offs = np.array([0, 7, 7, 20, 41], np.int32)
    S = int(offs[-1])
    dirs = synth.scenes._unit(rng.standard_normal((4, 3))).astype(np.float32)
    feat = rng.standard_normal((S, 12))
    rgb = orc.mlp_forward(mlp, offs, dirs, feat, half=True)
    ray_of = np.repeat(np.arange(4), np.diff(offs))
    trgb, f, W, b = _torch_mlp_half(mlp, feat, dirs[ray_of].astype(np.float64))
    np.testing.assert_allclose(rgb, trgb.detach().numpy(), rtol=1e-12, atol=1e-14)
    g = rng.standard_normal((S, 3))
    (trgb * torch.tensor(g)).sum().backward()
    gf, gW, gb = orc.mlp_backward(mlp, offs, dirs, feat, g, half=True)
    np.testing.assert_allclose(gf, f.grad.numpy(), rtol=1e-10, atol=1e-13)
    for a, t in zip(gW + gb, W + b):
        np.testing.assert_allclose(a, t.grad.numpy(), rtol=1e-10, atol=1e-13)
    # and it stays within FP16 rounding of the exact head (normwise, a few units of 2^-11)
    exact = orc.mlp_forward(mlp, offs, dirs, feat)
    assert np.linalg.norm(rgb - exact) <= 4 * 2.0 ** -11 * np.linalg.norm(exact)
    egf = orc.mlp_backward(mlp, offs, dirs, feat, g)[0]
    assert 0 < np.linalg.norm(gf - egf) <= 20 * 2.0 ** -11 * np.linalg.norm(egf)


@pytest.mark.parametrize("half", [False, True])
def test_mlp_magnitudes(orc, half):
    # an upper bound of every output's absolute value, and equal to it when nothing cancels:
    # non-negative weights, inputs and output gradients (the view encoding is made positive by
    # a direction with all components in (0, pi/16), so every sine and cosine is positive)
    rng = np.random.default_rng(45)
    mlp = synth.mlp_weights(rng, bias_std=0.3)
    offs = np.array([0, 9, 9, 30], np.int32)
    S = int(offs[-1])
    dirs = synth.scenes._unit(rng.standard_normal((3, 3))).astype(np.float32)
    feat = rng.standard_normal((S, 12))
    g = rng.standard_normal((S, 3))
    mr, mf, mW, mb = orc.mlp_magnitudes(mlp, offs, dirs, feat, g, half=half)
    gf, gW, gb = orc.mlp_backward(mlp, offs, dirs, feat, g, half=half)
    assert (mf >= np.abs(gf) * (1 - 1e-12)).all()
    for m, v in zip(mW + mb, gW + gb):
        assert (m >= np.abs(v) * (1 - 1e-12)).all()
    pos = synth.MLPWeights([np.abs(w) for w in mlp.W], [np.abs(b) for b in mlp.b])
    dpos = np.full((3, 3), 0.15, np.float32)
    mr, mf, mW, mb = orc.mlp_magnitudes(pos, offs, dpos, np.abs(feat), np.abs(g), half=half)
    gf, gW, gb = orc.mlp_backward(pos, offs, dpos, np.abs(feat), np.abs(g), half=half)
    np.testing.assert_allclose(mf, gf, rtol=1e-12)
    for m, v in zip(mW + mb, gW + gb):
        np.testing.assert_allclose(m, v, rtol=1e-12, atol=1e-300)
    assert (mr >= 0).all() and np.isfinite(mr).all()


def test_adam_matches_torch_and_skips_zero(orc):
    rng = np.random.default_rng(41)
    n = 1000
    p = rng.standard_normal(n)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=0.05, betas=(0.9, 0.99), eps=1e-8)
    m = np.zeros(n)
    v = np.zeros(n)
    for t in range(1, 4):
        g = rng.standard_normal(n)
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = orc.adam(p, g, m, v, 0.05, 0.9, 0.99, 1e-8, t)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)
    # zero-gradient elements (either sign of zero) are left bit-for-bit untouched
    g = rng.standard_normal(n)
    g[::3] = 0.0
    g[1::7] = -0.0
    p2, m2, v2 = orc.adam(p, g, m, v, 0.05, 0.9, 0.99, 1e-8, 4)
    z = (g == 0)
    assert np.array_equal(p2[z], p[z]) and np.array_equal(m2[z], m[z]) and np.array_equal(v2[z], v[z])
    assert (p2[~z] != p[~z]).all()


def _bf(t):
    return t.to(torch.bfloat16).to(torch.float64)


def test_bf16_rounding_matches_torch(orc):
    rng = np.random.default_rng(42)
    x = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-8, 8, 1000), [0.0, -0.0, 1.0, 3.0]])
    np.testing.assert_array_equal(orc.bf16_round(x), _bf(torch.tensor(x).to(torch.float32).to(torch.float64)).numpy())


def _torch_prop(pw, x, target):
    W = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in pw.W]
    b = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in pw.b]
    a = _bf(torch.tensor(x, dtype=torch.float64))
    L = len(W)
    for l in range(L):
        Wb = W[l] + (_bf(W[l].detach()) - W[l].detach())          # rounded weights, identity gradient
        z = torch.nn.functional.linear(a, Wb, b[l])
        z.register_hook(_bf)                                      # rounded output gradient
        if l + 1 < L:
            h = torch.relu(z)
            a = h + (_bf(h.detach()) - h.detach())
    logp = torch.log_softmax(z, dim=-1)
    loss = -(torch.tensor(target) * logp).sum() / x.shape[0]
    return z, loss, W, b


def test_proposal_matches_torch_bf16(orc):
    rng = np.random.default_rng(43)
    pw = synth.proposal_weights(rng, bias_std=0.1)
    R = 37
    x = rng.random((R, 64)) * 0.3
    tgt = rng.random((R, 64))
    tgt /= tgt.sum(1, keepdims=True)
    lg, pr, H = orc.prop_forward(pw, x)
    z, loss, W, b = _torch_prop(pw, x, tgt)
    np.testing.assert_allclose(lg, z.detach().numpy(), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(pr, torch.softmax(z, -1).detach().numpy(), rtol=1e-12)
    np.testing.assert_allclose(H, -(pr * np.log(pr)).sum(1), rtol=1e-12)
    loss.backward()
    L, gW, gb = orc.prop_backward(pw, x, tgt)
    assert L == pytest.approx(loss.item(), rel=1e-12)
    for a, t in zip(gW + gb, W + b):
        np.testing.assert_allclose(a, t.grad.numpy(), rtol=1e-9, atol=1e-14)


def test_proposal_entropy_uniform_and_ce_gradient(orc):
    pw = synth.proposal_weights(np.random.default_rng(44))
    for w in pw.W[-1:]:
        w[:] = 0.0
    x = np.random.default_rng(45).random((3, 64))
    lg, pr, H = orc.prop_forward(pw, x)
    np.testing.assert_allclose(H, np.log(64), rtol=1e-12)
    # with a zero last layer the bias gradient is sum_r bf16((softmax - p)/R) = sum_r bf16((1/64 - p)/R)
    tgt = np.zeros((3, 64))
    tgt[:, 5] = 1.0
    _, _, gb = orc.prop_backward(pw, x, tgt)
    expect = orc.bf16_round((1.0 / 64 - tgt) / 3).sum(0)
    np.testing.assert_allclose(gb[-1], expect, rtol=1e-12)


def test_histogram(orc):
    offs = np.array([0, 4, 4, 7], np.int32)
    w = np.array([0.1, 0.2, 0.3, 0.4, 1e-6, 1e-6, 1e-6])
    sm = np.array([0.01, 0.26, 0.51, 0.99, 0.1, 0.2, 0.3], np.float32)
    h = orc.histogram(offs, w, sm, B=4, min_mass=1e-4)
    np.testing.assert_allclose(h[0], [0.1, 0.2, 0.3, 0.4])
    np.testing.assert_allclose(h[1], 0.25)   # empty ray: uniform
    np.testing.assert_allclose(h[2], 0.25)   # too little mass: uniform
    np.testing.assert_allclose(h.sum(1), 1.0)


def test_resample_closed_forms(orc):
    R, B, n = 3, 64, 48
    rays = synth.Rays(np.zeros((R, 3), np.float32), np.tile(np.array([0, 0, 1], np.float32), (R, 1)),
                      np.array([1.0, 2.0, 0.5], np.float32), np.array([3.0, 2.5, 4.5], np.float32), np.ones(R, bool))
    p = np.zeros((R, B))
    p[0] = 1.0 / B                # uniform -> s_j = (j + 1/2)/n
    p[1, 17] = 1.0                # one-hot bin b -> s_j = (b + (j + 1/2)/n)/B
    p[2, [3, 40]] = [0.25, 0.75]  # two bins: the first quarter of u lands in bin 3
    out = orc.resample(p, n, rays, voxel=0.01)
    j = np.arange(n)
    sm = out["s_mid"].reshape(R, n)
    np.testing.assert_allclose(sm[0], (j + 0.5) / n, rtol=1e-13)
    np.testing.assert_allclose(sm[1], (17 + (j + 0.5) / n) / B, rtol=1e-13)
    # interval ends at u = k/n; the interval that straddles the empty bins 4..39 spans the gap
    u = np.arange(n + 1) / n
    ends = np.where(u < 0.25, (3 + u / 0.25) / B, (40 + (u - 0.25) / 0.75) / B)
    np.testing.assert_allclose(sm[2], 0.5 * (ends[1:] + ends[:-1]), rtol=1e-12)
    sl = out["s_len"].reshape(R, n)
    np.testing.assert_allclose(sl[2], np.diff(ends), rtol=1e-12)
    # the intervals tile the support of the density: [0,1], bin 17, bins 3..40
    np.testing.assert_allclose(sl.sum(1), [1.0, 1.0 / B, 38.0 / B], rtol=1e-12)
    assert (sl > 0).all() and (np.diff(sm, axis=1) > 0).all()
    span = (rays.t_far - rays.t_near).astype(np.float64)
    np.testing.assert_allclose(out["delta"].reshape(R, n), sl * span[:, None] / 0.01, rtol=1e-13)
    z = out["xyz"].reshape(R, n, 3)[..., 2]
    np.testing.assert_allclose(z, rays.t_near[:, None] + sm * span[:, None], rtol=1e-13)


def test_proposal_coarse_pins(orc):
    # weights of the coarse pass equal the render's weights on the same 64 uniform samples
    # (an independent code path), sum with the final transmittance to one, and a constant
    # field gives the closed form w_k = exp(-k s d)(1 - exp(-s d)).
    wl = synth.config2(R=64, n=32)
    vox = wl.density.voxel_size()
    w, f = orc.proposal_coarse(wl.rays, wl.density, vox)
    smp = synth.uniform_samples(wl.rays, 64, vox)
    o = orc.render_forward(smp, wl.density, srgb=np.zeros((smp.n_samples, 3)), want_w=True)
    hit = wl.rays.hit
    assert (w[~hit] == 0).all() and (f[~hit] == 0).all()
    # float32 sample positions in the render batch vs float64 positions here: tiny differences
    np.testing.assert_allclose(w[hit].ravel(), o["w"], rtol=1e-4, atol=1e-9)
    np.testing.assert_allclose(w[hit].sum(1) + o["T"][hit], 1.0, atol=1e-6)
    np.testing.assert_allclose(f, np.log1p(w / 1e-4), rtol=1e-13)
    const = synth.Grid(np.full((4, 4, 4, 1), 2.0, np.float32), wl.density.xyz_min, wl.density.xyz_max)
    wc, _ = orc.proposal_coarse(wl.rays, const, vox)
    sig = np.log1p(np.exp(2.0 + orc.act_shift()))
    for r in np.nonzero(hit)[0][:5]:
        dl = (float(wl.rays.t_far[r]) - float(wl.rays.t_near[r])) / 64 / vox
        k = np.arange(64)
        np.testing.assert_allclose(wc[r], np.exp(-k * sig * dl) * (1 - np.exp(-sig * dl)), rtol=1e-10)


def test_resample_batch_fallback_and_offsets(orc):
    R, B = 4, 64
    rays = synth.Rays(np.zeros((R, 3), np.float32), np.tile(np.array([1, 0, 0], np.float32), (R, 1)),
                      np.array([1.0, 0.0, 2.0, 0.5], np.float32), np.array([2.0, 0.0, 4.0, 1.5], np.float32),
                      np.array([True, False, True, True]))
    p = np.full((R, B), 1.0 / B)
    p[3] = 0.0
    p[3, 10] = 1.0
    H = np.array([0.5, 0.5, 9.0, 0.1])     # ray 2 above tau -> plain samples; ray 1 misses
    out = orc.resample_batch(p, H, tau=3.0, n_fine=48, n_plain=256, rays=rays, voxel=0.1)
    assert list(np.diff(out["ray_offsets"])) == [48, 0, 256, 48]
    o = out["ray_offsets"]
    j = np.arange(48)
    np.testing.assert_allclose(out["s_mid"][o[0]:o[1]], (j + 0.5) / 48, rtol=1e-13)
    k = np.arange(256)
    np.testing.assert_allclose(out["s_mid"][o[2]:o[3]], (k + 0.5) / 256, rtol=1e-13)
    np.testing.assert_allclose(out["s_len"][o[2]:o[3]], 1 / 256)
    np.testing.assert_allclose(out["delta"][o[2]:o[3]], 2.0 / 256 / 0.1)
    np.testing.assert_allclose(out["s_mid"][o[3]:o[4]], (10 + (j + 0.5) / 48) / 64, rtol=1e-13)
    np.testing.assert_allclose(out["xyz"][o[2]:o[3], 0], 2.0 + 2.0 * (k + 0.5) / 256, rtol=1e-13)
