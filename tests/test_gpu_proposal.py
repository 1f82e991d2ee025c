"""Parity of the proposal-stage kernels with the oracle, and a short training run showing
what the trained network gains."""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import FWD, GRAD, close

pytestmark = pytest.mark.gpu

# bfloat16 network outputs (8-bit significands, so values carry ~2^-9 relative rounding per layer):
# normwise 1e-2, elementwise 2e-2
BF = dict(rtol=1e-2, floor=1e-2)


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_05085_amd as p
    p.lib()
    from paper_2206_05085_amd import ops, proposal
    return ops, proposal


def say(*a):
    print("[case]", *a, flush=True)


def T(a, dt=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)


def dgrid(ops, g):
    return ops.DeviceGrid(T(g.data), g.xyz_min, g.xyz_max)


def drays(ops, rays):
    return ops.RayBatch.from_arrays(rays.origins, rays.dirs, rays.t_near, rays.t_far)


@pytest.fixture(scope="module")
def scene():
    wl = synth.config5(R=1000, n=64)
    return wl


def test_coarse_pass(pk, scene):
    ops, prop = pk
    wl = scene
    vox = wl.density.voxel_size()
    shift = float(np.float32(ops.act_shift()))
    say("proposal coarse pass, R =", wl.rays.origins.shape[0])
    feat, w = prop.coarse(drays(ops, wl.rays), dgrid(ops, wl.density), vox, shift)
    torch.cuda.synchronize()
    ow, of = oracle.proposal_coarse(wl.rays, wl.density, float(np.float32(vox)), shift=shift)
    close(w.cpu().numpy(), ow, **FWD, name="coarse weights")
    close(feat.cpu().numpy(), of, **FWD, name="coarse features")


def test_proposal_forward_backward(pk):
    ops, prop = pk
    rng = np.random.default_rng(70)
    pw = synth.proposal_weights(rng, bias_std=0.1)
    R = 777
    x = (rng.random((R, 64)) * 3.0).astype(np.float32)
    tgt = rng.random((R, 64))
    tgt[:, rng.integers(0, 64, 10)] += 3.0
    tgt = (tgt / tgt.sum(1, keepdims=True)).astype(np.float32)
    say("proposal forward/backward, R =", R)
    net = prop.ProposalNet(pw.W, pw.b)
    lg, pr, H = net.forward(T(x))
    loss = ops.proposal_backward(net.params, T(x), T(tgt))
    torch.cuda.synchronize()
    olg, opr, oH = oracle.prop_forward(pw, x)
    close(lg.cpu().numpy(), olg, **BF, name="logits")
    # softmax and entropy of the GPU's own logits
    sp, sH = oracle.softmax_entropy(lg.cpu().numpy())
    close(pr.cpu().numpy(), sp, **FWD, name="softmax")
    close(H.cpu().numpy(), sH, **FWD, name="entropy")
    oL, ogW, ogb = oracle.prop_backward(pw, x, tgt.astype(np.float64))
    close(loss.cpu().numpy(), [oL], rtol=1e-3, floor=1e-3, name="cross-entropy")
    for i in range(4):
        close(net.params.gW[i].cpu().numpy(), ogW[i], **BF, name=f"grad W{i}")
        close(net.params.gb[i].cpu().numpy(), ogb[i], **BF, name=f"grad b{i}")


def test_histogram_targets(pk, scene):
    ops, prop = pk
    wl = scene
    smp = wl.samples   # 256 uniform samples per ray
    shift = float(np.float32(ops.act_shift()))
    say("histogram targets from a plain 256-sample render")
    b = ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len)
    w = torch.empty(smp.n_samples, device="cuda")
    ops.render_forward(b, dgrid(ops, wl.density), None, None, act_shift_=shift, want_dist=False, sample_w=w,
                       density_only=True)
    h = ops.histogram(b.ray_offsets, w, b.s_mid)
    torch.cuda.synchronize()
    o = oracle.render_forward(smp, wl.density, srgb=np.zeros((smp.n_samples, 3)), shift=shift, want_w=True)
    close(w.cpu().numpy(), o["w"], **FWD, name="sample weights")
    close(h.cpu().numpy(), oracle.histogram(smp.ray_offsets, w.cpu().numpy().astype(np.float64), smp.s_mid), **FWD,
          name="histogram")


def test_resample(pk, scene):
    ops, prop = pk
    wl = scene
    rng = np.random.default_rng(71)
    R = wl.rays.origins.shape[0]
    p = rng.random((R, 64)) ** 4
    p[:, rng.integers(0, 64, 20)] = 0.0           # zero-mass bins are skipped
    p = (p / p.sum(1, keepdims=True)).astype(np.float32)
    H = (rng.random(R) * 4.2).astype(np.float32)
    tau = float(np.float32(3.5))
    vox = float(np.float32(wl.density.voxel_size()))
    say("resample, R =", R)
    rays = drays(ops, wl.rays)
    fb = prop.fine_batch(rays, T(p), T(H), tau, vox)
    torch.cuda.synchronize()
    o = oracle.resample_batch(p.astype(np.float64), H.astype(np.float64), tau, 48, 256, wl.rays, vox)
    assert np.array_equal(fb.ray_offsets.cpu().numpy(), o["ray_offsets"])
    # An interval end F^-1(u) is conditioned by 1/(64 p_b) in its bin b: a float32 CDF (a
    # 64-term prefix sum) and u = j/n carry an error of a few units of 2^-24 in u, which moves
    # the end by that over (64 p_b).  Allow 16 units per end.
    offs = o["ray_offsets"]
    ray = np.repeat(np.arange(R), np.diff(offs))
    jj = np.arange(offs[-1]) - offs[ray]
    n_r = np.diff(offs)[ray]
    pd = p.astype(np.float64)
    cdf = np.concatenate([np.zeros((R, 1)), np.cumsum(pd, axis=1)], axis=1)

    def end_cond(u_frac):
        tot = cdf[ray, -1]
        u = u_frac * tot
        b = np.array([np.searchsorted(cdf[r, 1:], x, side="right") for r, x in zip(ray, u)])
        last = np.array([np.nonzero(pd[r] > 0)[0][-1] for r in ray])
        b = np.where(u >= tot, last, np.minimum(b, 63))
        return 16 * 2.0 ** -24 / (64 * np.maximum(pd[ray, b], 1e-30))

    fine = n_r == 48
    c0 = np.where(fine, end_cond(jj / np.maximum(n_r, 1)), 0.0)
    c1 = np.where(fine, end_cond((jj + 1) / np.maximum(n_r, 1)), 0.0)
    span = (wl.rays.t_far - wl.rays.t_near).astype(np.float64)[ray]
    close(fb.s_mid.cpu().numpy(), o["s_mid"], **FWD, name="s_mid", slack=0.5 * (c0 + c1))
    close(fb.s_len.cpu().numpy(), o["s_len"], **FWD, name="s_len", slack=c0 + c1)
    close(fb.delta.cpu().numpy(), o["delta"], **FWD, name="delta", slack=(c0 + c1) * span / vox)
    close(fb.xyz.cpu().numpy(), o["xyz"], **FWD, name="xyz", slack=np.repeat(0.5 * (c0 + c1) * span, 3))


@pytest.mark.parametrize("n_extra,tau", [(0, 1e9), (32, 1e9), (48, 3.5)])
def test_resample_guarded(pk, scene, n_extra, tau):
    # fed the GPU's own coarse weights and probabilities (float32), both sides take the same
    # integer decisions: counts and offsets bit for bit; positions within the forward bar
    ops, prop = pk
    wl = scene
    rng = np.random.default_rng(72)
    vox = float(np.float32(wl.density.voxel_size()))
    shift = float(np.float32(ops.act_shift()))
    rays = drays(ops, wl.rays)
    say("guarded resampling, R =", rays.n_rays, "n_extra =", n_extra, "tau =", tau)
    _, w = prop.coarse(rays, dgrid(ops, wl.density), vox, shift)
    pw = synth.proposal_weights(rng, bias_std=0.1)
    net = prop.ProposalNet(pw.W, pw.b)
    feat = torch.log1p(w / 1e-4).contiguous()
    _, pr, H = net.forward(feat)
    fb = prop.guarded_batch(rays, pr, w, H, tau, vox, n_base=4, n_extra=n_extra, w_min=1e-4)
    counts = ops.resample_guarded_offsets(rays, pr, w, H, tau, 4, n_extra, 1e-4)[1]
    torch.cuda.synchronize()
    o = oracle.resample_guarded(pr.cpu().numpy(), w.cpu().numpy(), H.cpu().numpy(), np.float32(tau), 4, n_extra,
                                1e-4, wl.rays, vox)
    assert np.array_equal(counts.cpu().numpy(), o["counts"])
    assert np.array_equal(fb.ray_offsets.cpu().numpy(), o["ray_offsets"])
    occ = (o["counts"] > 0).sum(1)
    say("samples:", int(o["ray_offsets"][-1]), "; rays with samples:", int((occ > 0).sum()), "of", rays.n_rays)
    assert 0 < o["ray_offsets"][-1] < 256 * rays.n_rays
    close(fb.s_mid.cpu().numpy(), o["s_mid"], **FWD, name="s_mid")
    close(fb.s_len.cpu().numpy(), o["s_len"], **FWD, name="s_len")
    close(fb.delta.cpu().numpy(), o["delta"], **FWD, name="delta")
    close(fb.xyz.cpu().numpy(), o["xyz"], **FWD, name="xyz")


@pytest.mark.timeout(600)
def test_trained_network_gain(pk):
    """A short training run on the grids' own rendered histograms, cleared scene: the
    cross-entropy falls; the trained network's placement beats the untrained network and uniform
    placement at an equal budget of 48 interval-resampled samples per ray; with guarded resampling
    (coverage from the coarse pass, extras from the network) the trained network's extras beat the
    normalised coarse weights (the method without the network), uniform extras and the untrained
    network at an equal layout; and guarded resampling reaches plain-256's PSNR within 0.1 dB with
    no fallback and fewer samples than plain-256."""
    import bench
    say("proposal training + evaluation, cleared scene")
    r = bench.proposal_leg(steps=400, pool=16384, n_eval=4096, cleared=True)
    say({k: r[k] for k in ("ce_first", "ce_last", "target_entropy", "equal_48_interval_resampling_psnr",
                           "psnr_plain256_vs_1024", "guarded")})
    assert r["ce_last"] < r["ce_first"] - 0.1
    eq = r["equal_48_interval_resampling_psnr"]
    assert eq["trained"] > eq["untrained"] + 1.0
    assert eq["trained"] > eq["uniform48"] + 1.0
    g = r["guarded"]
    gain = g["equal_layout_psnr_by_extras"]
    assert gain["trained"] > gain["no_network"]
    assert gain["trained"] > gain["uniform"] + 1.0 and gain["trained"] > gain["untrained"] + 1.0
    assert g["found_within_0p1_db"] and g["psnr_drop_vs_plain256_db"] <= 0.1
    assert g["fallback_frac"] == 0.0 and g["samples"] < g["plain256_samples"]
