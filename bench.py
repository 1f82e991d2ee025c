"""Benchmark of the per-ray training step on one MI355X.

Workload (the fine-stage shape): 160^3 density + 160^3x12 feature grids, colour MLP
39-128-128-3, 8192 pinhole rays x 256 samples with a 20-100% live mask per ray (ragged),
distortion weight 0.01, Adam on both grids (zero-gradient skipping) and on the MLP.
One step = gather -> MLP fwd -> render fwd (+distortion) -> loss -> render bwd -> MLP bwd
-> scatter -> Adam x 3, all HIP kernels, replayed from a HIP graph.

Prints ONE JSON line.  `value` = live ray-samples processed per second by the whole step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray-samples/s fused fwd+bwd step (% HBM roofline); proposal vs plain at ≤0.1 dB"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP16_PEAK_TFLOPS = 2500.0   # dense FP16 matrix peak of MI355X
H, C_IN, N_IN = 128, 12, 39   # MLP widths: hidden, feature channels, input columns (12 + 27)


TRAFFIC_FILES = {"mlp_bwd": ("profiles/mlp_bwd_config2_hbm_traffic.md", ["paper_2206_05085_amd/csrc/mlp.hip",
                                                                       "paper_2206_05085_amd/csrc/dvgo_internal.h"]),
                 # render_fwd + render_bwd + brick_scatter, bytes per step
                 "render": ("profiles/render_config2_hbm_traffic.md", ["paper_2206_05085_amd/csrc/render.hip",
                                                                       "paper_2206_05085_amd/csrc/grid.hip",
                                                                       "paper_2206_05085_amd/csrc/dvgo_internal.h"])}


def measured_traffic(stage):
    """HBM bytes per launch of the stage's main kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter's reading for a plain copy), or
    None when there is none or the kernel sources changed since the counters were taken."""
    import hashlib
    spec = TRAFFIC_FILES.get(stage)
    root = os.path.dirname(os.path.abspath(__file__))
    if spec is None or not os.path.exists(os.path.join(root, spec[0])):
        return None
    h = hashlib.sha256()
    for f in spec[1]:
        h.update(open(os.path.join(root, f), "rb").read())
    vals = {}
    for line in open(os.path.join(root, spec[0])):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_sources_sha256") != h.hexdigest():
        return None
    try:
        return int(float(vals["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def mlp_flops_per_sample(backward: bool) -> float:
    """Algorithmic FLOPs of the colour MLP per sample (multiply-add = 2 FLOPs)."""
    fwd = 2 * (N_IN * H + H * H + H * 3)
    if not backward:
        return fwd
    # d hidden2, d hidden1, d features, dW3, dW2, dW1 (no recompute: that is a design choice)
    return 2 * (3 * H + H * H + H * C_IN) + 2 * (3 * H + H * H + H * N_IN)


def unique_vertices(xyz, n, lo, hi):
    """Number of distinct grid vertices touched by the trilinear stencils of xyz."""
    u = (xyz.astype(np.float64) - lo) / (hi - lo) * (n - 1)
    u = np.clip(u, 0, n - 1)
    i0 = np.minimum(np.floor(u).astype(np.int64), n - 2)
    keys = []
    for c in range(8):
        d = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1])
        v = i0 + d
        keys.append((v[:, 0] * n + v[:, 1]) * n + v[:, 2])
    return int(np.unique(np.concatenate(keys)).size)


def cpu_baseline(wl, max_rays=256):
    """FP64 oracle of the same step (gather, MLP, render, loss, backward, scatter, Adam) on
    the first `max_rays` rays of the batch; returns samples/s and what was run."""
    import oracle
    smp = wl.samples
    R = min(max_rays, smp.n_rays)
    offs = smp.ray_offsets[:R + 1].copy()
    S = int(offs[-1])
    sub = type(smp)(offs, smp.xyz[:S], smp.delta[:S], smp.s_mid[:S], smp.s_len[:S])
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    shift = float(np.float32(oracle.act_shift()))
    t0 = time.perf_counter()
    feat = oracle.gather(wl.feat, sub.xyz)
    srgb = oracle.mlp_forward(wl.mlp, offs, wl.rays.dirs[:R], feat)
    o = oracle.render_forward(sub, wl.density, srgb=srgb, shift=shift)
    L, GC, GD = oracle.loss_head(o["rgb"], wl.target[:R], o["D"], wl.dist_weight)
    og = oracle.render_backward(sub, wl.density, GC, GD, None, srgb=srgb, shift=shift)
    gf, gW, gb = oracle.mlp_backward(wl.mlp, offs, wl.rays.dirs[:R], feat, og["grad_srgb"])
    gfeat = oracle.scatter(wl.feat, sub.xyz, gf)
    for p, g in ((wl.density.data, og["grad_density"]), (wl.feat.data, gfeat)):
        oracle.adam(p.reshape(-1), g.reshape(-1), np.zeros(p.size), np.zeros(p.size), 0.1, 0.9, 0.99, 1e-8, 1)
    dt = time.perf_counter() - t0
    return {"value": S / dt, "unit": "ray-samples/s", "cores": threads, "kind": "oracle",
            "sample": f"first {R} of {smp.n_rays} rays ({S} live samples) of the same batch, one full step "
                      f"incl. Adam over both full grids; {dt:.1f} s wall; OpenMP over rays, scatters and "
                      f"MLP backward serial"}


def psnr(a, b):
    mse = float(((a - b) ** 2).mean())
    return 10.0 * np.log10(1.0 / max(mse, 1e-30))


def proposal_leg(steps=1500, batch=8192, pool=65536, n_eval=8192, log=None, cleared=False):
    """Train the proposal network on the grids' own plain-256 weight histograms, tune the
    entropy threshold on held-out rays, and evaluate on a third ray set against plain-256
    (the judge), with a 1024-sample render as the quadrature-limit reference.  At equal
    fine-sample count (48, no fallback) the trained network is also compared with the
    untrained one, the no-network histogram (normalised coarse weights) and uniform-48."""
    import torch

    import synth
    from paper_2206_05085_amd import ops
    from paper_2206_05085_amd import proposal as P

    def say(*a):
        if log:
            print("[proposal]", *a, file=sys.stderr, flush=True)

    wl = synth.config5(R=8, cleared=cleared)
    vox = float(np.float32(wl.density.voxel_size()))
    shift = float(np.float32(ops.act_shift()))
    dens = ops.DeviceGrid(torch.as_tensor(wl.density.data).cuda(), wl.density.xyz_min, wl.density.xyz_max)
    feat_grid = ops.DeviceGrid(torch.as_tensor(wl.feat.data).cuda(), wl.feat.xyz_min, wl.feat.xyz_max)
    mlp = ops.MLPParams([torch.as_tensor(w).cuda() for w in wl.mlp.W], [torch.as_tensor(b).cuda() for b in wl.mlp.b])
    INF = 1e9

    def rays_of(stream, R):
        r = synth.proposal_rays(R, stream)
        return ops.RayBatch.from_arrays(r.origins, r.dirs, r.t_near, r.t_far)

    def plain_batch(rays, n):
        H = torch.zeros(rays.n_rays, device="cuda")
        return P.fine_batch(rays, torch.zeros(rays.n_rays, 64, device="cuda"), H, -1.0, vox, n_plain=n)

    def colour_render(rays, b):
        f = ops.grid_gather(feat_grid, b.xyz)
        rgb_s = ops.mlp_forward(mlp, b.ray_offsets, rays.dirs, f)
        rgb, T, D, _ = ops.render_forward(b, dens, None, rgb_s, act_shift_=shift)
        return rgb, D

    def proposal_render(rays, net, tau, n_fine=48):
        fe, wc = P.coarse(rays, dens, vox, shift)
        _, pr, H = net.forward(fe)
        fb = P.fine_batch(rays, pr, H, tau, vox, n_fine=n_fine)
        rgb, D = colour_render(rays, fb)
        return rgb, D, float((H > tau).float().mean().item()), fb.n_samples, wc

    pw = wl.extra["proposal"]
    net = P.ProposalNet(pw.W, pw.b, lr=1e-3)
    net0 = P.ProposalNet(pw.W, pw.b)        # untrained copy
    train = rays_of(3, pool)
    say("scene", "cleared" if cleared else "fog", ": training features and targets for", pool, "rays")
    feats, targets = P.coarse(train, dens, vox, shift)[0], []
    for c in range(0, pool, batch):
        sub = ops.RayBatch(train.origins[c:c + batch], train.dirs[c:c + batch], train.t_near[c:c + batch],
                           train.t_far[c:c + batch])
        targets.append(P.plain_targets(plain_batch(sub, 256), dens, shift))
    targets = torch.cat(targets)
    tgt_entropy = float(-(targets * torch.log(targets.clamp_min(1e-30))).sum(1).mean().item())
    gen = torch.Generator(device="cpu").manual_seed(5)
    loss0 = None
    t0 = time.perf_counter()
    for it in range(steps):
        idx = torch.randint(0, pool, (batch,), generator=gen).cuda()
        loss = net.train_step(feats[idx].contiguous(), targets[idx].contiguous())
        if it == 0:
            loss0 = float(loss.item())
        if log and it % 500 == 0:
            say("step", it, "cross-entropy", float(loss.item()))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    loss_end = float(loss.item())

    # tau: the fewest samples whose PSNR stays within 0.1 dB of plain-256 on held-out rays
    tune = rays_of(6, n_eval)
    gt_t = colour_render(tune, plain_batch(tune, 1024))[0].cpu().numpy()
    ref_t = psnr(colour_render(tune, plain_batch(tune, 256))[0].cpu().numpy(), gt_t)
    sweep, best = [], None
    for n_fine in (48, 96, 128):
        for tau in (INF, 4.15, 4.1, 4.0, 3.8, 3.5, 3.0, 2.5, 2.0, 1.0, -1.0):
            rgb, _, fb_frac, n_s, _ = proposal_render(tune, net, tau, n_fine)
            ps = psnr(rgb.cpu().numpy(), gt_t)
            sweep.append({"n_fine": n_fine, "tau": tau, "psnr": round(ps, 3), "fallback": round(fb_frac, 4),
                          "samples": n_s})
            if ps >= ref_t - 0.1 and (best is None or n_s < best[2]):
                best = (tau, n_fine, n_s)
    say("tuning sweep (plain-256 psnr %.2f):" % ref_t, sweep)
    tau, n_fine = (best[0], best[1]) if best else (-1.0, 48)

    ev = rays_of(8, n_eval)
    gt = colour_render(ev, plain_batch(ev, 1024))[0].cpu().numpy()
    pb = plain_batch(ev, 256)
    rgb_plain, D_plain = colour_render(ev, pb)
    rgb_prop, D_prop, fb_frac, n_prop, wc = proposal_render(ev, net, tau, n_fine)
    rgb_nf = proposal_render(ev, net, INF)[0]
    rgb_untrained = proposal_render(ev, net0, INF)[0]
    s = wc.sum(1, keepdim=True)
    pn = torch.where(s > 0, wc / s.clamp_min(1e-30), torch.full_like(wc, 1.0 / 64)).contiguous()
    rgb_nonet = colour_render(ev, P.fine_batch(ev, pn, torch.zeros(ev.n_rays, device="cuda"), INF, vox))[0]
    rgb_u48 = colour_render(ev, plain_batch(ev, 48))[0]
    sc = {"proposal": psnr(rgb_prop.cpu().numpy(), gt), "plain256": psnr(rgb_plain.cpu().numpy(), gt)}
    eq = {k: round(psnr(v.cpu().numpy(), gt), 3) for k, v in (("trained", rgb_nf), ("untrained", rgb_untrained),
                                                              ("no_network", rgb_nonet), ("uniform48", rgb_u48))}
    dgap = float(((D_prop - D_plain).abs().mean() / D_plain.abs().mean().clamp_min(1e-30)).item())

    # timing: both paths include their own sample generation (the same resampler kernels)
    zH, zp = torch.zeros(ev.n_rays, device="cuda"), torch.zeros(ev.n_rays, 64, device="cuda")
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    reps = 20
    e[0].record()
    for _ in range(reps):
        fe, _ = P.coarse(ev, dens, vox, shift)
        _, pr2, H2 = net.forward(fe)
        offs = ops.resample_offsets(ev, H2, tau, n_fine=n_fine)
        colour_render(ev, ops.resample(ev, pr2, H2, tau, offs, n_prop, vox, n_fine=n_fine))
    e[1].record()
    for _ in range(reps):
        offs = ops.resample_offsets(ev, zH, -1.0, n_plain=256)
        colour_render(ev, ops.resample(ev, zp, zH, -1.0, offs, pb.n_samples, vox, n_plain=256))
    e[2].record()
    torch.cuda.synchronize()
    ms_prop, ms_plain = e[0].elapsed_time(e[1]) / reps, e[1].elapsed_time(e[2]) / reps
    return {"scene": "config-2 grids with free space cleared" if cleared else "config-2 grids (logit noise fog)",
            "train_steps": steps, "train_rays_per_step": batch, "train_s": round(train_s, 2),
            "ce_first": round(loss0, 4), "ce_last": round(loss_end, 4), "target_entropy": round(tgt_entropy, 4),
            "tau": tau, "n_fine": n_fine, "fallback_frac": round(fb_frac, 4),
            "psnr_vs_1024": {k: round(v, 3) for k, v in sc.items()},
            "psnr_drop_vs_plain256_db": round(sc["plain256"] - sc["proposal"], 3),
            "within_0p1_db": bool(sc["proposal"] >= sc["plain256"] - 0.1),
            "distortion_gap_rel": round(dgap, 4),
            "equal_48_samples_no_fallback_psnr": eq,
            "samples": {"proposal_fine": n_prop, "plain256": pb.n_samples, "coarse_density_only": 64 * ev.n_rays},
            "ms": {"proposal_path": round(ms_prop, 4), "plain256_path": round(ms_plain, 4)},
            "speedup_vs_plain256": round(ms_plain / ms_prop, 3), "eval_rays": n_eval, "tau_sweep": sweep}


def render_sweep_leg(sizes=(8192, 32768, 131072)):
    """The render path alone (density gather, alpha, compositing, distortion forward; the
    backward with per-sample density gradients; binning and the brick-binned density scatter)
    at growing batches of the same scene and ray recipe, autotuned longest-first schedule each:
    its algorithmic HBM rate and fraction of the peak (per-ray walks are latency-bound, so the
    fraction grows as the batch amortises the latency)."""
    import torch
    import synth
    from paper_2206_05085_amd import ops
    from paper_2206_05085_amd.step import TrainStep

    def timed(f, n=10):
        for _ in range(2):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    rows = []
    for R in sizes:
        wl = synth.config2(R=R)
        smp = wl.samples
        S = smp.n_samples
        n = wl.density.data.shape[0]
        lo, hi = float(wl.density.xyz_min[0]), float(wl.density.xyz_max[0])
        print(f"[bench] render sweep: {R} rays, S = {S}", file=sys.stderr, flush=True)
        st = TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                       mlp=(wl.mlp.W, wl.mlp.b), dist_weight=wl.dist_weight)
        b = ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len)
        st.bind(b, wl.rays.dirs, wl.target)
        st.forward()
        st.tune()
        dens = st.grid("density")
        fwd = timed(lambda: ops.render_forward(b, dens, None, st.rgb_s, act_shift_=st.shift, out=(st.rgb, st.T, st.dist),
                                               state=st.state, schedule=st.schedule))
        bwd = timed(lambda: ops.render_backward(b, dens, None, st.rgb_s, st.T, st.state, st.g_rgb, st.g_dist, None,
                                                act_shift_=st.shift, grad_sample_rgb=st.g_rgb_s,
                                                grad_sample_density=st.g_raw, schedule=st.schedule))
        binm = timed(lambda: ops.bin_samples(dens, b.xyz, ws=st.bin_ws))
        sc = timed(lambda: ops.grid_scatter_binned(dens, b.xyz, st.g_raw, st.bin_ws))
        U = unique_vertices(smp.xyz, n, lo, hi)
        byts = (S * 36 + U * 4 + R * 24) + (S * 52 + U * 4 + R * 24) + (S * 20 + U * 8)
        ms = fwd + bwd + sc
        rows.append({"rays": R, "samples": S, "ms": {"render_fwd": round(fwd, 4), "render_bwd": round(bwd, 4),
                                                    "bin": round(binm, 4), "scatter_density": round(sc, 4)},
                     "algorithmic_bytes": int(byts), "GB/s": round(byts / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "schedule": {"waves_per_block": st.schedule.waves_per_block, "grid_waves": st.schedule.grid_waves}})
        del st, b, wl
        torch.cuda.empty_cache()
    return {"kernels": "render_fwd + render_bwd + scatter_density (bytes and rate as in roofline_render; the "
                       "binning, which needs only the points, is timed beside them)", "sizes": rows}


def ragged_leg(R=8192, steps=20, log=None):
    """Unbounded ragged batch (320^3 contracted grids, lognormal lengths 32-1024): render
    forward + backward under three schedules (one wave per ray in batch order; the autotuned
    persistent longest-first launch; one launch per power-of-two length bucket), and the whole
    training step with the tuned schedule replayed from a HIP graph."""
    import torch

    import synth
    from paper_2206_05085_amd import ops
    from paper_2206_05085_amd.step import TrainStep

    def say(*a):
        if log:
            print("[ragged]", *a, file=sys.stderr, flush=True)

    say("generating the 320^3 unbounded workload")
    wl = synth.config3(R=R)
    smp = wl.samples
    S = smp.n_samples
    st = TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                   mlp=(wl.mlp.W, wl.mlp.b), dist_weight=wl.dist_weight, warp=(wl.density.warp, wl.density.warp_b))
    b = ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len)
    st.bind(b, wl.rays.dirs, wl.target)
    st.forward()
    torch.cuda.synchronize()
    order, cls = ops.ray_schedule(b.ray_offsets)
    c = cls.cpu().numpy()
    buckets = []
    for lo, hi in ((1, 1), (2, 2), (3, 4), (5, 8), (9, 16), (17, 63)):
        a, z = c[63 - hi], c[63 - lo + 1]
        if z > a:
            buckets.append(ops.Schedule(order[a:z].contiguous(), 4, 0))

    def time_render(scheds):
        def once():
            for sc in scheds:
                ops.render_forward(b, st.grid("density"), None, st.rgb_s, act_shift_=st.shift,
                                   out=(st.rgb, st.T, st.dist), state=st.state, schedule=sc)
            for sc in scheds:
                ops.render_backward(b, st.grid("density"), None, st.rgb_s, st.T, st.state, st.g_rgb, st.g_dist, None,
                                    act_shift_=st.shift, grad_sample_rgb=st.g_rgb_s, schedule=sc)
        for _ in range(3):
            once()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            once()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    st.loss.zero_()
    ops.loss_head(st.rgb, st.target, st.dist, st.lam, loss=st.loss, grad_rgb=st.g_rgb, grad_dist=st.g_dist)
    ms_plain = time_render([None])
    ms_bucket = time_render(buckets)
    tuned, ms_tune = st.tune(longest_first=True)
    ms_tuned = time_render([tuned])
    # the same samples contracted on the host and looked up on plain grids: the cost of the
    # in-kernel contraction (Eq. 4) in the density lookups of render forward + backward
    b_world = b
    b = ops.SampleBatch.from_arrays(smp.ray_offsets, synth.scenes._contract_inf(smp.xyz.astype(np.float64)),
                                    smp.delta, smp.s_mid, smp.s_len)
    warp_saved = st.warp
    st.warp = (0, 1.0)
    ms_host_contracted = time_render([tuned])
    st.warp = warp_saved
    b = b_world
    say("render fwd+bwd ms: batch order %.3f, per-bucket %.3f, tuned %.3f (wpb %d, grid %d)"
        % (ms_plain, ms_bucket, ms_tuned, tuned.waves_per_block, tuned.grid_waves))
    st.density["g"].zero_()
    st.feat["g"].zero_()
    st.mlp_flat["g"].zero_()
    g = st.capture(warmup=1)
    for _ in range(3):
        g.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / steps
    lens = smp.lengths()
    return {"workload": f"320^3 grids addressed through Eq. 4 (p = inf, b = 1), {R} rays, lognormal lengths 32-1024 (S={S}, max {lens.max()})",
            "render_fwd_bwd_ms": {"one_wave_per_ray_batch_order": round(ms_plain, 4),
                                  "per_length_bucket_launches": round(ms_bucket, 4),
                                  "autotuned_persistent_longest_first": round(ms_tuned, 4)},
            "render_samples_per_s": {"one_wave_per_ray_batch_order": round(S / (ms_plain * 1e-3), 1),
                                     "per_length_bucket_launches": round(S / (ms_bucket * 1e-3), 1),
                                     "autotuned_persistent_longest_first": round(S / (ms_tuned * 1e-3), 1)},
            "tuned_shape": {"waves_per_block": tuned.waves_per_block, "grid_waves": tuned.grid_waves},
            "contraction": {"in_kernel_eq4_p_inf_ms": round(ms_tuned, 4),
                            "host_contracted_points_ms": round(ms_host_contracted, 4)},
            "step_ms_graph": round(ms_step, 4), "step_samples_per_s": round(S / (ms_step * 1e-3), 1),
            "buckets": len(buckets)}


def tv_leg(ops, st, torch, reps=20):
    """Total-variation gradient on the step's grids (section 2): dense over all vertices, and
    sparse over the vertices an eager backward touched.  Weights 1e-5 (density) and 1e-6
    (features) as in section 5.3; Huber threshold 1.0 (the paper does not give one).
    Compulsory bytes: dense 12 B per element (value, gradient in and out); sparse 4 B per
    element (gradient test) + 8 B per element of a touched vertex."""
    st.forward()
    st.backward()          # leaves the step's gradients in the grid .grad buffers
    torch.cuda.synchronize()
    res = {"delta": 1.0, "weights": {"density": 1e-5, "feat": 1e-6}}
    for name, w in (("density", 1e-5), ("feat", 1e-6)):
        g = st.grid(name)
        N = g.data.shape[0] * g.data.shape[1] * g.data.shape[2]
        Cc = g.data.shape[3]
        touched = int((g.grad.reshape(N, Cc) != 0).any(dim=1).sum().item())
        snapshot = g.grad.clone()
        for dense in (True, False):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ops.tv_add_grad(g, w, 1.0, dense)
            e0.record()
            for _ in range(reps):
                ops.tv_add_grad(g, w, 1.0, dense)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            by = 12 * N * Cc if dense else 4 * N * Cc + 8 * touched * Cc
            gbs = by / (ms * 1e-3) / 1e9
            res[f"{name}_{'dense' if dense else 'sparse'}"] = {
                "ms": round(ms, 4), "bytes": by, "GB/s": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
            g.grad.copy_(snapshot)
        res[f"{name}_touched_vertices"] = touched
        res[f"{name}_vertices"] = N
    for d in (st.density, st.feat, st.mlp_flat):
        d["g"].zero_()
    torch.cuda.synchronize()
    return res


def sampler_leg(ops, torch, wl, steps=20, reps=20):
    """GPU sample producer on the step's scene (sections 1 and 3): occupancy update of the
    160^3 density (alpha >= 1e-3 at a half-voxel step, 27-neighbour dilation), then box
    clipping + compaction of the step's rays at a half-voxel step through that mask, then
    training steps (graph replays) on the produced batch.  Compulsory bytes: occupancy 4 B of
    density + 2 B of mask per vertex; producer 24 B per ray + 24 B per emitted sample (mask
    lookups hit L2)."""
    from paper_2206_05085_amd.step import TrainStep
    st = TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                   mlp=(wl.mlp.W, wl.mlp.b), dist_weight=wl.dist_weight)
    nx, ny, nz = wl.density.data.shape[:3]
    N = nx * ny * nz
    voxel = wl.density.voxel_size()
    mask = torch.ones(N, dtype=torch.uint8, device="cuda")

    def timed(f, n):
        f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    occ_ms = timed(lambda: st.update_occupancy(mask, 1e-3, 0.5), reps)   # idempotent on a fixed density
    active = float(mask.float().mean().item())
    og = torch.as_tensor(wl.rays.origins).cuda().contiguous()
    dg = torch.as_tensor(wl.rays.dirs).cuda().contiguous()
    R = og.shape[0]
    res = {"occupancy": {"grid": [nx, ny, nz], "alpha_thr": 1e-3, "delta": 0.5, "active_fraction": round(active, 4),
                         "ms": round(occ_ms, 4), "GB/s": round(6 * N / (occ_ms * 1e-3) / 1e9, 1)}}
    for name, m in (("unmasked", None), ("masked", mask.view(nx, ny, nz))):
        spec = ops.SamplerSpec(wl.density.xyz_min, wl.density.xyz_max, 0.5 * voxel, voxel, 0.0, 4096, m)
        offs = ops.sample_count(spec, og, dg)
        S = int(offs[-1].item())
        out = ops.sample_emit(spec, og, dg, offs, S)

        def produce():
            ops.sample_count(spec, og, dg, ray_offsets=offs)
            ops.sample_emit(spec, og, dg, offs, S, out=out)
        ms = timed(produce, reps)
        res[name] = {"rays": R, "samples": S, "ms": round(ms, 4), "samples_per_s": round(S / (ms * 1e-3), 1),
                     "GB/s": round((24 * R + 24 * S) / (ms * 1e-3) / 1e9, 1)}
        if m is not None:
            st.bind(out, dg, wl.target)
            g = st.capture(warmup=1)
            step_ms = timed(g.replay, steps)
            res[name]["step_ms_graph"] = round(step_ms, 4)
            res[name]["step_samples_per_s"] = round(S / (step_ms * 1e-3), 1)
            res[name]["produce_plus_step_ms"] = round(step_ms + ms, 4)
    res["workload"] = (f"{R} pinhole rays through the 160^3 blob scene, step 0.5 voxel, occupancy from the density "
                       f"(alpha >= 1e-3 at 0.5 voxel)")
    return res


def ff_leg(ops, torch, steps=10, reps=20):
    """Forward-facing scene on the GPU (section 5.3): 256 planes of 384 x 384 in NDC, occupancy
    from the density at the 1-plane step (alpha >= 1e-3), NDC plane sampling of 8192 rays at a
    step of one plane (the paper's setting) through that mask, then graph-replayed training steps
    on the produced batch."""
    import synth
    from paper_2206_05085_amd.step import TrainStep
    wl = synth.config6()
    fx, fy, planes = wl.extra["ndc"]
    nx, ny, nz = wl.density.data.shape[:3]
    st = TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                   mlp=(wl.mlp.W, wl.mlp.b), dist_weight=wl.dist_weight)
    del wl.feat
    mask = torch.ones(nx * ny * nz, dtype=torch.uint8, device="cuda")

    def timed(f, n):
        f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    occ_ms = timed(lambda: st.update_occupancy(mask, 1e-3, 1.0), reps)
    og = torch.as_tensor(wl.rays.origins).cuda().contiguous()
    dg = torch.as_tensor(wl.rays.dirs).cuda().contiguous()
    spec = ops.SamplerSpec(wl.density.xyz_min, wl.density.xyz_max, 1.0, near=1.0, mask=mask.view(nx, ny, nz),
                           ndc=(fx, fy, planes))
    offs = ops.sample_count(spec, og, dg)
    S = int(offs[-1].item())
    batch = ops.sample_emit(spec, og, dg, offs, S)

    def produce():
        ops.sample_count(spec, og, dg, ray_offsets=offs)
        ops.sample_emit(spec, og, dg, offs, S, out=batch)
    prod_ms = timed(produce, reps)
    st.bind(batch, dg, wl.target)
    g = st.capture(warmup=1)
    step_ms = timed(g.replay, steps)
    R = og.shape[0]
    return {"workload": f"{nx}x{ny}x{nz} NDC volume (density + 12-ch features + MLP), {R} forward-facing rays, "
                        f"step 1 plane, occupancy alpha >= 1e-3",
            "active_fraction": round(float(mask.float().mean().item()), 4), "occupancy_ms": round(occ_ms, 4),
            "samples": S, "candidates": R * planes, "producer_ms": round(prod_ms, 4),
            "step_ms_graph": round(step_ms, 4), "step_samples_per_s": round(S / (step_ms * 1e-3), 1)}


def f16_head_leg(ops, torch, wl, batch, steps=30):
    """The cheaper colour head (FP16 matrix operands, one product per product) in the same
    config-2 step: colour-head stage times and the graph-replayed step.  Reduced precision by
    design (its own tolerance), so it is reported beside the FP32-grade headline, not as it."""
    from paper_2206_05085_amd.step import TrainStep
    st = TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                   mlp=(wl.mlp.W, wl.mlp.b), dist_weight=wl.dist_weight, mlp_precision=ops.MLP_F16)
    st.bind(batch, wl.rays.dirs, wl.target)

    def timed(f, n):
        for _ in range(3):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    st.forward()
    st.backward()
    fwd = timed(lambda: ops.mlp_forward(st.mlp, batch.ray_offsets, st.dirs, st.feat_s, rgb=st.rgb_s, ws=st.mlp_ws), 10)
    bwd = timed(lambda: ops.mlp_backward(st.mlp, batch.ray_offsets, st.dirs, st.feat_s, st.g_rgb_s,
                                         grad_feat=st.g_feat_s, ws=st.mlp_ws), 10)
    for d in (st.density, st.feat, st.mlp_flat):
        d["g"].zero_()
    g = st.capture(warmup=1)
    step = timed(g.replay, steps)
    S = batch.n_samples
    return {"mlp_fwd_ms": round(fwd, 4), "mlp_bwd_ms": round(bwd, 4), "step_ms_graph": round(step, 4),
            "step_samples_per_s": round(S / (step * 1e-3), 1),
            "mlp_bwd_tflops_algorithmic": round(S * mlp_flops_per_sample(True) / (bwd * 1e-3) / 1e12, 2),
            "precision": "FP16 matrix operands (11-bit significands), FP32 accumulation"}


def stored_composite(raw, delta, srgb, m, l, shift, hit, R):
    """Compositing and the distortion loss as plain PyTorch operations on rays of one length N,
    the way an autograd graph keeps them: alpha = 1 - exp(-softplus(raw + shift) delta), exclusive
    cumulative product for the transmittance, weights, colour over a white background, and Eq. 2
    through cumulative sums.  raw, delta: [Rh*N]; srgb: [Rh*N, 3]; m, l: [Rh, N] (normalised
    midpoints and lengths); hit: indices of the Rh rays with samples among R.  Returns rgb [R, 3]
    and D [R] (rays without samples: the background, D = 0).  Used as the stored-intermediates
    baseline of the memory measurement."""
    import torch
    import torch.nn.functional as F
    Rh, N = m.shape
    a = -torch.expm1(-F.softplus(raw + shift) * delta).view(Rh, N)
    P = torch.cumprod(1.0 - a, 1)
    w = a * torch.cat([torch.ones(Rh, 1, device=a.device, dtype=a.dtype), P[:, :-1]], 1)
    rgb_h = (w.unsqueeze(-1) * srgb.view(Rh, N, 3)).sum(1) + P[:, -1:]
    W, Q = torch.cumsum(w, 1) - w, torch.cumsum(w * m, 1) - w * m
    D_h = 2.0 * (w * (m * W - Q)).sum(1) + (w * w * l).sum(1) / 3.0
    rgb = torch.ones(R, 3, device=a.device, dtype=a.dtype).index_copy(0, hit, rgb_h)
    D = torch.zeros(R, device=a.device, dtype=a.dtype).index_copy(0, hit, D_h)
    return rgb, D


def recompute_memory_leg(reps=5):
    """Config 4 (the config-2 grids, 16384 rays x 512 samples): device memory and time of one
    render + distortion forward and backward through the hand-written autograd Function, which
    keeps one 16-byte checkpoint per ray and 64-sample chunk and recomputes the rest in the
    backward, against the same loss under plain PyTorch autograd, which keeps its per-sample
    tensors (alpha, transmittance, weights, the prefix sums of Eq. 2) for the backward.  The
    density lookup is the same gather Function in both and the per-sample colours are inputs,
    so the two differ only in what the compositing and the distortion loss keep.  Memory is the
    peak allocated above the resident inputs, gradients included."""
    import torch
    import synth
    from paper_2206_05085_amd import autograd as ag, ops
    wl = synth.config4()
    smp = wl.samples
    R, S = smp.n_rays, smp.n_samples
    lens = np.diff(smp.ray_offsets)
    N = int(lens.max())
    if not np.all((lens == 0) | (lens == N)):
        raise RuntimeError("the stored-intermediates form needs rays of one length (or none)")
    batch = ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", torch.float32)
    dens = dev(wl.density.data).requires_grad_(True)
    srgb = dev(np.random.default_rng(7).random((S, 3))).requires_grad_(True)
    tgt = dev(wl.target)
    box = (tuple(wl.density.xyz_min), tuple(wl.density.xyz_max))
    shift = float(np.float32(ops.act_shift()))
    lam = wl.dist_weight
    Rh = S // N  # rays with samples; the others (missing the box) show the background
    hit = torch.as_tensor(np.flatnonzero(lens), device="cuda")
    m, l = batch.s_mid.view(Rh, N), batch.s_len.view(Rh, N)

    def recompute():
        rgb, _, D = ag.render(dens, srgb, batch, box, grid_color=False, act_shift=shift)
        (((rgb - tgt) ** 2).mean() + lam * D.mean()).backward()
        return rgb, D

    def stored():
        raw = ag.gather(dens, batch.xyz, box)[:, 0]
        rgb, D = stored_composite(raw, batch.delta, srgb, m, l, shift, hit, R)
        (((rgb - tgt) ** 2).mean() + lam * D.mean()).backward()
        return rgb, D

    res = {}
    for name, f in (("recompute", recompute), ("stored", stored)):
        dens.grad = srgb.grad = None
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        rgb, D = f()
        torch.cuda.synchronize()
        peak = torch.cuda.max_memory_allocated() - base
        out = (rgb.detach().clone(), D.detach().clone(), dens.grad.clone(), srgb.grad.clone())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            dens.grad = srgb.grad = None
            f()
        e1.record()
        torch.cuda.synchronize()
        res[name] = (peak, e0.elapsed_time(e1) / reps, out)
    rel = lambda x, y: float((x - y).norm() / y.norm().clamp_min(1e-30))
    (pr, tr, a), (ps, ts, b) = res["recompute"], res["stored"]
    return {"rays": R, "rays_with_samples": Rh, "samples": S, "recompute_peak_mb": round(pr / 1e6, 1), "stored_peak_mb": round(ps / 1e6, 1),
            "recompute_ms": round(tr, 3), "stored_ms": round(ts, 3),
            "stored_form": "PyTorch autograd of the same compositing and Eq. 2 distortion (per-sample tensors kept)",
            "rel_diff": {"rgb": rel(a[0], b[0]), "dist": rel(a[1], b[1]), "grad_density": rel(a[2], b[2]),
                         "grad_rgb": rel(a[3], b[3])}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=8192)
    ap.add_argument("--rays", type=int, default=8192)
    ap.add_argument("--no-proposal", action="store_true")
    ap.add_argument("--no-recompute-memory", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-render-sweep", action="store_true")
    ap.add_argument("--proposal-steps", type=int, default=1500)
    ap.add_argument("--no-tv", action="store_true")
    ap.add_argument("--no-sampler", action="store_true")
    ap.add_argument("--no-ff", action="store_true")
    ap.add_argument("--no-f16", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="end with a plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is described in "
                                   "DESIGN.md but not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import synth
    from paper_2206_05085_amd import ops
    from paper_2206_05085_amd.step import TrainStep

    torch.cuda.set_device(0)
    print("[bench] generating workload", file=sys.stderr, flush=True)
    wl = synth.config2(R=args.rays)
    smp = wl.samples
    R, S = smp.n_rays, smp.n_samples
    n = wl.density.data.shape[0]
    lo, hi = float(wl.density.xyz_min[0]), float(wl.density.xyz_max[0])
    st = TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                   mlp=(wl.mlp.W, wl.mlp.b), dist_weight=wl.dist_weight)
    batch = ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len)
    st.bind(batch, wl.rays.dirs, wl.target)
    torch.cuda.synchronize()
    # render kernels' launch shape: longest rays first, waves per block and grid size picked by
    # the library's autotuner on this batch (outside the timed region, like the capture)
    st.tune()
    torch.cuda.synchronize()

    # ---- per-stage times (eager, events on the launching stream)
    print("[bench] stage timing", file=sys.stderr, flush=True)
    stages = {
        # the step's forward: feature lookup inside the colour head (the separate gather and
        # forward are timed too, for comparison; the step does not run them)
        "gather": lambda: ops.grid_gather(st.grid("feat"), batch.xyz, out=st.feat_s),
        "mlp_fwd": lambda: ops.mlp_forward(st.mlp, batch.ray_offsets, st.dirs, st.feat_s, rgb=st.rgb_s, ws=st.mlp_ws),
        "mlp_fwd_gather": lambda: ops.mlp_forward_gather(st.mlp, batch.ray_offsets, st.dirs, st.grid("feat"), batch.xyz,
                                                         feat_out=st.feat_s, rgb=st.rgb_s, ws=st.mlp_ws),
        "render_fwd": lambda: ops.render_forward(batch, st.grid("density"), None, st.rgb_s, act_shift_=st.shift,
                                                 out=(st.rgb, st.T, st.dist), state=st.state, schedule=st.schedule),
        "loss": lambda: ops.loss_head(st.rgb, st.target, st.dist, st.lam, loss=st.loss, grad_rgb=st.g_rgb,
                                      grad_dist=st.g_dist),
        "bin": lambda: ops.bin_samples(st.grid("density"), batch.xyz, ws=st.bin_ws),
        "render_bwd": lambda: ops.render_backward(batch, st.grid("density"), None, st.rgb_s, st.T, st.state, st.g_rgb,
                                                  st.g_dist, None, act_shift_=st.shift, grad_sample_rgb=st.g_rgb_s,
                                                  grad_sample_density=st.g_raw, schedule=st.schedule),
        "scatter_density": lambda: ops.grid_scatter_binned(st.grid("density"), batch.xyz, st.g_raw, st.bin_ws),
        "mlp_bwd": lambda: ops.mlp_backward(st.mlp, batch.ray_offsets, st.dirs, st.feat_s, st.g_rgb_s,
                                            grad_feat=st.g_feat_s, ws=st.mlp_ws),
        "scatter": lambda: ops.grid_scatter(st.grid("feat"), batch.xyz, st.g_feat_s),
        "adam": st.optimise,
    }
    for _ in range(3):
        for f in stages.values():
            f()
    torch.cuda.synchronize()
    reps = 10
    stage_ms = {}
    for name, f in stages.items():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if name == "adam":
            # Adam zeroes the gradients it consumes, and a zero gradient skips its group: each
            # timed update gets one backward's gradients first (untimed; the events bracket the
            # update alone on the same stream)
            tot = 0.0
            for _ in range(reps):
                for pre in ("render_bwd", "scatter_density", "mlp_bwd", "scatter"):
                    stages[pre]()
                e0.record()
                f()
                e1.record()
                torch.cuda.synchronize()
                tot += e0.elapsed_time(e1)
            stage_ms[name] = tot / reps
            continue
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        stage_ms[name] = e0.elapsed_time(e1) / reps
    # restore a consistent state: grads were accumulated by the repeated stage calls
    for d in (st.density, st.feat, st.mlp_flat):
        d["g"].zero_()

    # ---- the timed step
    print("[bench] capture + timed steps", file=sys.stderr, flush=True)
    use_graph = not args.no_graph
    if use_graph:
        g = st.capture(warmup=1)
        run = g.replay
    else:
        run = st.step
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    loss = float(st.loss.item())
    value = S / (ms * 1e-3)

    # ---- roofline of the dominant stage
    U = unique_vertices(smp.xyz, n, lo, hi)
    b_render = {"render_fwd": S * 36 + U * 4 + R * 24, "render_bwd": S * 52 + U * 4 + R * 24,
                "scatter_density": S * 20 + U * 8}
    mlp_bwd_flops = S * mlp_flops_per_sample(True)
    mlp_fwd_flops = S * mlp_flops_per_sample(False)
    dom = max(stage_ms, key=stage_ms.get)
    if dom in ("mlp_bwd", "mlp_fwd"):
        fl = mlp_bwd_flops if dom == "mlp_bwd" else mlp_fwd_flops
        ach = fl / (stage_ms[dom] * 1e-3) / 1e12
        # the colour MLP runs on FP16 matrix cores with split (hi + lo) operands: three FP16
        # products per FP32-grade product, so FP16_PEAK / 3 is the ceiling of this formulation
        roof = {"kernel": dom, "bound": "mfma", "achieved": round(ach, 2), "peak": FP16_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP16_PEAK_TFLOPS, 4), "traffic": measured_traffic(dom),
                "algorithmic": f"{fl / S:.0f} FLOP/sample x {S} samples",
                "mfma_dtype": "f16 (split hi/lo, 3 products)",
                "frac_of_split_ceiling": round(ach / (FP16_PEAK_TFLOPS / 3), 4)}
    else:
        by = b_render.get(dom, 0)
        ach = by / (stage_ms[dom] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}
    rt = stage_ms["render_fwd"] + stage_ms["render_bwd"] + stage_ms["scatter_density"]
    r_bytes = b_render["render_fwd"] + b_render["render_bwd"] + b_render["scatter_density"]
    roof_render = {"kernels": "render_fwd + render_bwd + scatter_density (density gather, alpha, compositing, "
                              "distortion, per-sample density gradient, brick scatter)",
                   "bound": "hbm", "achieved": round(r_bytes / (rt * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                   "unit": "GB/s", "frac": round(r_bytes / (rt * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "algorithmic_bytes": int(r_bytes), "unique_density_vertices": U}
    # bytes the same kernels move past L2 (counter runs): the random trilinear gathers fetch whole
    # lines for 4-byte values, so this exceeds the algorithmic bytes several times
    r_traffic = measured_traffic("render")
    roof_render["traffic"] = r_traffic
    if r_traffic:
        roof_render["traffic_GB/s"] = round(r_traffic / (rt * 1e-3) / 1e9, 1)
        roof_render["traffic_frac"] = round(r_traffic / (rt * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    out = {"metric": METRIC, "value": round(value, 1), "unit": "ray-samples/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"fine-stage step: 160^3 density + 160^3x12 features, colour MLP 39-128-128-3, "
                                  f"{R} pinhole rays x 256 samples 20-100% live (S={S}), lambda_dist=0.01, "
                                  f"Adam on grids (skip zero grads) + MLP",
                      "rays": R, "live_samples": S, "graph": use_graph, "parallelism": "single GPU",
                      "render_schedule": {"order": "longest first", "waves_per_block": st.schedule.waves_per_block,
                                          "grid_waves": st.schedule.grid_waves}},
           "roofline": roof, "roofline_render": roof_render,
           "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()}, "loss": loss, "wall_s": round(wall, 3)}
    if not args.no_tv:
        print("[bench] total-variation gradients", file=sys.stderr, flush=True)
        out["tv"] = tv_leg(ops, st, torch)
    if not args.no_f16:
        print("[bench] cheaper colour head (FP16 operands)", file=sys.stderr, flush=True)
        out["cheaper_colour_head"] = f16_head_leg(ops, torch, wl, batch)
    if not args.no_sampler:
        print("[bench] GPU sample producer + occupancy mask", file=sys.stderr, flush=True)
        out["sampler"] = sampler_leg(ops, torch, wl)
    if not args.no_ff:
        print("[bench] forward-facing NDC volume: occupancy, plane sampling, step", file=sys.stderr, flush=True)
        out["forward_facing"] = ff_leg(ops, torch)
        torch.cuda.empty_cache()
    if not args.no_render_sweep:
        out["render_batch_sweep"] = render_sweep_leg()
        torch.cuda.empty_cache()
    if not args.no_recompute_memory:
        print("[bench] config 4: recompute-in-backward memory vs stored intermediates", file=sys.stderr, flush=True)
        out["recompute_memory"] = recompute_memory_leg()
        torch.cuda.empty_cache()
    if not args.no_ragged:
        print("[bench] ragged unbounded batch: schedules", file=sys.stderr, flush=True)
        out["ragged"] = ragged_leg(log=True)
    if not args.no_proposal:
        print("[bench] proposal stage: train, tune, evaluate", file=sys.stderr, flush=True)
        out["proposal"] = {
            "cleared_free_space": proposal_leg(steps=args.proposal_steps, log=True, cleared=True),
            "config2_grids_with_fog": proposal_leg(steps=args.proposal_steps, log=True, cleared=False)}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_rays)
    if args.calib_copy_mib > 0:
        # a plain copy of known size for the FETCH_SIZE / WRITE_SIZE calibration: reads and writes
        # exactly calib_copy_mib MiB (one torch copy kernel), the last dispatch of the process
        src = torch.ones(args.calib_copy_mib * 2**18, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
