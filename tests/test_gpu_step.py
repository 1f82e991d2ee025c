"""Whole-step parity, HIP-graph replays, autograd Functions, and the finite-difference
check of the hand-written backward at the 16384-ray x 512-sample shape."""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import FWD, GRAD, close, close_after_adam

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_05085_amd as p
    p.lib()
    from paper_2206_05085_amd import autograd, ops, step
    return ops, autograd, step


def say(*a):
    print("[case]", *a, flush=True)


def T(a, dt=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)


def oracle_step_grads(wl, shift):
    """FP64 gradients of the whole loss (gather -> MLP -> render -> loss) w.r.t. density,
    features and MLP parameters, plus the loss."""
    smp = wl.samples
    feat = oracle.gather(wl.feat, smp.xyz)
    srgb = oracle.mlp_forward(wl.mlp, smp.ray_offsets, wl.rays.dirs, feat)
    o = oracle.render_forward(smp, wl.density, srgb=srgb, shift=shift)
    L, GC, GD = oracle.loss_head(o["rgb"], wl.target, o["D"], wl.dist_weight)
    og = oracle.render_backward(smp, wl.density, GC, GD, None, srgb=srgb, shift=shift)
    gf, gW, gb = oracle.mlp_backward(wl.mlp, smp.ray_offsets, wl.rays.dirs, feat, og["grad_srgb"])
    gfeat = oracle.scatter(wl.feat, smp.xyz, gf)
    return L, o, og["grad_density"], gfeat, gW, gb


def make_step(step_mod, wl):
    from paper_2206_05085_amd import ops
    st = step_mod.TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                            mlp=(wl.mlp.W, wl.mlp.b), dist_weight=wl.dist_weight)
    smp = wl.samples
    b = ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len)
    st.bind(b, wl.rays.dirs, wl.target)
    return st


def test_whole_step_gradients(pkg):
    ops, _, step = pkg
    wl = synth.config2(R=384, n=64, mlp_bias_std=0.2)
    say("whole step, 64^3 grids, 384 pinhole rays, S =", wl.samples.n_samples)
    st = make_step(step, wl)
    st.forward()
    st.backward()
    torch.cuda.synchronize()
    shift = float(np.float32(st.shift))
    L, o, gd, gfeat, gW, gb = oracle_step_grads(wl, shift)
    close(st.rgb.cpu().numpy(), o["rgb"], **FWD, name="rgb")
    close(st.dist.cpu().numpy(), o["D"], **FWD, name="distortion")
    close(st.loss.cpu().numpy(), [L], **FWD, name="loss")
    close(st.density["g"].cpu().numpy(), gd, **GRAD, name="grad density")
    # A hidden unit whose pre-activation sits within float32 rounding of its ReLU kink may
    # switch side between float32 and float64; both are valid there.  The oracle computes,
    # per element, how much each gradient moves when such a unit switches (the slack).
    smp = wl.samples
    feat = oracle.gather(wl.feat, smp.xyz)
    srgb = oracle.mlp_forward(wl.mlp, smp.ray_offsets, wl.rays.dirs, feat)
    o2 = oracle.render_forward(smp, wl.density, srgb=srgb, shift=shift)
    _, GC, GD = oracle.loss_head(o2["rgb"], wl.target, o2["D"], wl.dist_weight)
    g_srgb = oracle.render_backward(smp, wl.density, GC, GD, None, srgb=srgb, shift=shift)["grad_srgb"]
    sf, sW, sb = oracle.mlp_kink_slack(wl.mlp, smp.ray_offsets, wl.rays.dirs, feat, g_srgb)
    slack_grid = oracle.scatter(wl.feat, smp.xyz, sf)   # every vertex weight is <= 1, so this bounds the move
    say("kink slack: max feature-grid slack", float(np.abs(slack_grid).max()))
    close(st.feat["g"].cpu().numpy(), gfeat, **GRAD, name="grad features", slack=np.abs(slack_grid))
    for i in range(3):
        close(st.mlp.gW[i].cpu().numpy(), gW[i], **GRAD, name=f"grad W{i + 1}", slack=sW[i])
        close(st.mlp.gb[i].cpu().numpy(), gb[i], **GRAD, name=f"grad b{i + 1}", slack=sb[i])


def test_graph_replays_match_eager(pkg):
    # Two identical steps: one runs eagerly, the other replays a captured graph, with eager
    # work and synchronisations between replays; every replay is checked against eager.
    ops, _, step = pkg
    wl = synth.config2(R=256, n=48)
    say("graph replay vs eager, 48^3, 256 rays")
    a, b = make_step(step, wl), make_step(step, wl)
    a.step()  # both take one eager step first; capturing records but does not execute
    b.step()
    g = b.capture(warmup=0)
    torch.cuda.synchronize()
    for rep in range(4):
        a.step()
        g.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work between replays
        close(b.loss.cpu().numpy(), a.loss.cpu().numpy(), rtol=1e-5, floor=1e-3, name=f"loss replay {rep}")
        close_after_adam(b.density["p"].cpu().numpy(), a.density["p"].cpu().numpy(), 2 + rep, a.lr_grid,
                         name=f"density replay {rep}")
        close(b.mlp_flat["p"].cpu().numpy(), a.mlp_flat["p"].cpu().numpy(), rtol=1e-5, floor=1e-3,
              name=f"mlp replay {rep}")


@pytest.mark.parametrize("gather_apart,tv,owner", [(False, True, True), (True, True, True), (False, False, True),
                                                   (True, False, True), (False, True, False)])
def test_two_stream_step_matches_sequential(pkg, gather_apart, tv, owner):
    # the step that overlaps the density update and the MLP Adam on a second stream (with the
    # feature gather fused into the colour head's forward or run apart, which moves the counter,
    # the preparation and the binning to the side stream; with a TV term, or without one, where
    # each grid's Adam is fused into its owner-brick scatter; or with the atomic scatters) takes the
    # same update as the strictly sequential step, eagerly and from a graph
    ops, _, step = pkg
    wl = synth.config2(R=256, n=48)
    say("two-stream step vs sequential, 48^3, 256 rays, gather apart", gather_apart, "TV", tv, "owner", owner)
    tvt = (1e-3, 1e-4, 1.0, True) if tv else None
    mk = lambda conc, fg=True: step.TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max),
                                              feat=wl.feat.data, mlp=(wl.mlp.W, wl.mlp.b),
                                              dist_weight=wl.dist_weight, tv=tvt, owner_scatter=owner,
                                              concurrent=conc, fused_gather=fg)
    smp = wl.samples
    seq, conc, gr = mk(False), mk(True, not gather_apart), mk(True, not gather_apart)
    assert conc.fused_gather == gr.fused_gather == (not gather_apart)
    for st in (seq, conc, gr):
        st.bind(ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len),
                wl.rays.dirs, wl.target)
    g = gr.capture(warmup=1)
    seq.step()
    conc.step()
    for rep in range(3):
        seq.step()
        conc.step()
        g.replay()
        torch.cuda.synchronize()
        for name in ("density", "feat", "mlp_flat"):
            ref = getattr(seq, name)["p"].cpu().numpy()
            for other, tag in ((conc, "eager"), (gr, "graph")):
                got = getattr(other, name)["p"].cpu().numpy()
                # grid gradients are sums whose order differs between runs (atomics, on-chip sums),
                # and the colour head's gradients follow from the grids of the steps before
                lr = seq.lr_mlp if name == "mlp_flat" else seq.lr_grid
                close_after_adam(got, ref, 2 + rep, lr, name=f"{name} two-stream {tag} step {rep}")
                assert not getattr(other, name)["g"].any(), f"{name} gradient not cleared ({tag})"


def test_chained_steps_rotate_batches(pkg):
    # one model trained on two batches in turn: chained steps sharing the parameters (each step
    # prepares the colour head for the next batch), replayed from graphs in turn, take the same
    # updates as a sequential step that is re-bound to each batch before it runs
    ops, _, step = pkg
    wa, wb = synth.config2(R=200, n=48), synth.config2(R=240, n=48, batch=1)
    say("chained steps over two batches, 48^3, 200 and 240 rays")
    mk = lambda conc: step.TrainStep(wa.density.data, (wa.density.xyz_min, wa.density.xyz_max), feat=wa.feat.data,
                                     mlp=(wa.mlp.W, wa.mlp.b), dist_weight=wa.dist_weight, concurrent=conc)
    bat = lambda w: ops.SampleBatch.from_arrays(w.samples.ray_offsets, w.samples.xyz, w.samples.delta,
                                                w.samples.s_mid, w.samples.s_len)
    sa, sb = mk(True), mk(True)
    sb.share_parameters(sa)
    sa.bind(bat(wa), wa.rays.dirs, wa.target)
    sb.bind(bat(wb), wb.rays.dirs, wb.target)
    sa.chain(sb)
    sb.chain(sa)
    ref = mk(False)
    order = [(wa, sa), (wb, sb)]
    for w, s_ in order:  # eager warm-up, same order on the reference
        s_.step()
        ref.bind(bat(w), w.rays.dirs, w.target)
        ref.step()
    graphs = [sa.capture(warmup=0), sb.capture(warmup=0)]
    for rep in range(4):
        w, _ = order[rep % 2]
        graphs[rep % 2].replay()
        ref.bind(bat(w), w.rays.dirs, w.target)
        ref.step()
        torch.cuda.synchronize()
        close(sa.mlp_flat["p"].cpu().numpy(), ref.mlp_flat["p"].cpu().numpy(), rtol=1e-5, floor=1e-3,
              name=f"mlp after replay {rep}")
        for name in ("density", "feat"):
            close_after_adam(sa.__dict__[name]["p"].cpu().numpy(), ref.__dict__[name]["p"].cpu().numpy(), 3 + rep,
                             sa.lr_grid, name=f"{name} after replay {rep}")
    assert int(sa.t_dev.item()) == int(ref.t_dev.item()) == 6


def test_prepared_ahead_follows_weight_edits(pkg):
    # A concurrent step leaves the colour head's preparation for the next step in its workspace;
    # an in-place torch edit of the MLP weights between steps (through a per-layer view) makes the
    # next step prepare again, so it matches the sequential step, which always prepares.
    ops, _, step = pkg
    wl = synth.config2(R=256, n=48)
    say("prepared-ahead colour head after an in-place weight edit, 48^3, 256 rays")
    smp = wl.samples
    mk = lambda conc: step.TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                                     mlp=(wl.mlp.W, wl.mlp.b), dist_weight=wl.dist_weight, concurrent=conc)
    seq, conc = mk(False), mk(True)
    for st in (seq, conc):
        st.bind(ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len),
                wl.rays.dirs, wl.target)
        st.step()
        st.step()
    assert conc.prepared_ahead and not seq.prepared_ahead
    for st in (seq, conc):
        with torch.no_grad():
            st.mlp.W[2].mul_(0.5)  # output layer, in place through its view of the flat parameters
            st.mlp.b[0].add_(0.25)
    for rep in range(2):
        seq.step()
        conc.step()
        torch.cuda.synchronize()
        close(conc.loss.cpu().numpy(), seq.loss.cpu().numpy(), rtol=1e-5, floor=1e-3, name=f"loss after edit {rep}")
        close(conc.mlp_flat["p"].cpu().numpy(), seq.mlp_flat["p"].cpu().numpy(), rtol=1e-5, floor=1e-3,
              name=f"mlp after edit {rep}")
        close_after_adam(conc.density["p"].cpu().numpy(), seq.density["p"].cpu().numpy(), 3 + rep, seq.lr_grid,
                         name=f"density after edit {rep}")


def test_upscale_then_step(pkg):
    # progressive scaling mid-training: 48^3 -> 72^3, moments restarted, the step runs on
    # eagerly and captured again
    ops, _, step = pkg
    wl = synth.config2(R=256, n=48)
    say("upscale 48^3 -> 72^3 then step")
    st = make_step(step, wl)
    st.step()
    st.upscale((72, 72, 72))
    assert st.density["p"].shape[:3] == (72, 72, 72) and not st.feat["m"].any()
    l1 = float(st.step().item())
    g = st.capture(warmup=0)
    g.replay()
    torch.cuda.synchronize()
    assert np.isfinite(l1) and np.isfinite(float(st.loss.item()))
    assert not st.density["g"].any() and not st.feat["g"].any()


def test_autograd_render_and_distortion(pkg):
    ops, ag, _ = pkg
    wl = synth.config1(R=200)
    smp = wl.samples
    rng = np.random.default_rng(50)
    say("autograd RenderFn / DistortionFn, config-1 shape")
    b = ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len)
    dens = T(wl.density.data).requires_grad_(True)
    col = T(wl.color.data).requires_grad_(True)
    shift = float(np.float32(oracle.act_shift()))
    box = (tuple(wl.density.xyz_min), tuple(wl.density.xyz_max))
    rgb, Tf, D = ag.render(dens, col, b, box, grid_color=True, act_shift=shift, bg=(0.3, 0.6, 0.9))
    GC, GD, GT = rng.standard_normal((200, 3)), rng.standard_normal(200), rng.standard_normal(200)
    ((rgb * T(GC)).sum() + (D * T(GD)).sum() + (Tf * T(GT)).sum()).backward()
    og = oracle.render_backward(smp, wl.density, GC, GD, GT, color=wl.color, shift=shift, bg=(0.3, 0.6, 0.9))
    close(dens.grad.cpu().numpy(), og["grad_density"], **GRAD, name="autograd density")
    close(col.grad.cpu().numpy(), og["grad_color"], **GRAD, name="autograd colour")
    # DistortionFn on the oracle's weights
    o = oracle.render_forward(smp, wl.density, wl.color, shift=shift, want_w=True)
    w = T(o["w"]).requires_grad_(True)
    Dd = ag.distortion(w, T(smp.ray_offsets, torch.int32), T(smp.s_mid), T(smp.s_len))
    (Dd * T(GD)).sum().backward()
    close(Dd.detach().cpu().numpy(), o["D"], **FWD, name="autograd distortion")
    close(w.grad.cpu().numpy(), oracle.distortion_grad(smp.ray_offsets, o["w"], smp.s_mid, smp.s_len, GD), **GRAD,
          name="autograd distortion grad")


def test_autograd_gather_and_mlp(pkg):
    ops, ag, _ = pkg
    wl = synth.config2(R=128, n=32, mlp_bias_std=0.2)
    smp = wl.samples
    rng = np.random.default_rng(51)
    say("autograd GatherFn + ColorMLPFn, S =", smp.n_samples)
    grid = T(wl.feat.data).requires_grad_(True)
    xyz = T(smp.xyz)
    box = (tuple(wl.feat.xyz_min), tuple(wl.feat.xyz_max))
    feat = ag.gather(grid, xyz, box)
    Ws = [T(w).requires_grad_(True) for w in wl.mlp.W]
    bs = [T(v).requires_grad_(True) for v in wl.mlp.b]
    rgb = ag.color_mlp(feat, Ws, bs, T(smp.ray_offsets, torch.int32), T(wl.rays.dirs))
    G = rng.standard_normal((smp.n_samples, 3))
    (rgb * T(G)).sum().backward()
    of = oracle.gather(wl.feat, smp.xyz)
    close(rgb.detach().cpu().numpy(), oracle.mlp_forward(wl.mlp, smp.ray_offsets, wl.rays.dirs, of), **FWD,
          name="mlp rgb")
    gf, gW, gb = oracle.mlp_backward(wl.mlp, smp.ray_offsets, wl.rays.dirs, of, G)
    close(grid.grad.cpu().numpy(), oracle.scatter(wl.feat, smp.xyz, gf), **GRAD, name="grad feature grid")
    for i in range(3):
        close(Ws[i].grad.cpu().numpy(), gW[i], **GRAD, name=f"grad W{i + 1}")
        close(bs[i].grad.cpu().numpy(), gb[i], **GRAD, name=f"grad b{i + 1}")


def _rays_touching(smp, n, vertex):
    """Rays with a sample inside one of the 8 cells around grid vertex (i, j, k)."""
    u = (smp.xyz.astype(np.float64) + 1.0) / 2.0 * (n - 1)
    i0 = np.minimum(np.floor(np.clip(u, 0, n - 1)).astype(np.int64), n - 2)
    hit = np.all((i0 <= vertex[None]) & (i0 >= vertex[None] - 1), axis=1)
    ray = np.repeat(np.arange(smp.n_rays), smp.lengths())
    return np.unique(ray[hit])


def _subset(wl, rays):
    smp = wl.samples
    offs, idx = [0], []
    for r in rays:
        a, b = smp.ray_offsets[r], smp.ray_offsets[r + 1]
        idx.append(np.arange(a, b))
        offs.append(offs[-1] + b - a)
    idx = np.concatenate(idx)
    return synth.Samples(np.asarray(offs, np.int32), smp.xyz[idx], smp.delta[idx], smp.s_mid[idx], smp.s_len[idx])


def _partial_loss(wl, sub, rays, shift, R_total):
    """Sum of the per-ray terms of the full loss for the given rays (FP64 oracle)."""
    feat = oracle.gather(wl.feat, sub.xyz)
    srgb = oracle.mlp_forward(wl.mlp, sub.ray_offsets, wl.rays.dirs[rays], feat)
    o = oracle.render_forward(sub, wl.density, srgb=srgb, shift=shift)
    e = o["rgb"] - wl.target[rays].astype(np.float64)
    return np.sum(e * e) / (3.0 * R_total) + wl.dist_weight * np.sum(o["D"]) / R_total


@pytest.mark.timeout(900)
def test_config4_finite_differences(pkg):
    """16384 rays x 512 samples on the 160^3 grids: the autograd backward (recompute, no
    stored per-sample intermediates) against FP64 central differences of the oracle loss on
    128 density + 128 feature-grid entries (eps 1e-4), and against the oracle's analytic
    gradient restricted to the rays that touch each entry."""
    ops, ag, _ = pkg
    wl = synth.config4()
    smp = wl.samples
    R, S = smp.n_rays, smp.n_samples
    say("config4 FD: R =", R, "S =", S)
    n = wl.density.data.shape[0]
    b = ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len)
    dens = T(wl.density.data).requires_grad_(True)
    fgrid = T(wl.feat.data).requires_grad_(True)
    Ws = [T(w) for w in wl.mlp.W]
    bs = [T(v) for v in wl.mlp.b]
    box = (tuple(wl.density.xyz_min), tuple(wl.density.xyz_max))
    shift = float(np.float32(ops.act_shift()))
    feat = ag.gather(fgrid, b.xyz, box)
    srgb = ag.color_mlp(feat, Ws, bs, b.ray_offsets, T(wl.rays.dirs))
    rgb, Tf, D = ag.render(dens, srgb, b, box, grid_color=False, act_shift=shift)
    tgt = T(wl.target)
    loss = ((rgb - tgt) ** 2).mean() + wl.dist_weight * D.mean()
    loss.backward()
    gd = dens.grad.cpu().numpy()
    gfg = fgrid.grad.cpu().numpy()
    # 128 entries of each grid at vertices of cells that samples fall in (chosen from the
    # inputs alone: a random sample, one of its 8 cell corners, a random channel)
    rng = np.random.default_rng(60)
    u = (smp.xyz.astype(np.float64) + 1.0) / 2.0 * (n - 1)
    cell = np.minimum(np.floor(np.clip(u, 0, n - 1)).astype(np.int64), n - 2)

    def pick(C, count):
        out = set()
        while len(out) < count:
            k = int(rng.integers(S))
            v = cell[k] + rng.integers(0, 2, 3)
            out.add(int(((v[0] * n + v[1]) * n + v[2]) * C + rng.integers(C)))
        return np.array(sorted(out))

    di = pick(1, 128)
    fi = pick(wl.feat.data.shape[-1], 128)
    fd, an, gp, curv = [], [], [], []
    eps = np.float32(1e-4)
    for grid, flat, gpu in ((wl.density, di, gd), (wl.feat, fi, gfg)):
        C = grid.data.shape[-1]
        for cnt, idx in enumerate(flat):
            if cnt % 32 == 0:
                say("FD entries done:", len(fd))
            v = np.array(np.unravel_index(idx // C, grid.data.shape[:3]))
            rays = _rays_touching(smp, n, v)
            sub = _subset(wl, rays)
            data = grid.data.reshape(-1)
            old = data[idx]
            data[idx] = old + eps
            hi_v = float(data[idx])
            lp = _partial_loss(wl, sub, rays, shift, R)
            data[idx] = old - eps
            lo_v = float(data[idx])
            lm = _partial_loss(wl, sub, rays, shift, R)
            data[idx] = old
            l0 = _partial_loss(wl, sub, rays, shift, R)
            fd.append((lp - lm) / (hi_v - lo_v))
            # one-sided slopes: they differ by O(eps) unless a ReLU kink lies inside the step
            curv.append(abs((lp - l0) / (hi_v - float(old)) - (l0 - lm) / (float(old) - lo_v)))
            gp.append(gpu.ravel()[idx])
            # analytic oracle gradient from the touching rays only
            feat_o = oracle.gather(wl.feat, sub.xyz)
            srgb_o = oracle.mlp_forward(wl.mlp, sub.ray_offsets, wl.rays.dirs[rays], feat_o)
            o = oracle.render_forward(sub, wl.density, srgb=srgb_o, shift=shift)
            GC = 2.0 * (o["rgb"] - wl.target[rays]) / (3.0 * R)
            GDv = np.full(len(rays), wl.dist_weight / R)
            og = oracle.render_backward(sub, wl.density, GC, GDv, None, srgb=srgb_o, shift=shift)
            if grid is wl.density:
                an.append(og["grad_density"].ravel()[idx])
            else:
                gfo, _, _ = oracle.mlp_backward(wl.mlp, sub.ray_offsets, wl.rays.dirs[rays], feat_o, og["grad_srgb"])
                an.append(oracle.scatter(wl.feat, sub.xyz, gfo).ravel()[idx])
    fd, an, gp, curv = np.array(fd), np.array(an), np.array(gp), np.array(curv)
    # An entry whose +-eps step crosses a ReLU kink of the colour head has no central
    # difference to compare with (the loss is not differentiable there); leave it out of the
    # finite-difference checks and keep the analytic comparison for every entry.
    smooth = curv <= 1e-3 * (np.abs(fd) + 1e-2 * np.abs(fd).max())
    say("FD entries across a kink:", int((~smooth).sum()), "of", len(fd))
    assert smooth.sum() >= 0.9 * len(fd)
    # the oracle's analytic gradient agrees with its own finite differences
    close(an[smooth], fd[smooth], rtol=1e-4, floor=1e-2, name="oracle analytic vs FD")
    close(gp[:128], an[:128], **GRAD, name="GPU vs oracle, density")
    close(gp[128:], an[128:], **GRAD, name="GPU vs oracle, features")
    close(gp[smooth], fd[smooth], rtol=2e-4, floor=1e-2, name="GPU vs FD")


def test_tuned_schedule_step_and_rebind(pkg):
    # the step with the autotuned longest-first render schedule takes the same update as the
    # default schedule; binding another batch drops the schedule (its ray list belongs to the
    # batch it was tuned on), and the step then runs on the new batch
    ops, _, step = pkg
    wl = synth.config2(R=256, n=48)
    say("tuned render schedule vs default, 48^3, 256 rays; rebind to 100 rays")
    mk = lambda: step.TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                                mlp=(wl.mlp.W, wl.mlp.b), dist_weight=wl.dist_weight)
    smp = wl.samples
    a, b = mk(), mk()
    for st in (a, b):
        st.bind(ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len),
                wl.rays.dirs, wl.target)
    sched, _ = b.tune()
    assert sched.ray_list is not None and sched.ray_list.numel() == 256
    for rep in range(2):
        a.step()
        b.step()
        torch.cuda.synchronize()
        close(b.loss.cpu().numpy(), a.loss.cpu().numpy(), rtol=1e-5, floor=1e-3, name=f"loss {rep}")
        close(b.mlp_flat["p"].cpu().numpy(), a.mlp_flat["p"].cpu().numpy(), rtol=1e-5, floor=1e-3,
              name=f"mlp tuned {rep}")
        close_after_adam(b.density["p"].cpu().numpy(), a.density["p"].cpu().numpy(), 1 + rep, a.lr_grid,
                         name=f"density tuned {rep}")
    small = synth.config2(R=100, n=48)
    s2 = small.samples
    b.bind(ops.SampleBatch.from_arrays(s2.ray_offsets, s2.xyz, s2.delta, s2.s_mid, s2.s_len), small.rays.dirs,
           small.target)
    assert b.schedule is None
    b.step()
    torch.cuda.synchronize()
    assert np.isfinite(b.loss.cpu().numpy()).all()


def _moment_gradient(m0, m1, v0, v1, p0, p1, b1, skip):
    """The gradient one Adam update consumed, read back from its first moment:
    m1 = b1 m0 + (1 - b1) g in float32, so g = (m1 - b1 m0) / (1 - b1) up to the rounding of
    m1 (returned as a per-element slack).  With skip, an element whose parameter and moments
    are bit-for-bit unchanged took a zero gradient."""
    b1 = np.float64(np.float32(b1))
    c = np.float64(np.float32(1.0) - np.float32(b1))
    m0d, m1d = m0.astype(np.float64).ravel(), m1.astype(np.float64).ravel()
    g = (m1d - b1 * m0d) / c
    slack = 4.0 * 2.0 ** -24 * (np.abs(m1d) + b1 * np.abs(m0d)) / c
    if skip:
        same = (m1.ravel() == m0.ravel()) & (v1.ravel() == v0.ravel()) & (p1.ravel() == p0.ravel())
        g[same] = 0.0
        slack[same] = 0.0
    return g, slack


def _full_size_captured_step(pkg, wl, label, **kw):
    """The launch configuration the benchmark times on this workload: the render kernels on the
    autotuned longest-first schedule, the two-stream step captured in a HIP graph after one
    warm-up step.  One replay is checked against the FP64 oracle run from the parameters it
    started from: colour, distortion and loss of every ray; the gradient of every grid entry and
    MLP parameter, read back from the first Adam moment the replay wrote; and the replay's Adam
    update of every parameter, given that gradient."""
    ops, _, step = pkg
    smp = wl.samples
    say(label, "full size, bench launch configuration: R =", smp.n_rays, "S =", smp.n_samples)
    st = step.TrainStep(wl.density.data, (wl.density.xyz_min, wl.density.xyz_max), feat=wl.feat.data,
                        mlp=(wl.mlp.W, wl.mlp.b), dist_weight=wl.dist_weight, **kw)
    st.bind(ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len), wl.rays.dirs,
            wl.target)
    assert st.concurrent and st.binned and st.fused_gather
    sched, _ = st.tune()
    assert sched.ray_list is not None
    say("tuned schedule: waves per block", sched.waves_per_block, "grid waves", sched.grid_waves)
    g = st.capture(warmup=1)
    torch.cuda.synchronize()
    groups = (("density", st.lr_grid, True), ("feat", st.lr_grid, True), ("mlp_flat", st.lr_mlp, False))
    before = {k: {q: getattr(st, k)[q].cpu().numpy().copy() for q in ("p", "m", "v", "g")} for k, _, _ in groups}
    for k, _, _ in groups:
        assert not before[k]["g"].any(), f"{k}: gradients not cleared by the warm-up step's Adam"
    g.replay()
    torch.cuda.synchronize()
    t = int(st.t_dev.item())
    assert t == 2
    after = {k: {q: getattr(st, k)[q].cpu().numpy() for q in ("p", "m", "v")} for k, _, _ in groups}
    say("replay done; oracle forward + backward from the replay's starting parameters")

    # the oracle's inputs: the parameters the replay started from
    import dataclasses
    p0 = {k: before[k]["p"] for k, _, _ in groups}
    shapes = [w.shape for w in wl.mlp.W] + [b.shape for b in wl.mlp.b]
    parts = np.split(p0["mlp_flat"], np.cumsum([int(np.prod(s)) for s in shapes])[:-1])
    mlp0 = synth.MLPWeights([parts[i].reshape(shapes[i]) for i in range(3)],
                            [parts[3 + i].reshape(shapes[3 + i]) for i in range(3)])
    wl0 = dataclasses.replace(wl, density=dataclasses.replace(wl.density, data=p0["density"].reshape(wl.density.data.shape)),
                              feat=dataclasses.replace(wl.feat, data=p0["feat"].reshape(wl.feat.data.shape)), mlp=mlp0)
    shift = float(np.float32(st.shift))
    L, o, gd, gfeat, gW, gb = oracle_step_grads(wl0, shift)
    close(st.rgb.cpu().numpy(), o["rgb"], **FWD, name="rgb")
    close(st.dist.cpu().numpy(), o["D"], **FWD, name="distortion")
    close(st.loss.cpu().numpy(), [L], **FWD, name="loss")

    # ReLU units within float32 rounding of their kink: both sides are valid there
    feat = oracle.gather(wl0.feat, smp.xyz)
    srgb = oracle.mlp_forward(mlp0, smp.ray_offsets, wl.rays.dirs, feat)
    _, GC, GD = oracle.loss_head(o["rgb"], wl.target, o["D"], wl.dist_weight)
    g_srgb = oracle.render_backward(smp, wl0.density, GC, GD, None, srgb=srgb, shift=shift)["grad_srgb"]
    sf, sW, sb = oracle.mlp_kink_slack(mlp0, smp.ray_offsets, wl.rays.dirs, feat, g_srgb)
    kink = {"density": np.zeros(gd.size), "feat": np.abs(oracle.scatter(wl0.feat, smp.xyz, sf)).ravel(),
            "mlp_flat": np.concatenate([np.abs(s).ravel() for s in list(sW) + list(sb)])}
    want = {"density": gd.ravel(), "feat": gfeat.ravel(),
            "mlp_flat": np.concatenate([np.asarray(x).ravel() for x in list(gW) + list(gb)])}
    b1, b2 = st.betas
    for k, lr, skip in groups:
        a, z = after[k], before[k]
        gk, rs = _moment_gradient(z["m"], a["m"], z["v"], a["v"], z["p"], a["p"], b1, skip)
        # how much the kink slack widens the normwise bound, against the bound itself
        say(k, "gradient from the first moment vs oracle;", int((gk != 0).sum()), "non-zero of", gk.size,
            "; ||kink slack|| / (rtol ||y||) = %.3g" % (np.linalg.norm(kink[k]) /
                                                         max(GRAD["rtol"] * np.linalg.norm(want[k]), 1e-300)))
        close(gk, want[k], **GRAD, name=f"grad {k}", slack=rs + kink[k])
        # the update itself, from the gradient the replay consumed
        pe, _, _ = oracle.adam(z["p"], gk, z["m"], z["v"], lr, float(np.float32(b1)), float(np.float32(b2)),
                               st.eps, t, skip_zero=skip)
        close_after_adam(a["p"], pe, 1, lr, name=f"{k} after Adam")


@pytest.mark.timeout(600)
def test_config2_full_size_captured_step(pkg):
    """Config 2 (the benchmark's workload): 160^3 density and 160^3x12 feature grids, 8192
    pinhole rays (S ~ 0.96 M live samples)."""
    _full_size_captured_step(pkg, synth.config2(), "config 2")


@pytest.mark.timeout(1200)
def test_config3_full_size_captured_step(pkg):
    """Config 3 (unbounded, section 5.4): 320^3 density and 320^3x12 feature grids addressed
    through Eq. 4 (p = inf, b = 1) inside the kernels, 8192 rays with lognormal live lengths
    32..1024 (S ~ 2.5 M), 16-chunk rays on the tuned persistent schedule."""
    wl = synth.config3()
    assert wl.density.warp == 1 and wl.feat.warp == 1 and wl.samples.lengths().max() > 960
    _full_size_captured_step(pkg, wl, "config 3", warp=(wl.density.warp, wl.density.warp_b))
