"""The fused render call (forward, loss gradient and backward of each ray in one launch) against
the three calls it replaces (render forward, the loss head's gradients, render backward), and
against the FP64 oracle.

Where every output element has one writer (colour, transmittance, distortion, render state,
per-sample colour and density-logit gradients) the fused call must agree bit for bit: it runs the
same walks with the same expressions.  Gradients summed by atomics (the in-kernel density scatter,
the colour grid) differ only in the order of their terms.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import FWD, GRAD, close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_05085_amd as pkg
    pkg.lib()
    from paper_2206_05085_amd import ops
    return ops


def say(*a):
    print("[case]", *a, flush=True)


def T(a, dt=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)


def dgrid(ops, g, grad=False):
    data = T(g.data)
    return ops.DeviceGrid(data, g.xyz_min, g.xyz_max, grad=torch.zeros_like(data) if grad else None,
                          warp=g.warp, warp_b=g.warp_b)


def dbatch(ops, s):
    return ops.SampleBatch.from_arrays(s.ray_offsets, s.xyz, s.delta, s.s_mid, s.s_len)


def _workload(name):
    if name == "config1_grid":
        return synth.config1(R=256)
    if name == "config3_contract":
        return synth.config3(R=192, n=96)
    if name == "edge":
        wl = synth.config1(R=8)
        lengths = [0, 1, 2, 63, 64, 65, 128, 129, 0, 1, 0]
        offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)
        rng = np.random.default_rng(91)
        S = int(offs[-1])
        t = np.concatenate([np.sort(rng.uniform(0, 1, n)) for n in lengths]) if S else np.zeros(0)
        xyz = rng.uniform(-1, 1, (S, 3)).astype(np.float32)
        xyz[:4] = [[1, 1, 1], [-1, -1, -1], [1, -1, 0], [0, 0, 1]]
        wl.samples = synth.Samples(offs, xyz, np.full(S, 0.5, np.float32), t.astype(np.float32),
                                   np.full(S, 1.0 / 128, np.float32))
        return wl
    return synth.config2(R=512)


def _run(dv, wl, mode, fused, *, halt_T=0.0, want_dist=True, per_sample=True, sched=None, lam=0.01, seed=0):
    smp = wl.samples
    R, S = smp.n_rays, smp.n_samples
    rng = np.random.default_rng(seed)
    shift = float(np.float32(oracle.act_shift()))
    srgb = T(rng.random((S, 3))) if mode == "samples" else None
    target = T(rng.random((R, 3)))
    dens = dgrid(dv, wl.density, grad=True)
    col = dgrid(dv, wl.color, grad=True) if mode == "grid" else None
    b = dbatch(dv, smp)
    rgb, Tf, D = (torch.full((R, 3), -1.0, device="cuda"), torch.full((R,), -1.0, device="cuda"),
                  torch.full((R,), -1.0, device="cuda"))
    state = torch.zeros(dv.render_state_size(R, S), dtype=torch.uint8, device="cuda")
    gs = torch.full((S, 3), 5.0, device="cuda") if mode == "samples" else None
    graw = torch.full((S,), 7.0, device="cuda") if per_sample else None
    if fused:
        dv.render_train(b, dens, col, srgb, target, lam, act_shift_=shift, halt_T=halt_T, want_dist=want_dist,
                        out=(rgb, Tf, D), state=state, grad_sample_rgb=gs, schedule=sched, grad_sample_density=graw)
    else:
        dv.render_forward(b, dens, col, srgb, act_shift_=shift, halt_T=halt_T, want_dist=want_dist, out=(rgb, Tf, D),
                          state=state, schedule=sched)
        _, gC, gD = dv.loss_head(rgb, target, D if want_dist else None, lam, want_loss=False)
        dv.render_backward(b, dens, col, srgb, Tf, state, gC, gD, None, act_shift_=shift, halt_T=halt_T,
                           want_dist=want_dist, grad_sample_rgb=gs, schedule=sched, grad_sample_density=graw)
    torch.cuda.synchronize()
    out = {"rgb": rgb, "T": Tf, "state": state, "grad_density": dens.grad}
    if want_dist:
        out["dist"] = D
    if gs is not None:
        out["grad_srgb"] = gs
    if graw is not None:
        out["grad_raw"] = graw
    if col is not None:
        out["grad_color"] = col.grad
    return {k: v.cpu().numpy() for k, v in out.items()}, (srgb, target, shift)


CASES = [
    # name, workload, mode, options
    ("config2 per-sample", "config2", "samples", {}),
    ("config2 tuned schedule", "config2", "samples", {"sched": "tuned"}),
    ("config2 halting paper mode", "config2", "samples", {"halt_T": 1e-3}),
    ("config2 no distortion term", "config2", "samples", {"want_dist": False}),
    ("config2 in-kernel density scatter", "config2", "samples", {"per_sample": False}),
    ("config3 Eq. 4 contraction, lognormal lengths", "config3_contract", "samples", {"sched": "tuned"}),
    ("config1 colour grid", "config1_grid", "grid", {"per_sample": False}),
    ("edge lengths (empty, 1, 63-65, 128-129)", "edge", "grid", {"per_sample": True}),
]


@pytest.mark.parametrize("name,wname,mode,opt", CASES, ids=[c[0] for c in CASES])
def test_render_train_matches_three_calls(dv, name, wname, mode, opt):
    wl = _workload(wname)
    smp = wl.samples
    opt = dict(opt)
    if opt.get("sched") == "tuned":
        order, _ = dv.ray_schedule(T(smp.ray_offsets, torch.int32))
        opt["sched"] = dv.Schedule(order, 4, 1024)
    say("render_train vs forward + loss head + backward:", name, "R =", smp.n_rays, "S =", smp.n_samples)
    fu, _ = _run(dv, wl, mode, True, seed=7, **opt)
    three, _ = _run(dv, wl, mode, False, seed=7, **opt)
    atomic = {"grad_color"} | ({"grad_density"} if not opt.get("per_sample", True) else set())
    assert set(fu) == set(three)
    for k in fu:
        if k in atomic:
            close(fu[k], three[k], **GRAD, name=k)
        else:
            np.testing.assert_array_equal(fu[k], three[k], err_msg=k)
    if "grad_raw" in fu:
        assert not (fu["grad_raw"] == 7.0).any()
    if "grad_srgb" in fu:
        assert not (fu["grad_srgb"] == 5.0).any()


def test_render_train_against_oracle(dv):
    # the fused call's outputs and gradients against the oracle's forward, its loss head (MSE +
    # lam * distortion) and its backward fed that loss head's gradients
    wl = synth.config2(R=384)
    smp = wl.samples
    lam = 0.01
    say("render_train vs oracle (loss head + render backward), 384 rays, S =", smp.n_samples)
    fu, (srgb, target, shift) = _run(dv, wl, "samples", True, per_sample=False, lam=lam, seed=11)
    srgb_np, tgt_np = srgb.cpu().numpy(), target.cpu().numpy()
    of = oracle.render_forward(smp, wl.density, srgb=srgb_np, shift=shift)
    close(fu["rgb"], of["rgb"], **FWD, name="rgb")
    close(fu["dist"], of["D"], **FWD, name="dist")
    _, GC, GD = oracle.loss_head(of["rgb"], tgt_np, of["D"], lam)
    ob = oracle.render_backward(smp, wl.density, GC, GD, None, srgb=srgb_np, shift=shift)
    close(fu["grad_density"], ob["grad_density"], **GRAD, name="grad density")
    close(fu["grad_srgb"], ob["grad_srgb"], **GRAD, name="grad sample rgb")


def test_render_train_rejects_bad_arguments(dv):
    wl = synth.config2(R=16)
    smp = wl.samples
    b = dbatch(dv, smp)
    dens = dgrid(dv, wl.density, grad=True)
    srgb = torch.zeros(smp.n_samples, 3, device="cuda")
    say("render_train argument checks")
    with pytest.raises(Exception):
        dv.render_train(b, dens, None, srgb, torch.zeros(smp.n_rays, 3, device="cuda"), -1.0, act_shift_=0.0)
    with pytest.raises(Exception):
        dv.render_train(b, dens, None, srgb, torch.zeros(smp.n_rays + 1, 3, device="cuda"), 0.01, act_shift_=0.0)
