"""Ragged scheduling of the render kernels: the schedule builder, persistent longest-first
launches, per-length-class launches and the autotuner all give the results of the plain
one-wave-per-ray launch."""
import numpy as np
import pytest
import torch

import synth
from parity import GRAD, close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_05085_amd as p
    p.lib()
    from paper_2206_05085_amd import ops
    return ops


def say(*a):
    print("[case]", *a, flush=True)


def T(a, dt=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)


def test_schedule_builder(ops):
    rng = np.random.default_rng(80)
    lengths = np.concatenate([rng.integers(0, 1100, 3000), [0, 64, 65, 4032, 4033, 10000]])
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)
    say("schedule builder, R =", len(lengths))
    order, cls = ops.ray_schedule(T(offs, torch.int32))
    order, cls = order.cpu().numpy(), cls.cpu().numpy()
    assert sorted(order.tolist()) == list(range(len(lengths)))          # a permutation
    chunks = np.minimum((lengths + 63) // 64, 63)
    c = chunks[order]
    assert (np.diff(c) <= 0).all()                                       # longest first
    for k in range(64):
        assert (chunks[order[cls[k]:cls[k + 1]]] == 63 - k).all()
    assert cls[0] == 0 and cls[64] == len(lengths)


def _run(ops, wl, sched, srgb, GC, GD):
    smp = wl.samples
    b = ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid, smp.s_len)
    d = ops.DeviceGrid(T(wl.density.data), wl.density.xyz_min, wl.density.xyz_max, warp=wl.density.warp,
                   warp_b=wl.density.warp_b)
    d.grad = torch.zeros_like(d.data)
    shift = ops.act_shift()
    outs = []
    for sc in (sched if isinstance(sched, list) else [sched]):
        outs.append(sc)
    rgb = torch.full((smp.n_rays, 3), -1.0, device="cuda")
    Tt = torch.full((smp.n_rays,), -1.0, device="cuda")
    D = torch.full((smp.n_rays,), -1.0, device="cuda")
    state = torch.empty(ops.render_state_size(smp.n_rays, smp.n_samples), dtype=torch.uint8, device="cuda")
    gs = torch.zeros(smp.n_samples, 3, device="cuda")
    for sc in outs:
        ops.render_forward(b, d, None, srgb, act_shift_=shift, out=(rgb, Tt, D), state=state, schedule=sc)
    for sc in outs:
        ops.render_backward(b, d, None, srgb, Tt, state, GC, GD, None, act_shift_=shift, grad_sample_rgb=gs,
                            schedule=sc)
    torch.cuda.synchronize()
    return rgb.cpu().numpy(), Tt.cpu().numpy(), D.cpu().numpy(), d.grad.cpu().numpy(), gs.cpu().numpy()


def test_schedules_agree(ops):
    wl = synth.config3(R=2048, n=96)
    smp = wl.samples
    rng = np.random.default_rng(81)
    srgb = T(rng.random((smp.n_samples, 3)))
    GC, GD = T(rng.standard_normal((smp.n_rays, 3))), T(rng.standard_normal(smp.n_rays))
    say("schedules agree, config-3 shape, R = 2048, S =", smp.n_samples)
    base = _run(ops, wl, None, srgb, GC, GD)
    order, cls = ops.ray_schedule(T(smp.ray_offsets, torch.int32))
    pers = _run(ops, wl, ops.Schedule(order, 8, 1024), srgb, GC, GD)
    c = cls.cpu().numpy()
    # per-class launches: one launch per length class (power-of-two sample buckets)
    bounds = [(1, 1), (2, 2), (3, 4), (5, 8), (9, 16), (17, 63), (0, 0)]
    lists = []
    for lo, hi in bounds:
        a, z = c[63 - hi], c[63 - lo + 1]
        if z > a:
            lists.append(ops.Schedule(order[a:z].contiguous(), 4, 0))
    buck = _run(ops, wl, lists, srgb, GC, GD)
    tuned, ms = ops.render_autotune(ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid,
                                                                smp.s_len),
                                    ops.DeviceGrid(T(wl.density.data), wl.density.xyz_min, wl.density.xyz_max, warp=wl.density.warp,
                   warp_b=wl.density.warp_b),
                                    None, srgb, act_shift_=ops.act_shift(), ray_list=order)
    say("autotuned:", tuned.waves_per_block, tuned.grid_waves, f"{ms:.3f} ms")
    assert 1 <= tuned.waves_per_block <= 16 and tuned.grid_waves >= 0 and ms > 0
    again, ms2 = ops.render_autotune(ops.SampleBatch.from_arrays(smp.ray_offsets, smp.xyz, smp.delta, smp.s_mid,
                                                                 smp.s_len),
                                     ops.DeviceGrid(T(wl.density.data), wl.density.xyz_min, wl.density.xyz_max, warp=wl.density.warp,
                   warp_b=wl.density.warp_b),
                                     None, srgb, act_shift_=ops.act_shift(), ray_list=order)
    assert (again.waves_per_block, again.grid_waves, ms2) == (tuned.waves_per_block, tuned.grid_waves, ms)  # cached
    tun = _run(ops, wl, tuned, srgb, GC, GD)
    for other, name in ((pers, "persistent"), (buck, "per-class"), (tun, "autotuned")):
        for i in range(3):   # forward outputs are bitwise identical: same per-ray code, no atomics
            assert np.array_equal(other[i], base[i]), name
        assert np.array_equal(other[4], base[4]), name   # per-sample colour gradients: one writer each
        close(other[3], base[3], **GRAD, name=f"density grad, {name}")   # atomics: order differs
