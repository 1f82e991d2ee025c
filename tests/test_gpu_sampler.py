"""GPU parity of the sample producer (dvgo_sample_count / dvgo_sample_emit) and the occupancy
mask update (dvgo_occupancy_update) against the oracle.

Every decision of the producer is a float32 IEEE operation (header definition), so counts,
offsets and the mask are compared bit for bit, and so are the emitted floats (each is one
rounded operation of identical operands).  Cases: special rays (axis-aligned, misses, zero
direction components, origins inside the box, a near plane), random rays with and without a
mask, a cap, a capacity smaller than the batch (nothing written past it), no rays, and the
full-size fine-stage case: 8192 pinhole rays through the 160^3 blob scene at a half-voxel step
with the mask the update builds from its density.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

BOX = (np.full(3, -1.0, np.float32), np.full(3, 1.0, np.float32))


@pytest.fixture(scope="module")
def dv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_05085_amd as pkg
    pkg.lib()  # raises if the HIP library is missing
    from paper_2206_05085_amd import ops
    return ops


def say(*a):
    print("[case]", *a, flush=True)


def T(a, dt=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)


def _gpu(dv, o, d, step, voxel, near=0.0, cap=4096, mask=None, box=BOX):
    spec = dv.SamplerSpec(box[0], box[1], step, voxel, near, cap, None if mask is None else T(mask, torch.uint8))
    R = len(o)
    tn = torch.empty(R, device="cuda")
    tf = torch.empty(R, device="cuda")
    og, dg = T(o), T(d)
    offs = dv.sample_count(spec, og, dg, t_near=tn, t_far=tf)
    S = int(offs[-1].item())
    b = dv.sample_emit(spec, og, dg, offs, S)
    torch.cuda.synchronize()
    return dict(ray_offsets=offs.cpu().numpy(), t_near=tn.cpu().numpy(), t_far=tf.cpu().numpy(),
                xyz=b.xyz.cpu().numpy(), delta=b.delta.cpu().numpy(), s_mid=b.s_mid.cpu().numpy(),
                s_len=b.s_len.cpu().numpy())


def _same(got, want, keys=("ray_offsets", "t_near", "t_far", "xyz", "delta", "s_mid", "s_len")):
    for k in keys:
        g, w = np.asarray(got[k]), np.asarray(want[k])
        assert g.shape == w.shape, (k, g.shape, w.shape)
        assert np.array_equal(g.view(np.uint32) if g.dtype == np.float32 else g,
                              w.view(np.uint32) if w.dtype == np.float32 else w), k


def _special_rays():
    o = [[-3, 0.1, 0.2], [-3, 5, 0], [3, 0, 0], [0, 0, 0], [0.3, -0.2, 0.1], [-3, 0.5, 0.5], [1, 1, 1],
         [-1.5, -1.5, -1.5], [0, 0, -3]]
    d = [[1, 0, 0], [1, 0, 0], [1, 0, 0], [0, 0, 1], [0, -1, 0], [0, 1, 0], [-1, -1, -1], [1, 1, 1],
         [0.6, 0, -0.8]]
    o = np.array(o, np.float32)
    d = np.array(d, np.float64)
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    return o, d


@pytest.mark.parametrize("near", [0.0, 0.125, 2.5])
def test_special_rays(dv, near):
    o, d = _special_rays()
    say("special rays, near", near)
    got = _gpu(dv, o, d, 0.0625, 0.125, near=near)
    want = oracle.sample_rays(o, d, BOX[0], BOX[1], near, 0.0625, 0.125, 4096)
    _same(got, want)


@pytest.mark.parametrize("masked", [False, True])
@pytest.mark.parametrize("kind", ["box", "pinhole"])
def test_random_rays(dv, masked, kind):
    rng = np.random.default_rng(100)
    rays = synth.scenes.rays_at_box(rng, 1500) if kind == "box" else synth.scenes.pinhole_rays(rng, 1500)
    mask = (rng.random((13, 17, 11)) < 0.35).astype(np.uint8) if masked else None
    step = 2.0 / 31 * 0.5
    say("random rays", kind, "masked", masked)
    got = _gpu(dv, rays.origins, rays.dirs, step, 2.0 / 31, mask=mask)
    want = oracle.sample_rays(rays.origins, rays.dirs, BOX[0], BOX[1], 0.0, step, 2.0 / 31, 4096, mask)
    assert want["ray_offsets"][-1] > 1500 * (5 if masked else 20)
    _same(got, want)


def test_cap_and_offset_box(dv):
    rng = np.random.default_rng(101)
    box = (np.float32([-0.5, 0.25, -2.0]), np.float32([1.5, 0.75, 1.0]))
    rays = synth.scenes.rays_at_box(rng, 700, bmin=tuple(box[0]), bmax=tuple(box[1]))
    mask = (rng.random((5, 6, 7)) < 0.6).astype(np.uint8)
    say("cap 37, off-centre box")
    got = _gpu(dv, rays.origins, rays.dirs, 0.01, 0.02, cap=37, mask=mask, box=box)
    want = oracle.sample_rays(rays.origins, rays.dirs, box[0], box[1], 0.0, 0.01, 0.02, 37, mask)
    _same(got, want)
    assert np.diff(want["ray_offsets"]).max() <= 37


def test_capacity_bounds_writes(dv):
    rng = np.random.default_rng(102)
    rays = synth.scenes.rays_at_box(rng, 300)
    spec = dv.SamplerSpec(BOX[0], BOX[1], 0.02, 0.02)
    og, dg = T(rays.origins), T(rays.dirs)
    say("capacity below the total")
    offs = dv.sample_count(spec, og, dg)
    S = int(offs[-1].item())
    cap = S // 3
    pad = 1000
    out = dv.SampleBatch(offs, torch.full((cap + pad, 3), 7.0, device="cuda"), torch.full((cap + pad,), 7.0, device="cuda"),
                         torch.full((cap + pad,), 7.0, device="cuda"), torch.full((cap + pad,), 7.0, device="cuda"),
                         len(rays.origins), cap + pad)
    from paper_2206_05085_amd._lib import call
    call("dvgo_sample_emit", spec.struct(), len(rays.origins), og.data_ptr(), dg.data_ptr(), offs.data_ptr(), cap,
         out.xyz.data_ptr(), out.delta.data_ptr(), out.s_mid.data_ptr(), out.s_len.data_ptr(),
         torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    want = oracle.sample_rays(rays.origins, rays.dirs, BOX[0], BOX[1], 0.0, 0.02, 0.02, 4096)
    assert np.array_equal(out.xyz[:cap].cpu().numpy(), want["xyz"][:cap])
    assert np.array_equal(out.s_mid[:cap].cpu().numpy(), want["s_mid"][:cap])
    assert (out.xyz[cap:] == 7.0).all() and (out.delta[cap:] == 7.0).all()
    assert (out.s_mid[cap:] == 7.0).all() and (out.s_len[cap:] == 7.0).all()


def test_many_rays_multi_pass_offsets(dv):
    # more rays than one pass of the prefix sum (8192 per pass), with a mask
    rng = np.random.default_rng(104)
    rays = synth.scenes.rays_at_box(rng, 20001)
    mask = (rng.random((9, 9, 9)) < 0.5).astype(np.uint8)
    say("20001 rays, three prefix-sum passes")
    got = _gpu(dv, rays.origins, rays.dirs, 0.1, 0.1, mask=mask)
    want = oracle.sample_rays(rays.origins, rays.dirs, BOX[0], BOX[1], 0.0, 0.1, 0.1, 4096, mask)
    _same(got, want)


# ------------------------------------------------------------------ forward-facing (NDC)

FF = dict(W=1008, H=756, focal=815.0)
FX, FY = 2 * FF["focal"] / FF["W"], 2 * FF["focal"] / FF["H"]


def _gpu_ndc(dv, o, d, planes, step, near=1.0, cap=4096, mask=None):
    spec = dv.SamplerSpec(BOX[0], BOX[1], step, near=near, max_per_ray=cap,
                          mask=None if mask is None else T(mask, torch.uint8), ndc=(FX, FY, planes))
    R = len(o)
    og, dg = T(o), T(d)
    tn = torch.empty(R, device="cuda")
    tf = torch.empty(R, device="cuda")
    offs = dv.sample_count(spec, og, dg, t_near=tn, t_far=tf)
    S = int(offs[-1].item())
    b = dv.sample_emit(spec, og, dg, offs, S)
    torch.cuda.synchronize()
    n = np.diff(offs.cpu().numpy())
    assert (tf.cpu().numpy()[n > 0] == 1.0).all() and not tn.cpu().numpy().any()
    return dict(ray_offsets=offs.cpu().numpy(), xyz=b.xyz.cpu().numpy(), delta=b.delta.cpu().numpy(),
                s_mid=b.s_mid.cpu().numpy(), s_len=b.s_len.cpu().numpy())


@pytest.mark.parametrize("planes,step,masked", [(8, 0.5, False), (64, 0.5, True), (33, 0.75, True),
                                                (256, 1.0, False)])
def test_ndc_rays(dv, planes, step, masked):
    rng = np.random.default_rng(105)
    o, d = synth.scenes.forward_facing_rays(rng, 2000, spread=0.3, tilt_deg=6.0, **FF)
    d[:3] = np.float32([[0, 0, 1], [1, 0, 0], [0, 0, -1]])      # backwards, sideways, central
    mask = (rng.random((24, 20, planes)) < 0.5).astype(np.uint8) if masked else None
    say("NDC rays, planes", planes, "step", step, "masked", masked)
    got = _gpu_ndc(dv, o, d, planes, step, mask=mask)
    want = oracle.sample_ndc(o, d, BOX[0], BOX[1], FX, FY, 1.0, planes, step, 4096, mask)
    _same(got, want, keys=("ray_offsets", "xyz", "delta", "s_mid", "s_len"))
    n = np.diff(want["ray_offsets"])
    assert n[0] == 0 and n[1] == 0
    if not masked:
        assert n[2] == int(np.floor((planes - 1) / step)) + 1


def test_ndc_full_size_mpi(dv):
    # section 5.3's volume: 256 planes of 384 x 384, step 1 plane; 8192 rays, a mask with blobs
    rng = np.random.default_rng(106)
    o, d = synth.scenes.forward_facing_rays(rng, 8192, **FF)
    shape = (384, 384, 256)
    mask = np.zeros(shape, np.uint8)
    for _ in range(40):
        c = rng.integers(0, shape)
        r = rng.integers(8, 40, 3)
        mask[max(c[0] - r[0], 0):c[0] + r[0], max(c[1] - r[1], 0):c[1] + r[1], max(c[2] - r[2], 0):c[2] + r[2]] = 1
    say("NDC full size 384x384x256, 8192 rays, mask active", round(float(mask.mean()), 3))
    got = _gpu_ndc(dv, o, d, 256, 1.0, mask=mask)
    want = oracle.sample_ndc(o, d, BOX[0], BOX[1], FX, FY, 1.0, 256, 1.0, 4096, mask)
    _same(got, want, keys=("ray_offsets", "xyz", "delta", "s_mid", "s_len"))
    assert want["ray_offsets"][-1] > 8192 * 5


def test_no_rays(dv):
    spec = dv.SamplerSpec(BOX[0], BOX[1], 0.02, 0.02)
    e = torch.empty(0, 3, device="cuda")
    offs = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    dv.sample_count(spec, e, e, ray_offsets=offs)
    assert offs.item() == 0


# ------------------------------------------------------------------ occupancy


def f32(v):
    # the entry point takes float32 arguments; the oracle is handed the same values
    return float(np.float32(v))


def _occ_gpu(dv, raw, b, delta, thr, mask):
    g = dv.DeviceGrid(T(raw[..., None]), BOX[0], BOX[1])
    m = T(mask, torch.uint8).reshape(-1)
    dv.occupancy_update(g, b, delta, thr, m)
    torch.cuda.synchronize()
    return m.cpu().numpy().reshape(raw.shape)


def _grid1(raw):
    return synth.Grid(np.ascontiguousarray(raw[..., None], np.float32), BOX[0], BOX[1])


@pytest.mark.parametrize("shape,thr", [((9, 8, 10), 1e-3), ((2, 3, 2), 1e-3), ((33, 17, 65), 0.05),
                                       ((7, 7, 7), 0.0), ((6, 5, 4), 0.9999)])
def test_occupancy_small(dv, shape, thr):
    rng = np.random.default_rng(103)
    raw = rng.uniform(-10.0, 6.0, shape).astype(np.float32)
    old = (rng.random(shape) < 0.85).astype(np.uint8) * rng.integers(1, 255, shape).astype(np.uint8)
    b, thr = f32(oracle.act_shift()), f32(thr)
    say("occupancy", shape, "thr", thr)
    got = _occ_gpu(dv, raw, b, 0.5, thr, old)
    want = oracle.occupancy_update(_grid1(raw), b, 0.5, thr, old)
    np.testing.assert_array_equal(got, want)


def test_occupancy_full_size_then_sample(dv):
    # the fine-stage scene: 160^3 blob density, mask at a half-voxel step and alpha 1e-3, then
    # 8192 pinhole rays sampled at a half-voxel step through that mask
    w = synth.scenes.config2(R=8192)
    raw = w.density.data[..., 0]
    b, thr = f32(oracle.act_shift()), f32(1e-3)
    say("occupancy 160^3")
    got_mask = _occ_gpu(dv, raw, b, 0.5, thr, np.ones(raw.shape, np.uint8))
    want_mask = oracle.occupancy_update(w.density, b, 0.5, thr)
    np.testing.assert_array_equal(got_mask, want_mask)
    frac = want_mask.mean()
    assert 0.02 < frac < 0.9, frac
    voxel = w.density.voxel_size()
    say("sampler 8192 rays, 160^3 mask, active fraction", round(float(frac), 3))
    got = _gpu(dv, w.rays.origins, w.rays.dirs, 0.5 * voxel, voxel, mask=want_mask)
    want = oracle.sample_rays(w.rays.origins, w.rays.dirs, w.density.xyz_min, w.density.xyz_max, 0.0, 0.5 * voxel,
                              voxel, 4096, want_mask)
    _same(got, want)
    full = oracle.sample_rays(w.rays.origins, w.rays.dirs, w.density.xyz_min, w.density.xyz_max, 0.0, 0.5 * voxel,
                              voxel, 4096)
    say("kept", int(want["ray_offsets"][-1]), "of", int(full["ray_offsets"][-1]), "candidates")
