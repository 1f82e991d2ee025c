"""Pins of the oracle's forward-facing sampler (section 5.3: NeRF's normalised device coordinates,
D planes at fixed depths, rays traced from the first plane to the last at a step of s planes).

Pinned by the paper's own count (2D - 1 points at s = 0.5), the central ray's plane depths in
closed form, the defining property of the NDC ray (every emitted point is the NDC projection of a
world point on the original ray, checked with an independent float64 projection), a float64
brute force of which samples stay inside the box, rays that never reach the near plane, and the
mask.
"""
import numpy as np
import pytest

import synth

BOX = (np.full(3, -1.0, np.float32), np.full(3, 1.0, np.float32))
W, H, F = 1008, 756, 815.0
FX, FY = 2 * F / W, 2 * F / H


def _ndc(orc, o, d, planes, step, near=1.0, mask=None, cap=4096):
    return orc.sample_ndc(np.asarray(o, np.float32), np.asarray(d, np.float32), BOX[0], BOX[1], FX, FY, near,
                          planes, step, cap, mask)


@pytest.mark.parametrize("D", [4, 8, 64, 256])
def test_two_d_minus_one_points_at_half_step(orc, D):
    # section 5.3: tracing from the first to the D-th plane with s = 0.5 gives 2D - 1 points
    r = _ndc(orc, [[0, 0, 0]], [[0, 0, -1]], D, 0.5)
    assert r["ray_offsets"].tolist() == [0, 2 * D - 1]
    r = _ndc(orc, [[0, 0, 0]], [[0, 0, -1]], D, 1.0)
    assert r["ray_offsets"].tolist() == [0, D]


def test_central_ray_closed_form(orc):
    D, s = 8, 0.5
    r = _ndc(orc, [[0, 0, 0]], [[0, 0, -1]], D, s)
    j = np.arange(2 * D - 1)
    assert not r["xyz"][:, :2].any()
    np.testing.assert_allclose(r["xyz"][:, 2], -1.0 + 2.0 * j * s / (D - 1), atol=2e-7)
    np.testing.assert_allclose(r["s_mid"], (j + 0.5) / (2 * D - 1), rtol=1e-7)
    assert (r["delta"] == np.float32(s)).all() and (r["s_len"] == np.float32(1 / (2 * D - 1))).all()


def test_points_are_projections_of_the_world_ray(orc):
    rng = np.random.default_rng(120)
    o, d = synth.scenes.forward_facing_rays(rng, 400)
    near = 1.0
    r = _ndc(orc, o, d, 64, 1.0, near=near)
    n = np.diff(r["ray_offsets"])
    ray = np.repeat(np.arange(len(o)), n)
    keep = r["xyz"][:, 2] < 0.98             # depth -> infinity as z' -> 1
    x = r["xyz"][keep].astype(np.float64)
    ray = ray[keep]
    oo, dd = o[ray].astype(np.float64), d[ray].astype(np.float64)
    z = 2.0 * near / (x[:, 2] - 1.0)         # world depth of the NDC depth
    t = (z - oo[:, 2]) / dd[:, 2]
    X = oo + t[:, None] * dd
    proj = np.stack([-FX * X[:, 0] / X[:, 2], -FY * X[:, 1] / X[:, 2], 1.0 + 2.0 * near / X[:, 2]], axis=1)
    np.testing.assert_allclose(x, proj, atol=5e-5)
    assert keep.mean() > 0.9


def test_inside_box_brute_force(orc):
    rng = np.random.default_rng(121)
    o, d = synth.scenes.forward_facing_rays(rng, 600, spread=0.4, tilt_deg=8.0)
    D, s, near = 32, 0.5, 1.0
    r = _ndc(orc, o, d, D, s, near=near)
    # float64: NDC ray, then the points at t' = j s / (D - 1)
    o64, d64 = o.astype(np.float64), d.astype(np.float64)
    t0 = -(near + o64[:, 2]) / d64[:, 2]
    p = o64 + t0[:, None] * d64
    on = np.stack([-FX * p[:, 0] / p[:, 2], -FY * p[:, 1] / p[:, 2], 1 + 2 * near / p[:, 2]], axis=1)
    dn = np.stack([-FX * (d64[:, 0] / d64[:, 2] - p[:, 0] / p[:, 2]),
                   -FY * (d64[:, 1] / d64[:, 2] - p[:, 1] / p[:, 2]), -2 * near / p[:, 2]], axis=1)
    j = np.arange(2 * D - 1)
    pts = on[:, None, :] + (j * s / (D - 1))[None, :, None] * dn[:, None, :]
    # kept when inside across the image axes (depth runs from face to face by construction)
    inside = (np.abs(pts[..., :2]) <= 1.0).all(axis=2)
    margin = np.abs(np.abs(pts[..., :2]) - 1.0).min(axis=2) < 1e-5
    clear = ~margin.any(axis=1)
    assert clear.mean() > 0.95
    n = np.diff(r["ray_offsets"])
    np.testing.assert_array_equal(n[clear], inside.sum(axis=1)[clear])
    assert (n < 2 * D - 1).sum() > 50      # the spread makes many rays leave the volume


def test_rays_that_never_reach_the_near_plane(orc):
    r = _ndc(orc, [[0, 0, 0], [0.1, 0, 0], [0, 0, 0]], [[0, 0, 1], [1, 0, 0], [0, 0, -1]], 16, 1.0)
    assert r["ray_offsets"].tolist() == [0, 0, 0, 16]


def test_mask(orc):
    rng = np.random.default_rng(122)
    o, d = synth.scenes.forward_facing_rays(rng, 300)
    full = _ndc(orc, o, d, 16, 0.5)
    ones = _ndc(orc, o, d, 16, 0.5, mask=np.ones((9, 9, 16), np.uint8))
    for k in ("ray_offsets", "xyz", "s_mid"):
        np.testing.assert_array_equal(ones[k], full[k])
    none = _ndc(orc, o, d, 16, 0.5, mask=np.zeros((9, 9, 16), np.uint8))
    assert none["ray_offsets"][-1] == 0
    # a mask that keeps only the far half of the planes keeps exactly the points on those planes
    # (step 1: every point sits on a plane, so the nearest vertex along depth is unambiguous)
    full = _ndc(orc, o, d, 16, 1.0)
    m = np.zeros((9, 9, 16), np.uint8)
    m[:, :, 8:] = 1
    half = _ndc(orc, o, d, 16, 1.0, mask=m)
    u = (full["xyz"][:, 2].astype(np.float64) + 1.0) / 2.0 * 15
    far = np.rint(u) >= 8
    ambiguous = np.abs(u - np.floor(u) - 0.5) < 1e-5
    assert not ambiguous.any()
    np.testing.assert_array_equal(half["xyz"], full["xyz"][far])
