"""Pins of the oracle's sample producer: parsimonious sampling inside the scene box (section 3,
re-implemented rendering utilities) and the occupancy mask that switches off empty space
(section 1).

The sampler is pinned by closed forms (axis-aligned rays with dyadic sizes, misses, an origin
inside the box), by float64 geometry computed independently with numpy (the slab interval of
the input generator, candidate counts and positions), by the cap, and by a brute-force numpy
nearest-vertex selection for the mask.  The mask update is pinned by numpy brute force (alpha
in double, 27-neighbour dilation by array shifts), by a single dense vertex, by the alpha_init
identity of the activation and by its monotonicity.
"""
import numpy as np

import synth
from synth.scenes import slab_interval

BOX = (np.full(3, -1.0, np.float32), np.full(3, 1.0, np.float32))


def _sample(orc, o, d, near=0.0, step=0.25, voxel=0.25, cap=100000, mask=None, box=BOX):
    return orc.sample_rays(np.asarray(o, np.float32), np.asarray(d, np.float32), box[0], box[1], near, step, voxel,
                           cap, mask)


def test_axis_aligned_ray_closed_form(orc):
    # along +x from x = -3: enters at t = 2, leaves at t = 4; a 0.25 step gives 8 candidates at
    # x = -0.875 + 0.25 k with s_mid = (k + 1/2)/8, s_len = 1/8, delta = step / voxel
    r = _sample(orc, [[-3, 0.1, 0.2]], [[1, 0, 0]], step=0.25, voxel=0.125)
    assert r["ray_offsets"].tolist() == [0, 8]
    assert r["t_near"][0] == 2.0 and r["t_far"][0] == 4.0
    k = np.arange(8)
    np.testing.assert_array_equal(r["xyz"][:, 0], (-0.875 + 0.25 * k).astype(np.float32))
    np.testing.assert_array_equal(r["xyz"][:, 1:], np.tile(np.float32([0.1, 0.2]), (8, 1)))
    np.testing.assert_array_equal(r["s_mid"], ((k + 0.5) / 8).astype(np.float32))
    assert (r["s_len"] == np.float32(1 / 8)).all() and (r["delta"] == 2.0).all()


def test_misses_and_rays_pointing_away(orc):
    o = [[-3, 5, 0], [3, 0, 0], [-3, 0.5, 0.5], [0, 0, -3]]
    d = [[1, 0, 0], [1, 0, 0], [0, 1, 0], [0.6, 0, -0.8]]
    r = _sample(orc, o, d)
    assert r["ray_offsets"].tolist() == [0, 0, 0, 0, 0]
    assert not r["t_near"].any() and not r["t_far"].any()


def test_origin_inside_box_starts_at_near(orc):
    # t_near = near = 0.125, exit at t = 1: candidates at t = 0.25, 0.5, 0.75 (t = 1 is not < exit)
    r = _sample(orc, [[0, 0, 0]], [[0, 0, 1]], near=0.125, step=0.25)
    assert r["ray_offsets"].tolist() == [0, 3]
    assert r["t_near"][0] == 0.125 and r["t_far"][0] == 1.0
    np.testing.assert_array_equal(r["xyz"][:, 2], np.float32([0.25, 0.5, 0.75]))
    # a near plane beyond the exit: no samples
    r = _sample(orc, [[0, 0, 0]], [[0, 0, 1]], near=1.5)
    assert r["ray_offsets"].tolist() == [0, 0]


def test_cap_on_candidates(orc):
    r = _sample(orc, [[-3, 0.1, 0.2], [-3, 0.1, 0.2]], [[1, 0, 0], [1, 0, 0]], step=0.01, cap=37)
    assert r["ray_offsets"].tolist() == [0, 37, 74]
    # s stays normalised over the capped count
    np.testing.assert_array_equal(r["s_mid"][:37], ((np.arange(37) + 0.5) / 37).astype(np.float32))


def test_random_rays_match_float64_geometry(orc):
    rng = np.random.default_rng(90)
    rays = synth.scenes.pinhole_rays(rng, 3000)
    step = 2.0 / 159 * 0.5
    r = _sample(orc, rays.origins, rays.dirs, step=step, voxel=2.0 / 159)
    o = rays.origins.astype(np.float64)
    d = rays.dirs.astype(np.float64)
    tn, tf, hit = slab_interval(o, d, BOX[0].astype(np.float64), BOX[1].astype(np.float64))
    np.testing.assert_allclose(r["t_near"], np.where(hit, tn, 0), atol=2e-6)
    np.testing.assert_allclose(r["t_far"], np.where(hit, tf, 0), atol=2e-6)
    c = (tf - tn) / np.float64(np.float32(step)) - 0.5
    n64 = np.where(hit & (c > 0), np.ceil(c), 0).astype(np.int64)
    n = np.diff(r["ray_offsets"])
    clear = np.abs(c - np.round(c)) > 1e-3
    assert clear.mean() > 0.99
    np.testing.assert_array_equal(n[clear], n64[clear])
    assert np.abs(n - n64).max() <= 1
    assert n.sum() > 100 * 3000
    # every point lies on its ray at t_k = t_near + (k + 1/2) step and inside the box
    ray = np.repeat(np.arange(3000), n)
    k = r["s_mid"].astype(np.float64) * n[ray] - 0.5
    np.testing.assert_allclose(k, np.round(k), atol=1e-3)
    t = tn[ray] + (np.round(k) + 0.5) * np.float64(np.float32(step))
    np.testing.assert_allclose(r["xyz"], o[ray] + t[:, None] * d[ray], atol=1e-5)
    assert np.abs(r["xyz"]).max() <= 1.0 + 1e-5
    assert (r["delta"] == np.float32(np.float32(step) / np.float32(2.0 / 159))).all()


def test_mask_selection_matches_brute_force(orc):
    rng = np.random.default_rng(91)
    mshape = (7, 9, 11)
    mask = (rng.random(mshape) < 0.4).astype(np.uint8)
    rays = synth.scenes.rays_at_box(rng, 500)
    full = _sample(orc, rays.origins, rays.dirs, step=0.05)
    kept = _sample(orc, rays.origins, rays.dirs, step=0.05, mask=mask)
    # nearest vertex in float64 from the float32 points of the unmasked run
    x = full["xyz"].astype(np.float64)
    u = (x + 1.0) / 2.0 * (np.array(mshape) - 1)
    idx = np.clip(np.rint(u), 0, np.array(mshape) - 1).astype(np.int64)
    live = mask[idx[:, 0], idx[:, 1], idx[:, 2]] != 0
    ambiguous = (np.abs(u - np.floor(u) - 0.5) < 1e-5).any(axis=1)
    assert ambiguous.sum() < 5
    n_full = np.diff(full["ray_offsets"])
    ray = np.repeat(np.arange(500), n_full)
    want_counts = np.bincount(ray[live], minlength=500)
    got_counts = np.diff(kept["ray_offsets"])
    if not ambiguous.any():
        np.testing.assert_array_equal(got_counts, want_counts)
        np.testing.assert_array_equal(kept["xyz"], full["xyz"][live])
        np.testing.assert_array_equal(kept["s_mid"], full["s_mid"][live])
        np.testing.assert_array_equal(kept["s_len"], full["s_len"][live])
    else:
        assert np.abs(got_counts - want_counts).sum() <= ambiguous.sum()
    # an all-active mask changes nothing
    ones = _sample(orc, rays.origins, rays.dirs, step=0.05, mask=np.ones(mshape, np.uint8))
    for key in ("ray_offsets", "xyz", "s_mid", "s_len", "delta"):
        np.testing.assert_array_equal(ones[key], full[key])


# ------------------------------------------------------------------ occupancy mask


def _grid1(raw):
    return synth.Grid(np.ascontiguousarray(raw[..., None], np.float32), BOX[0], BOX[1])


def _softplus(z):
    return np.logaddexp(0.0, z)


def test_occupancy_matches_brute_force(orc):
    rng = np.random.default_rng(92)
    shape = (9, 8, 10)
    raw = rng.uniform(-10.0, 3.0, shape).astype(np.float32)
    old = (rng.random(shape) < 0.8).astype(np.uint8)
    b, delta, thr = orc.act_shift(), 0.5, 1e-3
    got = orc.occupancy_update(_grid1(raw), b, delta, thr, old)
    alpha = -np.expm1(-_softplus(raw.astype(np.float64) + b) * delta)
    assert np.abs(alpha / thr - 1).min() > 1e-6          # no decision within rounding
    dense = np.pad(alpha >= thr, 1)
    near = np.zeros(shape, bool)
    for a in range(3):
        for c in range(3):
            for e in range(3):
                near |= dense[a:a + shape[0], c:c + shape[1], e:e + shape[2]]
    np.testing.assert_array_equal(got, (old.astype(bool) & near).astype(np.uint8))
    assert 0 < got.sum() < old.sum()


def test_occupancy_single_dense_vertex(orc):
    raw = np.full((6, 7, 8), -30.0, np.float32)
    raw[2, 3, 4] = 5.0
    raw[0, 0, 0] = 5.0
    got = orc.occupancy_update(_grid1(raw), orc.act_shift(), 0.5, 1e-3)
    want = np.zeros(raw.shape, np.uint8)
    want[1:4, 2:5, 3:6] = 1
    want[0:2, 0:2, 0:2] = 1
    np.testing.assert_array_equal(got, want)


def test_occupancy_alpha_init_identity(orc):
    # raw = 0 at delta = 0.5 has alpha = alpha_init = 1e-4 under the activation of section 5.4
    raw = np.zeros((3, 4, 5), np.float32)
    b = orc.act_shift(1e-4, 0.5)
    assert orc.occupancy_update(_grid1(raw), b, 0.5, 0.999e-4).all()
    assert not orc.occupancy_update(_grid1(raw), b, 0.5, 1.001e-4).any()


def test_occupancy_only_deactivates(orc):
    rng = np.random.default_rng(93)
    raw = rng.uniform(-10.0, 3.0, (8, 8, 8)).astype(np.float32)
    g = _grid1(raw)
    b = orc.act_shift()
    once = orc.occupancy_update(g, b, 0.5, 1e-3)
    twice = orc.occupancy_update(g, b, 0.5, 1e-3, once)
    np.testing.assert_array_equal(once, twice)
    old = (rng.random(raw.shape) < 0.5).astype(np.uint8)
    new = orc.occupancy_update(g, b, 0.5, 1e-3, old)
    assert not (new.astype(bool) & ~old.astype(bool)).any()
