"""Pins of the oracle's guarded resampling (occupied coarse bins cut into n_base equal
sub-intervals plus a share of n_extra allotted by the predicted probabilities).

Pinned by its closed forms (every bin occupied and no extras: plain uniform sampling; fallback
rays: the same; an isolated occupied bin: itself and its two neighbours; one-hot and uniform
probabilities), by the invariants of the sample layout (counts, ordering, coverage of exactly
the occupied bins), and by an exact-rational re-derivation of the extra allotment on random rays.
"""
from fractions import Fraction
from types import SimpleNamespace

import numpy as np
import pytest

B = 64


def _rays(R, rng=None):
    rng = rng or np.random.default_rng(0)
    o = rng.uniform(-1, 1, (R, 3)).astype(np.float32)
    d = rng.standard_normal((R, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    tn = np.full(R, 0.5, np.float32)
    tf = np.full(R, 3.0, np.float32)
    return SimpleNamespace(origins=o, dirs=d, t_near=tn, t_far=tf)


def test_all_occupied_without_extras_is_plain_uniform(orc):
    R = 5
    rays = _rays(R)
    w = np.full((R, B), 1e-3, np.float32)
    prob = np.random.default_rng(1).random((R, B)).astype(np.float32)
    out = orc.resample_guarded(prob, w, np.zeros(R, np.float32), 10.0, 4, 0, 1e-4, rays, 0.02)
    assert (out["counts"] == 4).all()
    assert np.array_equal(out["ray_offsets"], np.arange(R + 1) * 256)
    k = np.arange(256)
    for r in range(R):
        sm = out["s_mid"][256 * r:256 * (r + 1)]
        np.testing.assert_allclose(sm, (k + 0.5) / 256, rtol=0, atol=1e-15)
        np.testing.assert_allclose(out["s_len"][256 * r:256 * (r + 1)], 1 / 256, rtol=1e-15)
        t = 0.5 + sm * 2.5
        np.testing.assert_allclose(out["xyz"][256 * r:256 * (r + 1)], rays.origins[r] + t[:, None] * rays.dirs[r],
                                   rtol=0, atol=1e-12)
        np.testing.assert_allclose(out["delta"][256 * r:256 * (r + 1)], 2.5 / 256 / 0.02, rtol=1e-12)


def test_fallback_and_missing_rays(orc):
    R = 3
    rays = _rays(R)
    rays.t_far[2] = rays.t_near[2]  # misses the box
    w = np.zeros((R, B), np.float32)  # nothing occupied
    prob = np.full((R, B), 1 / B, np.float32)
    H = np.array([5.0, 1.0, 5.0], np.float32)
    out = orc.resample_guarded(prob, w, H, 4.0, 4, 32, 1e-4, rays, 0.02)
    assert (out["counts"][0] == 4).all()        # entropy above tau: plain uniform, no extras
    assert not out["counts"][1].any()           # nothing occupied: no samples at all
    assert not out["counts"][2].any()           # misses the box
    assert list(out["ray_offsets"]) == [0, 256, 256, 256]


@pytest.mark.parametrize("b", [0, 17, 63])
def test_isolated_bin_is_dilated_and_takes_the_extras(orc, b):
    R = 1
    rays = _rays(R)
    w = np.zeros((R, B), np.float32)
    w[0, b] = 2e-4
    prob = np.zeros((R, B), np.float32)
    prob[0, b] = 1.0
    out = orc.resample_guarded(prob, w, np.zeros(R, np.float32), 10.0, 4, 24, 1e-4, rays, 0.02)
    occ = [x for x in (b - 1, b, b + 1) if 0 <= x < B]
    want = np.zeros(B, np.int32)
    want[occ] = 4
    want[b] += 24
    assert np.array_equal(out["counts"][0], want)
    # a weight just below the threshold occupies nothing
    w[0, b] = np.nextafter(np.float32(1e-4), np.float32(0))
    out = orc.resample_guarded(prob, w, np.zeros(R, np.float32), 10.0, 4, 24, 1e-4, rays, 0.02)
    assert not out["counts"].any()


def test_uniform_and_zero_probabilities_share_extras_evenly(orc):
    R = 2
    rays = _rays(R)
    w = np.zeros((R, B), np.float32)
    w[:, 10:20] = 1.0                    # occupied: bins 9..20 (12 bins)
    prob = np.zeros((R, B), np.float32)
    prob[0, 9:21] = 0.25                 # uniform over the occupied bins
    out = orc.resample_guarded(prob, w, np.zeros(R, np.float32), 10.0, 4, 36, 1e-4, rays, 0.02)
    for r in range(R):                   # ray 1 has zero mass there: every occupied bin counts 1
        assert np.array_equal(out["counts"][r, 9:21], np.full(12, 7))
        assert not out["counts"][r, :9].any() and not out["counts"][r, 21:].any()


def _exact_counts(prob, w, n_base, n_extra, w_min):
    """The allotment re-derived with exact rationals (the float32 inputs are exact binary
    fractions), for comparison with the oracle's double arithmetic."""
    occ = []
    for b in range(B):
        mx = max(w[max(b - 1, 0):b + 2])
        occ.append(mx >= w_min)
    p = [Fraction(float(prob[b])) if occ[b] else Fraction(0) for b in range(B)]
    tot = sum(p)
    if tot == 0:
        p = [Fraction(1) if occ[b] else Fraction(0) for b in range(B)]
        tot = sum(p)
    out, S = [], Fraction(0)
    rnd = lambda x: (x + Fraction(1, 2)).__floor__()
    for b in range(B):
        if not occ[b]:
            out.append(0)
            continue
        lo = rnd(n_extra * S / tot)
        S += p[b]
        out.append(n_base + rnd(n_extra * S / tot) - lo)
    return out


def test_random_rays_layout_and_exact_allotment(orc):
    rng = np.random.default_rng(7)
    R = 40
    rays = _rays(R, rng)
    w = (rng.random((R, B)) ** 6).astype(np.float32) * np.float32(1e-2)
    w[rng.random((R, B)) < 0.6] = 0.0
    prob = rng.dirichlet(np.full(B, 0.3), size=R).astype(np.float32)
    n_base, n_extra, w_min = 4, 48, np.float32(1e-4)
    out = orc.resample_guarded(prob, w, np.zeros(R, np.float32), 10.0, n_base, n_extra, float(w_min), rays, 0.02)
    offs, counts = out["ray_offsets"], out["counts"]
    assert np.array_equal(np.diff(offs), counts.sum(1))
    for r in range(R):
        assert list(counts[r]) == _exact_counts(prob[r], w[r], n_base, n_extra, w_min)
        occ = counts[r] > 0
        if occ.any():
            assert counts[r].sum() == n_base * occ.sum() + n_extra
        sm = out["s_mid"][offs[r]:offs[r + 1]]
        sl = out["s_len"][offs[r]:offs[r + 1]]
        assert (np.diff(sm) > 0).all()
        np.testing.assert_allclose(sl.sum(), occ.sum() / B, rtol=1e-12)
        # every sample interval lies inside an occupied bin
        lo, hi = sm - sl / 2, sm + sl / 2
        bins = np.floor(sm * B).astype(int)
        assert occ[bins].all()
        assert (lo >= bins / B - 1e-15).all() and (hi <= (bins + 1) / B + 1e-15).all()
