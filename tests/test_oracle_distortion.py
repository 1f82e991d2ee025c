"""Pins of the oracle's distortion loss (Eq. 1) and its gradient.

None of these re-types the oracle's formula: they use closed forms of Eq. 1, the
paper's own O(N) rewrite (Eq. 2 / Eq. 3 with its typo corrected), homogeneity,
symmetry and finite differences.
"""
import numpy as np
import pytest

import synth


def _single(w, m, l):
    offs = np.array([0, len(w)], np.int32)
    return offs, np.asarray(w, np.float64), np.asarray(m, np.float32), np.asarray(l, np.float32)


@pytest.mark.parametrize("N", [1, 2, 3, 7, 64, 128, 1000])
def test_uniform_box_closed_form(orc, N):
    # Uniform weights W/N on N equal intervals of [a, b]: the double sum of Eq. 1 plus the
    # 1/3 term is exactly W^2 (b - a) / 3 (the quadratic form of a flat density).
    a, b, W = 0.125, 0.875, 0.75
    edges = a + (b - a) * np.arange(N + 1) / N
    m = 0.5 * (edges[1:] + edges[:-1])
    l = np.diff(edges)
    offs, w, m32, l32 = _single(np.full(N, W / N), m, l)
    # the fp32 cast of m, l moves the exact value by O(1e-8)
    D = orc.distortion(offs, w, m32, l32)[0]
    assert abs(D - W * W * (b - a) / 3.0) < 1e-7


def test_single_interval_and_pair(orc):
    offs, w, m, l = _single([0.6], [0.3], [0.25])
    assert orc.distortion(offs, w, m, l)[0] == pytest.approx(0.36 * float(np.float32(0.25)) / 3, rel=1e-15)
    # two intervals: cross term 2 w0 w1 |m1 - m0|
    offs, w, m, l = _single([0.2, 0.5], [0.25, 0.75], [0.5, 0.5])
    expect = 2 * 0.2 * 0.5 * 0.5 + (0.04 * 0.5 + 0.25 * 0.5) / 3
    assert orc.distortion(offs, w, m, l)[0] == pytest.approx(expect, rel=1e-15)


def test_empty_rays(orc):
    offs = np.array([0, 0, 3, 3], np.int32)
    w = np.array([0.1, 0.2, 0.3])
    m = np.array([0.1, 0.5, 0.9], np.float32)
    l = np.array([0.2, 0.2, 0.2], np.float32)
    D = orc.distortion(offs, w, m, l)
    assert D[0] == 0.0 and D[2] == 0.0 and D[1] > 0


def test_paper_linear_rewrite_matches_definition(orc):
    rng = np.random.default_rng(0)
    lengths = [0, 1, 2, 3, 7, 63, 64, 65, 256]
    offs, w, m, l = synth.random_ragged(rng, lengths)
    Dd = orc.distortion(offs, w.astype(np.float64), m, l)
    Dp = orc.distortion(offs, w.astype(np.float64), m, l, form="prefix")
    np.testing.assert_allclose(Dp, Dd, rtol=1e-12, atol=1e-15)
    gd = orc.distortion_grad(offs, w.astype(np.float64), m, l)
    gp = orc.distortion_grad(offs, w.astype(np.float64), m, l, form="prefix")
    np.testing.assert_allclose(gp, gd, rtol=1e-10, atol=1e-13)


def test_homogeneity_and_invariances(orc):
    rng = np.random.default_rng(1)
    offs, w, m, l = synth.random_ragged(rng, [5, 17, 40])
    w = w.astype(np.float64)
    D = orc.distortion(offs, w, m, l)
    # 2-homogeneous in w
    np.testing.assert_allclose(orc.distortion(offs, 3.0 * w, m, l), 9.0 * D, rtol=1e-13)
    # shift of all midpoints leaves D unchanged; reflection s -> 1 - s (with order reversed)
    # leaves it unchanged as well
    m_shift = (m.astype(np.float64) + 0.5).astype(np.float32)
    Ds = orc.distortion(offs, w, m_shift, l)
    np.testing.assert_allclose(Ds, D, rtol=1e-6)
    wr, mr, lr = [], [], []
    for r in range(len(offs) - 1):
        sl = slice(offs[r], offs[r + 1])
        wr.append(w[sl][::-1]); mr.append((1.0 - m[sl].astype(np.float64))[::-1]); lr.append(l[sl][::-1])
    Dr = orc.distortion(offs, np.concatenate(wr), np.concatenate(mr).astype(np.float32), np.concatenate(lr))
    np.testing.assert_allclose(Dr, D, rtol=1e-6)


def test_gradient_euler_identity(orc):
    # D is 2-homogeneous in w, so sum_k w_k dD/dw_k = 2 D.
    rng = np.random.default_rng(2)
    offs, w, m, l = synth.random_ragged(rng, [1, 4, 33, 128])
    w = w.astype(np.float64)
    g = orc.distortion_grad(offs, w, m, l)
    D = orc.distortion(offs, w, m, l)
    per_ray = np.add.reduceat(w * g, offs[:-1])
    np.testing.assert_allclose(per_ray, 2.0 * D, rtol=1e-12)


def test_gradient_finite_differences(orc):
    rng = np.random.default_rng(3)
    offs, w, m, l = synth.random_ragged(rng, [3, 9, 20])
    w = w.astype(np.float64)
    gD = np.array([0.7, -1.3, 2.0])
    g = orc.distortion_grad(offs, w, m, l, gD)
    eps = 1e-6
    for k in range(len(w)):
        wp, wm = w.copy(), w.copy()
        wp[k] += eps
        wm[k] -= eps
        fd = (gD @ orc.distortion(offs, wp, m, l) - gD @ orc.distortion(offs, wm, m, l)) / (2 * eps)
        assert fd == pytest.approx(g[k], rel=1e-7, abs=1e-10)
