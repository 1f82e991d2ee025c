"""Pins of the oracle's tolerance helpers: the ReLU-kink slack of the colour head, the
softmax / entropy of the proposal stage, and the magnitude the TV gradient is conditioned on.

Each helper widens or sets a parity bound, so each is checked against something other than
itself: torch float64 autograd with a forced ReLU mask (the slack must be exactly the move of
the gradient when a unit at its kink switches side, zero when no unit is near a kink, and it
must respect its threshold), torch float64 softmax and the closed forms of the entropy, and
the triangle inequality of the TV sum with its equality case.
"""
import numpy as np
import pytest
import torch

import synth

torch.set_num_threads(4)

F = 4


def _pe(d):
    d = torch.as_tensor(d, dtype=torch.float64)
    fr = [d * (2.0 ** q) for q in range(F)]
    return torch.cat([d] + [torch.sin(v) for v in fr] + [torch.cos(v) for v in fr], dim=-1)


def _torch_grads(mlp, feat, d, g, flip=None):
    """Gradients of sum(g * rgb) for one sample in float64, with the ReLU masks of the forward
    values, except unit flip = (layer, unit), whose mask is inverted.  Forward values stay
    relu(z) (a unit at its kink has z within rounding of 0, so inverting its mask changes only
    the backward).  Returns one vector: [dfeat, dW1, db1, dW2, db2, dW3, db3] (the oracle's order)."""
    W = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in mlp.W]
    b = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in mlp.b]
    f = torch.tensor(feat, dtype=torch.float64, requires_grad=True)
    x = torch.cat([f, _pe(d)])

    def relu_masked(z, layer):
        m = (z.detach() > 0).to(torch.float64)
        if flip is not None and flip[0] == layer:
            m[flip[1]] = 1.0 - m[flip[1]]
        return torch.relu(z.detach()) + (z - z.detach()) * m

    h1 = relu_masked(W[0] @ x + b[0], 1)
    h2 = relu_masked(W[1] @ h1 + b[1], 2)
    rgb = torch.sigmoid(W[2] @ h2 + b[2])
    (rgb * torch.tensor(g, dtype=torch.float64)).sum().backward()
    return np.concatenate([f.grad.numpy()] + [t.grad.numpy().ravel() for t in (W[0], b[0], W[1], b[1], W[2], b[2])])


def _ratios(mlp, x):
    """|z| / (|b| + sum |W x|) of every hidden unit of both layers (float64)."""
    W1, W2 = (np.asarray(w, np.float64) for w in mlp.W[:2])
    b1, b2 = (np.asarray(v, np.float64) for v in mlp.b[:2])
    z1 = W1 @ x + b1
    r1 = np.abs(z1) / (np.abs(b1) + np.abs(W1 * x).sum(axis=1))
    h1 = np.maximum(z1, 0.0)
    z2 = W2 @ h1 + b2
    r2 = np.abs(z2) / (np.abs(b2) + np.abs(W2 * h1).sum(axis=1))
    return r1, r2, h1


def _kink_case(seed=70):
    """One sample and a colour head with unit a of layer 1 exactly at its kink (|z| at float32
    rounding), unit c of layer 1 at 5e-5 of its magnitude, and unit e of layer 2 at its kink;
    every other unit at least 2e-4 of its magnitude away from its kink (beyond every threshold
    tested)."""
    rng = np.random.default_rng(seed)
    mlp = synth.mlp_weights(rng, bias_std=0.3)
    feat = rng.standard_normal(12)
    d = synth.scenes._unit(rng.standard_normal((1, 3))).astype(np.float32)
    x = np.concatenate([feat, _pe(d[0].astype(np.float64)).numpy()])
    W1 = np.asarray(mlp.W[0], np.float64)
    a, c = 5, 77
    mag_c = np.abs(mlp.b[0][c]) + np.abs(W1[c] * x).sum()
    mlp.b[0][a] = np.float32(-(W1[a] @ x))
    mlp.b[0][c] = np.float32(-(W1[c] @ x) + 5e-5 * mag_c)
    r1, _, h1 = _ratios(mlp, x)
    e = int(np.argmax(np.asarray(mlp.W[1], np.float64) @ h1 != 0))  # any unit of layer 2
    mlp.b[1][e] = np.float32(-(np.asarray(mlp.W[1][e], np.float64) @ h1))
    r1, r2, _ = _ratios(mlp, x)
    assert r1[a] < 1e-6 and 3e-5 < r1[c] < 8e-5 and r2[e] < 1e-6
    others1 = np.delete(r1, [a, c])
    others2 = np.delete(r2, [e])
    assert others1.min() > 2e-4 and others2.min() > 2e-4, "seed gives a unit near its kink by chance"
    g = rng.standard_normal(3)
    return mlp, feat, d, g, (a, c, e)


def _oracle_slack(orc, mlp, feat, d, g, thr):
    offs = np.array([0, 1], np.int32)
    sf, sW, sb = orc.mlp_kink_slack(mlp, offs, d, feat[None, :], g[None, :], thr=thr)
    return np.concatenate([sf.ravel()] + [t.ravel() for t in (sW[0], sb[0], sW[1], sb[1], sW[2], sb[2])])


def test_kink_slack_equals_gradient_move_at_the_kink(orc):
    mlp, feat, d, g, (a, c, e) = _kink_case()
    base = _torch_grads(mlp, feat, d[0], g)
    move_a = np.abs(_torch_grads(mlp, feat, d[0], g, flip=(1, a)) - base)
    move_c = np.abs(_torch_grads(mlp, feat, d[0], g, flip=(1, c)) - base)
    move_e = np.abs(_torch_grads(mlp, feat, d[0], g, flip=(2, e)) - base)
    assert move_a.max() > 0 and move_c.max() > 0 and move_e.max() > 0
    # thr 1e-5: the two units at their kinks count, the one at 5e-5 does not
    s = _oracle_slack(orc, mlp, feat, d, g, thr=1e-5)
    np.testing.assert_allclose(s, move_a + move_e, rtol=1e-9, atol=1e-14)
    # thr 1e-4: all three
    s = _oracle_slack(orc, mlp, feat, d, g, thr=1e-4)
    np.testing.assert_allclose(s, move_a + move_c + move_e, rtol=1e-9, atol=1e-14)
    # thr 1e-7: only units within 1e-7 of their magnitude (the two at float32 rounding)
    s = _oracle_slack(orc, mlp, feat, d, g, thr=1e-7)
    np.testing.assert_allclose(s, move_a + move_e, rtol=1e-9, atol=1e-14)


def test_kink_slack_is_zero_away_from_kinks(orc):
    # samples drawn at random, keeping those whose every hidden unit is beyond the threshold
    rng = np.random.default_rng(71)
    mlp = synth.mlp_weights(rng, bias_std=0.3)
    dirs = synth.scenes._unit(rng.standard_normal((3, 3))).astype(np.float32)
    rows = [[], [], []]
    for k in range(60):
        r = k % 3
        f = rng.standard_normal(12)
        x = np.concatenate([f, _pe(dirs[r].astype(np.float64)).numpy()])
        r1, r2, _ = _ratios(mlp, x)
        if min(r1.min(), r2.min()) > 1e-5:
            rows[r].append(f)
    assert sum(len(v) for v in rows) >= 30
    feat = np.concatenate([np.asarray(v).reshape(-1, 12) for v in rows])
    offs = np.concatenate([[0], np.cumsum([len(v) for v in rows])]).astype(np.int32)
    S = int(offs[-1])
    sf, sW, sb = orc.mlp_kink_slack(mlp, offs, dirs, feat, rng.standard_normal((S, 3)), thr=1e-5)
    assert not sf.any() and not any(t.any() for t in sW) and not any(t.any() for t in sb)


def test_softmax_entropy_matches_torch_and_closed_forms(orc):
    rng = np.random.default_rng(72)
    lg = rng.standard_normal((50, 64)) * 3.0
    lg[0] = 0.0                      # uniform: H = ln 64
    lg[1] = 0.0
    lg[1, 17] = 1000.0               # one dominant logit: p one-hot, H = 0
    lg[2] = np.linspace(-700, 700, 64)  # extreme range (no overflow)
    p, H = orc.softmax_entropy(lg)
    t = torch.tensor(lg, dtype=torch.float64)
    tp = torch.softmax(t, dim=1)
    tH = -(tp * torch.log_softmax(t, dim=1)).sum(dim=1)
    np.testing.assert_allclose(p, tp.numpy(), rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(H, tH.numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(H[0], np.log(64.0), rtol=1e-14)
    np.testing.assert_allclose(p[0], 1.0 / 64.0, rtol=1e-15)
    assert p[1, 17] == 1.0 and H[1] == 0.0
    np.testing.assert_allclose(p.sum(axis=1), 1.0, rtol=1e-14)
    assert (H >= 0).all() and (H <= np.log(64.0) + 1e-14).all()


def _tv_grid(data):
    data = np.ascontiguousarray(data, np.float32)
    return synth.Grid(data, np.full(3, -1.0, np.float32), np.full(3, 1.0, np.float32))


@pytest.mark.parametrize("C", [1, 4])
def test_tv_magnitude_bounds_the_gradient(orc, C):
    # mag = coef * sum_n |clamp(v_p - v_n)| >= |coef * sum_n clamp(v_p - v_n)| = |grad| everywhere
    # (triangle inequality), with equality exactly where all the clamped differences share a sign
    rng = np.random.default_rng(73 + C)
    data = rng.standard_normal((6, 5, 7, C)).astype(np.float32)
    delta = 0.6
    _, grad, mag = orc.tv(_tv_grid(data), 0.3, delta, dense=True, want_mag=True)
    assert (mag >= np.abs(grad) * (1 - 1e-14)).all()
    v = data.astype(np.float64)
    same_sign = np.ones(v.shape, bool)
    pos = np.zeros(v.shape, bool)
    neg = np.zeros(v.shape, bool)
    for ax in range(3):
        for sh in (1, -1):
            nb = np.roll(v, sh, axis=ax)
            valid = np.ones(v.shape, bool)
            idx = [slice(None)] * 4
            idx[ax] = 0 if sh == 1 else -1
            valid[tuple(idx)] = False
            dlt = np.clip(v - nb, -delta, delta)
            pos |= valid & (dlt > 0)
            neg |= valid & (dlt < 0)
    same_sign = ~(pos & neg)
    np.testing.assert_allclose(mag[same_sign], np.abs(grad[same_sign]), rtol=1e-13, atol=0)
    assert (mag[~same_sign] > np.abs(grad[~same_sign])).all()
    assert same_sign.any() and (~same_sign).any()


def test_tv_magnitude_of_a_spike(orc):
    # a spike of height h above a zero field: at the spike every difference is +h (clamped to
    # delta), at its six neighbours the one difference is -h; elsewhere 0
    data = np.zeros((5, 5, 5, 1), np.float32)
    data[2, 2, 2, 0] = 2.0
    w, delta = 0.5, 0.75
    _, grad, mag = orc.tv(_tv_grid(data), w, delta, dense=True, want_mag=True)
    coef = 2.0 * w / (125 * 1)
    assert mag[2, 2, 2, 0] == pytest.approx(6 * delta * coef, rel=1e-15)
    for n in ((1, 2, 2), (3, 2, 2), (2, 1, 2), (2, 3, 2), (2, 2, 1), (2, 2, 3)):
        assert mag[n + (0,)] == pytest.approx(delta * coef, rel=1e-15)
    np.testing.assert_array_equal(mag, np.abs(grad))
    assert np.count_nonzero(mag) == 7
