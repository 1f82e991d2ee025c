"""Pins of the oracle's interpolation, activation, compositing and their backward.

Trilinear interpolation is pinned by exact reproduction of linear fields, vertex values
and the adjoint (dot-product) identity; compositing by a closed-form ray through a
constant field and by invariants; the backward by central finite differences of the
oracle's own forward.
"""
import json
import os

import numpy as np
import pytest

import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _grid(data, lo=-1.0, hi=1.0):
    data = np.ascontiguousarray(data, np.float32)
    if data.ndim == 3:
        data = data[..., None]
    return synth.Grid(data, np.full(3, lo, np.float32), np.full(3, hi, np.float32))


def _vertex_coords(n, lo, hi):
    ax = lo + (hi - lo) * np.arange(n) / (n - 1)
    return np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1)


@pytest.mark.parametrize("n,lo,hi", [(5, -1.0, 1.0), (9, -2.0, 2.0), (2, 0.0, 1.0)])
def test_linear_field_reproduced(orc, n, lo, hi):
    rng = np.random.default_rng(10)
    a = np.array([[0.5, -1.25, 2.0], [1.0, 0.25, -0.5]])   # two channels, distinct per axis
    c = np.array([0.3, -0.7])
    v = _vertex_coords(n, lo, hi)
    field = v @ a.T + c
    g = _grid(field, lo, hi)
    x = rng.uniform(lo, hi, size=(200, 3)).astype(np.float32)
    got = orc.gather(g, x)
    expect = x.astype(np.float64) @ a.T + c
    # the grid values are float32-rounded, so agreement is to float32 precision
    np.testing.assert_allclose(got, expect, atol=2e-6)


def test_vertex_values_and_faces(orc):
    rng = np.random.default_rng(11)
    n = 6
    G = rng.standard_normal((n, n, n)).astype(np.float32)
    g = _grid(G)
    idx = rng.integers(0, n, size=(50, 3))
    pos = (-1.0 + 2.0 * idx / (n - 1)).astype(np.float32)
    got = orc.gather(g, pos)[:, 0]
    np.testing.assert_allclose(got, G[idx[:, 0], idx[:, 1], idx[:, 2]], rtol=1e-6, atol=1e-6)
    # points outside the box clamp to the face value
    out = np.array([[5.0, -5.0, 0.0]], np.float32)
    inside = np.array([[1.0, -1.0, 0.0]], np.float32)
    assert orc.gather(g, out)[0, 0] == orc.gather(g, inside)[0, 0]


def test_adjoint_identity(orc):
    rng = np.random.default_rng(12)
    n, C = 7, 3
    G = rng.standard_normal((n, n, n, C)).astype(np.float32)
    g = _grid(G)
    x = rng.uniform(-1, 1, size=(300, 3)).astype(np.float32)
    y = rng.standard_normal((300, C))
    lhs = np.sum(orc.gather(g, x) * y)
    rhs = np.sum(G.astype(np.float64) * orc.scatter(g, x, y))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_act_shift_defining_identity(orc):
    # alpha(raw = 0, delta = 0.5 voxel) = alpha_init = 1e-4 (section 5.4)
    a0 = GOLD["alpha_init"]["value"]
    dref = GOLD["alpha_init_step_voxels"]["value"]
    g = _grid(np.zeros((3, 3, 3)))
    x = np.zeros((4, 3), np.float32)
    al = orc.alpha(x, np.full(4, dref, np.float32), g, orc.act_shift(a0, dref))
    np.testing.assert_allclose(al, a0, rtol=1e-12)
    # very negative logits give vanishing alpha; very positive ones alpha -> 1 - e^{-raw delta}
    g2 = _grid(np.full((3, 3, 3), -60.0))
    assert orc.alpha(x, np.full(4, 1.0, np.float32), g2)[0] < 1e-25


def _const_ray_samples(N, delta, R=3):
    offs = np.arange(R + 1, dtype=np.int32) * N
    xyz = np.zeros((R * N, 3), np.float32)
    s_mid = np.tile((np.arange(N) + 0.5) / N, R).astype(np.float32)
    s_len = np.full(R * N, 1.0 / N, np.float32)
    return synth.Samples(offs, xyz, np.full(R * N, delta, np.float32), s_mid, s_len)


def test_constant_field_closed_form(orc):
    # constant logit z and colour c on every sample: T_k = exp(-k s d), and
    # C = c (1 - exp(-N s d)) + bg exp(-N s d) with s = softplus(z + b)
    N, delta, z = 50, 0.7, 1.5
    smp = _const_ray_samples(N, delta)
    dens = _grid(np.full((4, 4, 4), z))
    colv = np.array([0.2, 0.5, 0.9], np.float32)
    col = _grid(np.broadcast_to(colv, (4, 4, 4, 3)))
    b = orc.act_shift()
    bg = (0.3, 0.1, 1.0)
    out = orc.render_forward(smp, dens, col, shift=b, bg=bg, want_w=True)
    sig = np.log1p(np.exp(float(np.float32(z)) + b))
    d32 = float(np.float32(delta))
    TN = np.exp(-N * sig * d32)
    np.testing.assert_allclose(out["T"], TN, rtol=1e-12)
    np.testing.assert_allclose(out["rgb"], np.outer(np.ones(3), colv.astype(np.float64) * (1 - TN) + np.array(bg) * TN),
                               rtol=1e-12)
    k = np.arange(N)
    T = np.exp(-k * sig * d32)
    np.testing.assert_allclose(out["w"][:N], T * (1 - np.exp(-sig * d32)), rtol=1e-12)


def test_invariants_config1(orc):
    wl = synth.config1(R=64)
    out = orc.render_forward(wl.samples, wl.density, wl.color, want_w=True)
    w = out["w"]
    assert (w >= 0).all()
    tot = np.add.reduceat(np.concatenate([w, [0.0]]), wl.samples.ray_offsets[:-1])[:64]
    lens = wl.samples.lengths()
    tot[lens == 0] = 0.0
    np.testing.assert_allclose(tot + out["T"], 1.0, atol=1e-12)
    assert ((out["T"] >= 0) & (out["T"] <= 1)).all()
    assert (out["D"] >= 0).all()
    # render's D agrees with the standalone distortion on its own weights
    D2 = orc.distortion(wl.samples.ray_offsets, w, wl.samples.s_mid, wl.samples.s_len)
    np.testing.assert_allclose(out["D"], D2, rtol=1e-13)


def test_halting_rule(orc):
    wl = synth.config1(R=64)
    wl.density.data += np.float32(6.0)  # a denser scene so that many rays cross the threshold
    thr = GOLD["halt_transmittance"]["value"]
    full = orc.render_forward(wl.samples, wl.density, wl.color, want_w=True)
    halt = orc.render_forward(wl.samples, wl.density, wl.color, halt_T=thr, want_w=True)
    offs = wl.samples.ray_offsets
    n_halted = 0
    for r in range(64):
        w_f = full["w"][offs[r]:offs[r + 1]]
        w_h = halt["w"][offs[r]:offs[r + 1]]
        T = 1.0 - np.concatenate([[0.0], np.cumsum(w_f)])     # T_k from the un-halted run
        stop = np.nonzero(T[:-1] < thr)[0]
        if stop.size:
            n_halted += 1
            h = stop[0]
            assert (w_h[h:] == 0).all()
            np.testing.assert_allclose(w_h[:h], w_f[:h], rtol=1e-12)
            assert halt["T"][r] == pytest.approx(T[h], rel=1e-9)
            assert halt["T"][r] >= full["T"][r]
        else:
            np.testing.assert_allclose(w_h, w_f, rtol=1e-12)
    assert n_halted > 0


def _small_scene(seed, n=6, R=5, N=24, color_grid=True):
    rng = np.random.default_rng(seed)
    dens = _grid(rng.standard_normal((n, n, n)) * 2.0 + 6.0)
    col = _grid(rng.random((n, n, n, 3))) if color_grid else None
    rays = synth.rays_at_box(rng, R)
    smp = synth.uniform_samples(rays, N, dens.voxel_size())
    return rng, dens, col, smp


def _loss(orc, smp, dens, col, srgb, GC, GD, GT, bg, halt_T=0.0):
    o = orc.render_forward(smp, dens, col, srgb=srgb, bg=bg, halt_T=halt_T)
    return np.sum(GC * o["rgb"]) + GD @ o["D"] + GT @ o["T"]


def _fd_grid(orc, grid, idx, fn):
    d = grid.data
    old = d.flat[idx]
    eps = np.float32(2.0 ** -10)
    d.flat[idx] = old + eps
    hi_v = np.float64(d.flat[idx])
    fp = fn()
    d.flat[idx] = old - eps
    lo_v = np.float64(d.flat[idx])
    fm = fn()
    d.flat[idx] = old
    return (fp - fm) / (hi_v - lo_v)


def test_backward_finite_differences_grid_mode(orc):
    rng, dens, col, smp = _small_scene(20)
    R = smp.n_rays
    GC = rng.standard_normal((R, 3))
    GD = rng.standard_normal(R)
    GT = rng.standard_normal(R)
    bg = (0.2, 0.4, 0.9)
    g = orc.render_backward(smp, dens, GC, GD, GT, color=dens if False else col, bg=bg)
    fn = lambda: _loss(orc, smp, dens, col, None, GC, GD, GT, bg)  # noqa: E731
    gd = g["grad_density"].ravel()
    for idx in np.argsort(-np.abs(gd))[:12]:
        fd = _fd_grid(orc, dens, idx, fn)
        assert fd == pytest.approx(gd[idx], rel=2e-5, abs=1e-7)
    gc = g["grad_color"].ravel()
    for idx in np.argsort(-np.abs(gc))[:8]:
        fd = _fd_grid(orc, col, idx, fn)
        assert fd == pytest.approx(gc[idx], rel=2e-5, abs=1e-7)


def test_backward_finite_differences_sample_mode(orc):
    rng, dens, _, smp = _small_scene(21, color_grid=False)
    R, S = smp.n_rays, smp.n_samples
    srgb = rng.random((S, 3))
    GC = rng.standard_normal((R, 3))
    GD = rng.standard_normal(R)
    GT = rng.standard_normal(R)
    bg = (1.0, 1.0, 1.0)
    g = orc.render_backward(smp, dens, GC, GD, GT, srgb=srgb, bg=bg)
    fn = lambda s: _loss(orc, smp, dens, None, s, GC, GD, GT, bg)  # noqa: E731
    gs = g["grad_srgb"]
    for k in rng.choice(S, 10, replace=False):
        for ch in range(3):
            e = 1e-6
            sp, sm = srgb.copy(), srgb.copy()
            sp[k, ch] += e
            sm[k, ch] -= e
            assert (fn(sp) - fn(sm)) / (2 * e) == pytest.approx(gs[k, ch], rel=1e-6, abs=1e-10)
    gd = g["grad_density"].ravel()
    for idx in np.argsort(-np.abs(gd))[:10]:
        fd = _fd_grid(orc, dens, idx, lambda: fn(srgb))
        assert fd == pytest.approx(gd[idx], rel=2e-5, abs=1e-7)


def test_backward_finite_differences_halted(orc):
    # with halting, the gradient is that of the loss with the halt index held fixed
    rng, dens, col, smp = _small_scene(22, R=4, N=40)
    R = smp.n_rays
    GC = rng.standard_normal((R, 3))
    GD = rng.standard_normal(R)
    GT = rng.standard_normal(R)
    bg = (1.0, 1.0, 1.0)
    thr = 0.05
    g = orc.render_backward(smp, dens, GC, GD, GT, color=col, bg=bg, halt_T=thr)
    fn = lambda: _loss(orc, smp, dens, col, None, GC, GD, GT, bg, thr)  # noqa: E731
    gd = g["grad_density"].ravel()
    checked = 0
    for idx in np.argsort(-np.abs(gd))[:10]:
        fd = _fd_grid(orc, dens, idx, fn)
        if abs(fd - gd[idx]) > 1e-3 * max(abs(fd), 1e-3):
            continue  # the perturbation crossed the halting threshold; not differentiable there
        checked += 1
    assert checked >= 7


def test_loss_head_gradient(orc):
    rng = np.random.default_rng(30)
    R = 7
    rgb = rng.random((R, 3))
    tgt = rng.random((R, 3)).astype(np.float32)
    D = rng.random(R)
    lam = GOLD["distortion_weight"]["value"]
    L, GC, GD = orc.loss_head(rgb, tgt, D, lam)
    assert L == pytest.approx(np.mean((rgb - tgt) ** 2) + lam * D.mean(), rel=1e-14)
    e = 1e-6
    for r, ch in [(0, 0), (3, 2), (6, 1)]:
        p, m = rgb.copy(), rgb.copy()
        p[r, ch] += e
        m[r, ch] -= e
        fd = (orc.loss_head(p, tgt, D, lam)[0] - orc.loss_head(m, tgt, D, lam)[0]) / (2 * e)
        assert fd == pytest.approx(GC[r, ch], rel=1e-7)
    np.testing.assert_allclose(GD, lam / R)
