"""Owner-computes scatter (every vertex summed by the 4x4x32-vertex brick that owns it, no atomics)
and its fusion with the zero-gradient-skipping Adam update, against the FP64 oracle and against
the two-call path (scatter, then Adam)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import FWD, GRAD, close, close_after_adam

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


def _pairs(ws, nb, S):
    raw = ws.cpu().numpy().view(np.int32)
    offs = raw[:nb + 1]
    perm_at = ((4 * (nb + 1) + 255) // 256 * 256 + (4 * nb + 255) // 256 * 256) // 4
    return offs, raw[perm_at:perm_at + int(offs[-1])]


@pytest.mark.parametrize("n,C,warp", [(24, 1, 0), (17, 3, 0), (40, 12, 0), (33, 12, 1), (9, 16, 0), (21, 8, 2),
                                      (160, 12, 0)])
def test_owner_scatter(dv, n, C, warp):
    # points along the config-2 rays (runs of consecutive samples in one cell), uniform points
    # (ragged tail, faces, outside the box); the bins hold every sample 1, 2, 4 or 8 times
    rng = np.random.default_rng(40 + n + C)
    g = synth.normal_grid(rng, n, C, -2.0, 2.0) if warp else synth.normal_grid(rng, n, C)
    g.warp = warp
    wl = synth.config2(R=64)
    xyz = wl.samples.xyz
    if warp:
        xyz = (xyz * 5.0).astype(np.float32)
    extra = rng.uniform(-1.2, 1.2, (3001, 3)).astype(np.float32)
    extra[:6] = [[1, 1, 1], [-1, -1, -1], [1, -1, 0], [0, 0, 1], [-1.5, 0, 0], [0.0, 2.0, 0.0]]
    xyz = np.concatenate([xyz, extra])
    S = xyz.shape[0]
    y = rng.standard_normal((S, C)).astype(np.float32)
    say("owner scatter n =", n, "C =", C, "warp", warp, "S =", S)
    dg = dgrid(dv, g, grad=True)
    ws = dv.owner_bin(dg, T(xyz))
    dv.grid_scatter_owned(dg, T(xyz), T(y), ws)
    torch.cuda.synchronize()
    nb = ((n + 3) // 4) ** 2 * ((n + 31) // 32)
    offs, perm = _pairs(ws, nb, S)
    assert offs[0] == 0 and (np.diff(offs) >= 0).all() and S <= offs[-1] <= 8 * S
    mult = np.bincount(perm, minlength=S)
    assert set(np.unique(mult)) <= {1, 2, 4, 8}
    close(dg.grad.cpu().numpy(), oracle.scatter(g, xyz, y.astype(np.float64)), **GRAD, name="owner scatter")


def test_owner_scatter_accumulates_and_empty(dv):
    # += into an existing gradient; an empty batch leaves it unchanged
    rng = np.random.default_rng(47)
    g = synth.normal_grid(rng, 20, 4)
    xyz = rng.uniform(-1, 1, (4000, 3)).astype(np.float32)
    y = rng.standard_normal((4000, 4)).astype(np.float32)
    g0 = rng.standard_normal(g.data.shape).astype(np.float32)
    say("owner scatter into a non-zero gradient; empty batch")
    dg = dgrid(dv, g)
    dg.grad = T(g0)
    ws = dv.owner_bin(dg, T(xyz))
    dv.grid_scatter_owned(dg, T(xyz), T(y), ws)
    empty = torch.zeros(0, 3, device="cuda")
    ws0 = dv.owner_bin(dg, empty)
    dv.grid_scatter_owned(dg, empty, torch.zeros(0, 4, device="cuda"), ws0)
    torch.cuda.synchronize()
    close(dg.grad.cpu().numpy(), g0 + oracle.scatter(g, xyz, y.astype(np.float64)), **GRAD, name="accumulate")


def _adam_pair(dv, g, xyz, y, steps, lr=0.1):
    """Runs the fused update and the two-call path (owner scatter into a zeroed gradient, then the
    skipping Adam step) for `steps` steps on the same data; returns both (p, m, v)."""
    out = []
    for fused in (True, False):
        dg = dgrid(dv, g, grad=True)
        m, v = torch.zeros_like(dg.data), torch.zeros_like(dg.data)
        t = torch.zeros(1, dtype=torch.int32, device="cuda")
        ws = dv.owner_bin(dg, T(xyz))
        for _ in range(steps):
            dv.counter_add(t, 1)
            if fused:
                dv.grid_scatter_adam(dg, T(xyz), T(y), ws, m, v, lr=lr, step_dev=t)
            else:
                dv.grid_scatter_owned(dg, T(xyz), T(y), ws)
                dv.grid_adam_step(dg.data, dg.grad, m, v, lr=lr, step_dev=t, skip_zero_grad=True,
                                  zero_grad_after=True)
        torch.cuda.synchronize()
        out.append(tuple(a.cpu().numpy() for a in (dg.data, m, v)))
    return out


@pytest.mark.parametrize("C", [1, 12])
def test_scatter_adam_bitwise_on_distinct_vertices(dv, C):
    # every point sits exactly on its own vertex (box [0, n-1]: integer coordinates, weights 0/1),
    # so each gradient is one exact term and both paths must agree bit for bit, including the
    # untouched elements (skipped) and the line-wide write-back of unchanged elements
    n = 24
    rng = np.random.default_rng(48 + C)
    data = rng.standard_normal((n, n, n, C)).astype(np.float32)
    g = synth.Grid(data, np.zeros(3, np.float32), np.full(3, n - 1, np.float32))
    verts = rng.choice(n ** 3, 3000, replace=False)
    xyz = np.stack(np.unravel_index(verts, (n, n, n)), axis=1).astype(np.float32)
    y = rng.standard_normal((3000, C)).astype(np.float32)
    y[::7] = 0.0  # some touched vertices with an exactly zero gradient: skipped as well
    say("scatter + Adam fused vs two calls, distinct vertices, C =", C)
    (pf, mf, vf), (pt, mt, vt) = _adam_pair(dv, g, xyz, y, steps=3)
    np.testing.assert_array_equal(pf, pt)
    np.testing.assert_array_equal(mf, mt)
    np.testing.assert_array_equal(vf, vt)
    untouched = np.ones(n ** 3, bool)
    untouched[verts[np.abs(y).sum(1) != 0]] = False
    assert np.array_equal(pf.reshape(n ** 3, C)[untouched], data.reshape(n ** 3, C)[untouched])
    assert not mf.reshape(n ** 3, C)[untouched].any()


@pytest.mark.parametrize("n,C,warp", [(40, 12, 0), (33, 1, 1), (160, 12, 0)])
def test_scatter_adam_matches_two_calls(dv, n, C, warp):
    # general points: the per-element sums differ only in the order of their terms
    rng = np.random.default_rng(50 + n + C)
    g = synth.normal_grid(rng, n, C, -2.0, 2.0) if warp else synth.normal_grid(rng, n, C)
    g.warp = warp
    wl = synth.config2(R=512)
    xyz = wl.samples.xyz if not warp else (wl.samples.xyz * 5.0).astype(np.float32)
    y = rng.standard_normal((xyz.shape[0], C)).astype(np.float32)
    say("scatter + Adam fused vs two calls, n =", n, "C =", C, "warp", warp, "S =", xyz.shape[0])
    (pf, mf, vf), (pt, mt, vt) = _adam_pair(dv, g, xyz, y, steps=2)
    close_after_adam(pf, pt, 2, 0.1, name="param")
    close(mf, mt, **GRAD, name="first moment")
    close(vf, vt, **GRAD, name="second moment")


def test_scatter_adam_against_oracle(dv):
    # one fused step against the oracle's Adam fed the oracle's scatter
    rng = np.random.default_rng(55)
    g = synth.normal_grid(rng, 48, 12)
    wl = synth.config2(R=1024, n=48)
    xyz = wl.samples.xyz
    y = rng.standard_normal((xyz.shape[0], 12)).astype(np.float32)
    say("fused scatter + Adam vs oracle, 48^3 x 12, S =", xyz.shape[0])
    dg = dgrid(dv, g)
    m, v = torch.zeros_like(dg.data), torch.zeros_like(dg.data)
    ws = dv.owner_bin(dg, T(xyz))
    dv.grid_scatter_adam(dg, T(xyz), T(y), ws, m, v, lr=0.1, step=1)
    torch.cuda.synchronize()
    grad = oracle.scatter(g, xyz, y.astype(np.float64))
    pe, me, ve = oracle.adam(g.data, grad, np.zeros(g.data.size), np.zeros(g.data.size), 0.1,
                             float(np.float32(0.9)), float(np.float32(0.99)), 1e-8, 1, skip_zero=True)
    close(m.cpu().numpy(), me, **GRAD, name="first moment")
    close_after_adam(dg.data.cpu().numpy(), pe, 1, 0.1, name="param after Adam")
