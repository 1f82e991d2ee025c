"""FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  It loads ``liborc.so`` built from ``dvgo_oracle.c`` by
``oracle.build_lib()`` with gcc (strict IEEE, no FMA contraction, OpenMP over rays)
and wraps it with numpy.  It shares nothing with the HIP library.

Parity status per function (pins live in ``tests/test_oracle_*.py``):

* gather / scatter: pinned (linear-field reproduction, vertex values, adjoint identity).
  Through the unbounded-scene contraction (Eq. 4, p = inf and 2): pinned (identity-field
  reproduction of an independent Eq. 4, its radius law and direction, continuity at the unit
  sphere, the limit radius, the plain lookup inside, the warped adjoint identity).
* distortion (Eq. 1) and its gradient: pinned (closed forms, the paper's O(N) rewrite,
  2-homogeneity, shift and reflection invariance, Euler identity, finite differences).
* render forward / backward: pinned (closed-form constant-density ray, invariants,
  the alpha_init identity, halting rule, finite differences of the oracle's forward).
* colour MLP: pinned against torch float64 Linear/ReLU/Sigmoid and autograd.  Its cheaper
  mode (matrix-product operands rounded to FP16 significands): pinned against a torch float64
  head with the same operands rounded by numpy's float16 conversion (straight-through values,
  rounded product-output gradients), and within a few 2^-11 of the exact head.
* Adam: pinned against torch.optim.Adam in float64; skip rule checked bitwise.
* proposal network: pinned against torch float64 with bfloat16-rounded operands;
  softmax/CE gradient closed form; resample closed forms (uniform and one-hot).
* total variation (Huber to the six axis neighbours, dense and sparse gradient modes):
  pinned (constant field, linear-ramp and saturated-spike closed forms, finite
  differences of the loss, 2-homogeneity of the quadratic regime, the sparse rule).
  The Huber threshold is unstated in the paper; it is an argument.
* sample producer (box clipping, candidate placement, nearest-vertex mask compaction; its
  integer decisions are taken in float32): pinned (axis-aligned closed forms, misses,
  float64 slab geometry and counts, the cap, brute-force mask selection).
* forward-facing NDC plane sampler: pinned (the paper's 2D - 1 points at s = 0.5, the
  central ray's plane depths, every point is the NDC projection of a world point on its ray
  (independent float64 projection), float64 brute force of the image-axis box test, rays that
  never reach the near plane, masks).
* occupancy mask update (alpha threshold, 27-neighbour dilation, deactivation only):
  pinned (numpy brute force, a single dense vertex, the alpha_init identity, idempotence
  and monotonicity).
* the alpha activation itself (the paper names it but never writes it): parity
  unpinned beyond its defining identity alpha(raw=0, delta_ref) = alpha_init.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dvgo_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
VP = C.c_void_p


def build_lib(force: bool = True) -> str:
    """Compile the oracle with gcc (strict floating point; no -ffast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcGrid(C.Structure):
    _fields_ = [("data", VP), ("n", C.c_int32 * 3), ("cs", C.c_int32), ("C", C.c_int32),
                ("bmin", C.c_float * 3), ("bmax", C.c_float * 3), ("warp", C.c_int32), ("wb", C.c_double)]


class OrcMLP(C.Structure):
    _fields_ = [("W1", VP), ("b1", VP), ("W2", VP), ("b2", VP), ("W3", VP), ("b3", VP),
                ("C", C.c_int32), ("F", C.c_int32), ("H", C.c_int32), ("half", C.c_int32)]


class OrcProp(C.Structure):
    _fields_ = [("L", C.c_int32), ("sizes", C.c_int32 * 8), ("W", VP * 8), ("b", VP * 8)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_lib(force=True)
        L = C.CDLL(_LIB)
        L.orc_act_shift.restype = C.c_double
        L.orc_act_shift.argtypes = [C.c_double, C.c_double]
        L.orc_loss_head.restype = C.c_double
        L.orc_prop_backward.restype = C.c_double
        L.orc_tv.restype = C.c_double
        _lib = L
    return _lib


# ------------------------------------------------------------------ helpers


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(VP)


class _Keep:
    """Holds numpy buffers alive while a ctypes struct points at them."""

    def __init__(self):
        self.bufs = []

    def __call__(self, a):
        self.bufs.append(a)
        return a


def grid_struct(grid, keep):
    data = keep(_c(grid.data, np.float32))
    g = OrcGrid()
    g.data = data.ctypes.data
    g.n[:] = [int(s) for s in data.shape[:3]]
    g.cs = int(data.shape[3])
    g.C = int(data.shape[3])
    g.bmin[:] = [float(v) for v in grid.xyz_min]
    g.bmax[:] = [float(v) for v in grid.xyz_max]
    g.warp = int(getattr(grid, "warp", 0))
    g.wb = float(getattr(grid, "warp_b", 1.0))
    return g


def threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(lib().orc_threads())


def set_threads(n: int) -> int:
    """Sets the oracle's OpenMP thread count; returns the previous one."""
    return int(lib().orc_set_threads(C.c_int32(n)))


def act_shift(alpha_init=1e-4, delta_ref=0.5) -> float:
    return float(lib().orc_act_shift(alpha_init, delta_ref))


# ---------------------------------------------------------------- functions


def gather(grid, xyz):
    keep = _Keep()
    g = grid_struct(grid, keep)
    xyz = keep(_c(xyz, np.float32))
    S = xyz.shape[0]
    out = np.zeros((S, g.C), np.float64)
    lib().orc_gather(C.byref(g), C.c_int64(S), _ptr(xyz), _ptr(out))
    return out


def scatter(grid, xyz, gv):
    keep = _Keep()
    g = grid_struct(grid, keep)
    xyz = keep(_c(xyz, np.float32))
    gv = keep(_c(gv, np.float64).reshape(xyz.shape[0], g.C))
    grad = np.zeros(grid.data.shape, np.float64)
    lib().orc_scatter(C.byref(g), C.c_int64(xyz.shape[0]), _ptr(xyz), _ptr(gv), _ptr(grad))
    return grad


def distortion(offs, w, m, l, form="definition"):
    offs = _c(offs, np.int32)
    w = _c(w, np.float64)
    m = _c(m, np.float32)
    l = _c(l, np.float32)
    R = offs.shape[0] - 1
    D = np.zeros(R, np.float64)
    fn = lib().orc_distortion if form == "definition" else lib().orc_distortion_prefix
    fn(C.c_int32(R), _ptr(offs), _ptr(w), _ptr(m), _ptr(l), _ptr(D))
    return D


def distortion_grad(offs, w, m, l, gD=None, form="definition"):
    offs = _c(offs, np.int32)
    w = _c(w, np.float64)
    m = _c(m, np.float32)
    l = _c(l, np.float32)
    R = offs.shape[0] - 1
    gw = np.zeros(w.shape[0], np.float64)
    if form == "definition":
        gD = _c(np.ones(R) if gD is None else gD, np.float64)
        lib().orc_distortion_grad(C.c_int32(R), _ptr(offs), _ptr(w), _ptr(m), _ptr(l), _ptr(gD), _ptr(gw))
    else:
        lib().orc_distortion_prefix_grad(C.c_int32(R), _ptr(offs), _ptr(w), _ptr(m), _ptr(l), _ptr(gw))
        if gD is not None:
            gw *= np.repeat(np.asarray(gD, np.float64), np.diff(offs))
    return gw


def _render_args(samples, density, color, srgb, keep):
    offs = keep(_c(samples.ray_offsets, np.int32))
    xyz = keep(_c(samples.xyz, np.float32))
    dl = keep(_c(samples.delta, np.float32))
    sm = keep(_c(samples.s_mid, np.float32))
    sl = keep(_c(samples.s_len, np.float32))
    gd = grid_struct(density, keep)
    gc = grid_struct(color, keep) if color is not None else None
    sr = keep(_c(srgb, np.float64).reshape(-1, 3)) if srgb is not None else None
    return offs, xyz, dl, sm, sl, gd, gc, sr


def render_forward(samples, density, color=None, srgb=None, shift=None, halt_T=0.0, bg=(1.0, 1.0, 1.0),
                   want_w=False):
    """Returns dict(rgb[R,3], T[R], D[R], and w[S], alpha[S] when want_w)."""
    keep = _Keep()
    offs, xyz, dl, sm, sl, gd, gc, sr = _render_args(samples, density, color, srgb, keep)
    R = offs.shape[0] - 1
    S = int(offs[-1])
    shift = act_shift() if shift is None else shift
    bgv = keep(_c(bg, np.float64))
    rgb = np.zeros((R, 3))
    T = np.zeros(R)
    D = np.zeros(R)
    w = np.zeros(S) if want_w else None
    al = np.zeros(S) if want_w else None
    lib().orc_render_forward(C.c_int32(R), _ptr(offs), _ptr(xyz), _ptr(dl), _ptr(sm), _ptr(sl), C.byref(gd),
                             C.byref(gc) if gc is not None else None, _ptr(sr), C.c_double(shift),
                             C.c_double(halt_T), _ptr(bgv), _ptr(rgb), _ptr(T), _ptr(D), _ptr(w), _ptr(al))
    out = dict(rgb=rgb, T=T, D=D)
    if want_w:
        out["w"] = w
        out["alpha"] = al
    return out


def render_backward(samples, density, G_C, G_D=None, G_T=None, color=None, srgb=None, shift=None, halt_T=0.0,
                    bg=(1.0, 1.0, 1.0)):
    """Returns dict(grad_density (grid shape), grad_color (grid shape) or grad_srgb [S,3])."""
    keep = _Keep()
    offs, xyz, dl, sm, sl, gd, gc, sr = _render_args(samples, density, color, srgb, keep)
    R = offs.shape[0] - 1
    S = int(offs[-1])
    shift = act_shift() if shift is None else shift
    bgv = keep(_c(bg, np.float64))
    GC = keep(_c(G_C, np.float64).reshape(R, 3))
    GD = keep(_c(G_D, np.float64)) if G_D is not None else None
    GT = keep(_c(G_T, np.float64)) if G_T is not None else None
    gdens = np.zeros(density.data.shape, np.float64)
    gcol = np.zeros(color.data.shape, np.float64) if color is not None else None
    gs = np.zeros((S, 3)) if srgb is not None else None
    lib().orc_render_backward(C.c_int32(R), _ptr(offs), _ptr(xyz), _ptr(dl), _ptr(sm), _ptr(sl), C.byref(gd),
                              C.byref(gc) if gc is not None else None, _ptr(sr), C.c_double(shift),
                              C.c_double(halt_T), _ptr(bgv), _ptr(GC), _ptr(GD), _ptr(GT), _ptr(gdens),
                              _ptr(gcol), _ptr(gs))
    out = dict(grad_density=gdens)
    if color is not None:
        out["grad_color"] = gcol
    if srgb is not None:
        out["grad_srgb"] = gs
    return out


def alpha(xyz, delta, density, shift=None):
    keep = _Keep()
    gd = grid_struct(density, keep)
    xyz = keep(_c(xyz, np.float32))
    dl = keep(_c(delta, np.float32))
    S = xyz.shape[0]
    out = np.zeros(S)
    shift = act_shift() if shift is None else shift
    lib().orc_alpha(C.c_int64(S), _ptr(xyz), _ptr(dl), C.byref(gd), C.c_double(shift), _ptr(out))
    return out


def loss_head(rgb, target, D, lam):
    rgb = _c(rgb, np.float64)
    target = _c(target, np.float32)
    R = rgb.shape[0]
    Dv = _c(D, np.float64) if D is not None else None
    GC = np.zeros((R, 3))
    GD = np.zeros(R)
    L = lib().orc_loss_head(C.c_int32(R), _ptr(rgb), _ptr(target), _ptr(Dv), C.c_double(lam), _ptr(GC), _ptr(GD))
    return float(L), GC, GD


def _mlp_struct(mlp, keep, C_feat, F, half=False):
    P = OrcMLP()
    P.half = 1 if half else 0
    W1, W2, W3 = [keep(_c(w, np.float32)) for w in mlp.W]
    b1, b2, b3 = [keep(_c(b, np.float32)) for b in mlp.b]
    P.W1, P.b1, P.W2, P.b2, P.W3, P.b3 = [a.ctypes.data for a in (W1, b1, W2, b2, W3, b3)]
    P.C, P.F, P.H = C_feat, F, W2.shape[0]
    return P


def mlp_forward(mlp, offs, dirs, feat, F=4, half=False):
    """Colour head forward (orc_mlp_forward); half: matrix-product operands rounded to FP16
    significands, as the cheaper colour head computes them."""
    keep = _Keep()
    feat = keep(_c(feat, np.float64))
    P = _mlp_struct(mlp, keep, feat.shape[1], F, half)
    offs = keep(_c(offs, np.int32))
    dirs = keep(_c(dirs, np.float32))
    R = offs.shape[0] - 1
    rgb = np.zeros((feat.shape[0], 3))
    lib().orc_mlp_forward(C.byref(P), C.c_int32(R), _ptr(offs), _ptr(dirs), _ptr(feat), _ptr(rgb))
    return rgb


def mlp_kink_slack(mlp, offs, dirs, feat, grad_rgb, thr=1e-5, F=4, half=False):
    """Per-element slack of the colour-head gradients at ReLU kinks (see orc_mlp_kink_slack).
    Returns (slack_feat [S,C], [W1, W2, W3] slacks, [b1, b2, b3] slacks)."""
    keep = _Keep()
    feat = keep(_c(feat, np.float64))
    P = _mlp_struct(mlp, keep, feat.shape[1], F, half)
    offs = keep(_c(offs, np.int32))
    dirs = keep(_c(dirs, np.float32))
    gr = keep(_c(grad_rgb, np.float64))
    sizes = [mlp.W[0].size, mlp.b[0].size, mlp.W[1].size, mlp.b[1].size, mlp.W[2].size, mlp.b[2].size]
    sf = np.zeros_like(feat)
    sp = np.zeros(sum(sizes))
    lib().orc_mlp_kink_slack(C.byref(P), C.c_int32(offs.shape[0] - 1), _ptr(offs), _ptr(dirs), _ptr(feat), _ptr(gr),
                             C.c_double(thr), _ptr(sf), _ptr(sp))
    parts = np.split(sp, np.cumsum(sizes)[:-1])
    W = [parts[0].reshape(mlp.W[0].shape), parts[2].reshape(mlp.W[1].shape), parts[4].reshape(mlp.W[2].shape)]
    b = [parts[1], parts[3], parts[5]]
    return sf, W, b


def mlp_backward(mlp, offs, dirs, feat, grad_rgb, F=4, half=False):
    """Returns (grad_feat [S,C], [gW1, gW2, gW3], [gb1, gb2, gb3]); half as in mlp_forward."""
    keep = _Keep()
    feat = keep(_c(feat, np.float64))
    P = _mlp_struct(mlp, keep, feat.shape[1], F, half)
    offs = keep(_c(offs, np.int32))
    dirs = keep(_c(dirs, np.float32))
    gr = keep(_c(grad_rgb, np.float64))
    R = offs.shape[0] - 1
    gf = np.zeros_like(feat)
    gW = [np.zeros(w.shape) for w in mlp.W]
    gb = [np.zeros(b.shape) for b in mlp.b]
    lib().orc_mlp_backward(C.byref(P), C.c_int32(R), _ptr(offs), _ptr(dirs), _ptr(feat), _ptr(gr), _ptr(gf),
                           _ptr(gW[0]), _ptr(gb[0]), _ptr(gW[1]), _ptr(gb[1]), _ptr(gW[2]), _ptr(gb[2]))
    return gf, gW, gb


def adam(p, g, m, v, lr, beta1, beta2, eps, step, skip_zero=True):
    """In-place FP64 Adam on copies; returns (p, m, v)."""
    p = _c(p, np.float64).copy()
    m = _c(m, np.float64).copy()
    v = _c(v, np.float64).copy()
    g = _c(g, np.float64)
    lib().orc_adam(C.c_int64(p.size), _ptr(p), _ptr(g), _ptr(m), _ptr(v), C.c_double(lr), C.c_double(beta1),
                   C.c_double(beta2), C.c_double(eps), C.c_int32(step), C.c_int32(1 if skip_zero else 0))
    return p, m, v


def bf16_round(x):
    x = _c(x, np.float64)
    out = np.empty_like(x)
    lib().orc_bf16_round(C.c_int64(x.size), _ptr(x), _ptr(out))
    return out


def _prop_struct(pw, keep):
    P = OrcProp()
    P.L = len(pw.W)
    sizes = [pw.W[0].shape[1]] + [w.shape[0] for w in pw.W]
    for i, s in enumerate(sizes):
        P.sizes[i] = s
    for i, (w, b) in enumerate(zip(pw.W, pw.b)):
        P.W[i] = keep(_c(w, np.float32)).ctypes.data
        P.b[i] = keep(_c(b, np.float32)).ctypes.data
    return P, sizes


def prop_forward(pw, x):
    """Returns (logits [R,B], prob [R,B], entropy [R])."""
    keep = _Keep()
    P, sizes = _prop_struct(pw, keep)
    x = keep(_c(x, np.float64))
    R = x.shape[0]
    B = sizes[-1]
    lg = np.zeros((R, B))
    pr = np.zeros((R, B))
    H = np.zeros(R)
    lib().orc_prop_forward(C.byref(P), C.c_int32(R), _ptr(x), _ptr(lg), _ptr(pr), _ptr(H))
    return lg, pr, H


def prop_backward(pw, x, target):
    """Returns (loss, [gW], [gb])."""
    keep = _Keep()
    P, sizes = _prop_struct(pw, keep)
    x = keep(_c(x, np.float64))
    tg = keep(_c(target, np.float64))
    R = x.shape[0]
    gW = [np.zeros(w.shape) for w in pw.W]
    gb = [np.zeros(b.shape) for b in pw.b]
    gWp = (VP * len(gW))(*[a.ctypes.data for a in gW])
    gbp = (VP * len(gb))(*[a.ctypes.data for a in gb])
    loss = lib().orc_prop_backward(C.byref(P), C.c_int32(R), _ptr(x), _ptr(tg), gWp, gbp)
    return float(loss), gW, gb


def histogram(offs, w, s_mid, B=64, min_mass=1e-4):
    offs = _c(offs, np.int32)
    w = _c(w, np.float64)
    sm = _c(s_mid, np.float32)
    R = offs.shape[0] - 1
    h = np.zeros((R, B))
    lib().orc_histogram(C.c_int32(R), _ptr(offs), _ptr(w), _ptr(sm), C.c_int32(B), C.c_double(min_mass), _ptr(h))
    return h


def resample(prob, n, rays, voxel):
    """Returns dict(xyz [R*n,3], delta, s_mid, s_len) in float64."""
    prob = _c(prob, np.float64)
    R, B = prob.shape
    o = _c(rays.origins, np.float32)
    d = _c(rays.dirs, np.float32)
    tn = _c(rays.t_near, np.float32)
    tf = _c(rays.t_far, np.float32)
    xyz = np.zeros((R * n, 3))
    dl = np.zeros(R * n)
    sm = np.zeros(R * n)
    sl = np.zeros(R * n)
    lib().orc_resample(C.c_int32(R), C.c_int32(B), _ptr(prob), C.c_int32(n), _ptr(o), _ptr(d), _ptr(tn), _ptr(tf),
                       C.c_double(voxel), _ptr(xyz), _ptr(dl), _ptr(sm), _ptr(sl))
    return dict(xyz=xyz, delta=dl, s_mid=sm, s_len=sl)


def proposal_coarse(rays, density, voxel, B=64, eps=1e-4, shift=None):
    """Returns (w_coarse [R,B], feat [R,B]) of the proposal's coarse pass."""
    keep = _Keep()
    gd = grid_struct(density, keep)
    o, d = keep(_c(rays.origins, np.float32)), keep(_c(rays.dirs, np.float32))
    tn, tf = keep(_c(rays.t_near, np.float32)), keep(_c(rays.t_far, np.float32))
    R = o.shape[0]
    w = np.zeros((R, B))
    f = np.zeros((R, B))
    shift = act_shift() if shift is None else shift
    lib().orc_proposal_coarse(C.c_int32(R), _ptr(o), _ptr(d), _ptr(tn), _ptr(tf), C.byref(gd), C.c_double(shift),
                              C.c_double(voxel), C.c_int32(B), C.c_double(eps), _ptr(w), _ptr(f))
    return w, f


def resample_batch(prob, H, tau, n_fine, n_plain, rays, voxel):
    """Returns dict(ray_offsets, xyz, delta, s_mid, s_len) of the proposal's ragged fine batch."""
    prob = _c(prob, np.float64)
    Hh = _c(H, np.float64)
    R, B = prob.shape
    o, d = _c(rays.origins, np.float32), _c(rays.dirs, np.float32)
    tn, tf = _c(rays.t_near, np.float32), _c(rays.t_far, np.float32)
    cap = R * max(n_fine, n_plain)
    offs = np.zeros(R + 1, np.int32)
    xyz, dl, sm, sl = np.zeros((cap, 3)), np.zeros(cap), np.zeros(cap), np.zeros(cap)
    lib().orc_resample_batch(C.c_int32(R), C.c_int32(B), _ptr(prob), _ptr(Hh), C.c_double(tau), C.c_int32(n_fine),
                             C.c_int32(n_plain), _ptr(o), _ptr(d), _ptr(tn), _ptr(tf), C.c_double(voxel), _ptr(offs),
                             _ptr(xyz), _ptr(dl), _ptr(sm), _ptr(sl))
    S = int(offs[-1])
    return dict(ray_offsets=offs, xyz=xyz[:S], delta=dl[:S], s_mid=sm[:S], s_len=sl[:S])


def resample_guarded(prob, w_coarse, H, tau, n_base, n_extra, w_min, rays, voxel, want_samples=True):
    """Guarded resampling (orc_resample_guarded) from the float32 prob, w_coarse [R,64] and H [R]:
    returns dict(ray_offsets, counts [R,64], and xyz, delta, s_mid, s_len when want_samples)."""
    keep = _Keep()
    pr = keep(_c(prob, np.float32))
    wc = keep(_c(w_coarse, np.float32))
    Hh = keep(_c(H, np.float32))
    R, B = pr.shape
    o = keep(_c(rays.origins, np.float32))
    d = keep(_c(rays.dirs, np.float32))
    tn = keep(_c(rays.t_near, np.float32))
    tf = keep(_c(rays.t_far, np.float32))
    offs = np.zeros(R + 1, np.int32)
    counts = np.zeros((R, B), np.int32)
    lib().orc_resample_guarded(C.c_int32(R), C.c_int32(B), _ptr(pr), _ptr(wc), _ptr(Hh), C.c_float(tau),
                               C.c_int32(n_base), C.c_int32(n_extra), C.c_float(w_min), _ptr(o), _ptr(d), _ptr(tn),
                               _ptr(tf), C.c_double(voxel), _ptr(offs), _ptr(counts), None, None, None, None)
    out = dict(ray_offsets=offs, counts=counts)
    if want_samples:
        S = int(offs[-1])
        xyz, dl, sm, sl = np.zeros((max(S, 1), 3)), np.zeros(max(S, 1)), np.zeros(max(S, 1)), np.zeros(max(S, 1))
        lib().orc_resample_guarded(C.c_int32(R), C.c_int32(B), _ptr(pr), _ptr(wc), _ptr(Hh), C.c_float(tau),
                                   C.c_int32(n_base), C.c_int32(n_extra), C.c_float(w_min), _ptr(o), _ptr(d),
                                   _ptr(tn), _ptr(tf), C.c_double(voxel), _ptr(offs), None, _ptr(xyz), _ptr(dl),
                                   _ptr(sm), _ptr(sl))
        out.update(xyz=xyz[:S], delta=dl[:S], s_mid=sm[:S], s_len=sl[:S])
    return out


def softmax_entropy(logits):
    lg = _c(logits, np.float64)
    R, B = lg.shape
    p = np.zeros((R, B))
    H = np.zeros(R)
    lib().orc_softmax_entropy(C.c_int32(R), C.c_int32(B), _ptr(lg), _ptr(p), _ptr(H))
    return p, H


def tv(grid, weight, delta, dense=True, grad=None, want_mag=False):
    """Total-variation loss and gradient of a grid (orc_tv): returns (L, grad_in + dL/dv) where
    the gradient is added at every vertex (dense) or only where some channel of grad_in is
    non-zero.  grid: synth.Grid (data [nx,ny,nz,C] float32); grad: float64 array of the
    same shape, or None (zeros).  want_mag: also return the per-element magnitude the
    gradient sum is conditioned on."""
    keep = _Keep()
    g = grid_struct(grid, keep)
    out = np.zeros(grid.data.shape, np.float64) if grad is None else np.array(grad, np.float64, copy=True)
    out = np.ascontiguousarray(out)
    mag = np.zeros(grid.data.shape, np.float64) if want_mag else None
    L = lib().orc_tv(C.byref(g), C.c_double(weight), C.c_double(delta), C.c_int32(1 if dense else 0), _ptr(out),
                     _ptr(mag) if want_mag else None)
    return (float(L), out, mag) if want_mag else (float(L), out)


def occupancy_update(density, act_shift, delta, alpha_thr, mask=None):
    """Occupancy mask update (orc_occupancy_update): returns the new uint8 mask [nx,ny,nz].
    density: synth.Grid with one channel; mask: the current mask (None = all active)."""
    keep = _Keep()
    g = grid_struct(density, keep)
    out = np.ones(density.data.shape[:3], np.uint8) if mask is None else np.array(mask, np.uint8, copy=True)
    out = np.ascontiguousarray(out)
    lib().orc_occupancy_update(C.byref(g), C.c_double(act_shift), C.c_double(delta), C.c_double(alpha_thr),
                               _ptr(out))
    return out


def sample_rays(origins, dirs, bmin, bmax, near, step, voxel, max_per_ray, mask=None):
    """Parsimonious box sampling with occupancy compaction (orc_sample_rays).  Returns a dict
    with ray_offsets [R+1] int32, t_near/t_far [R], xyz [S,3], delta, s_mid, s_len [S]
    (float32: these are the float32 decisions and values the sampler defines)."""
    o = _c(origins, np.float32).reshape(-1, 3)
    d = _c(dirs, np.float32).reshape(-1, 3)
    R = o.shape[0]
    lo = _c(bmin, np.float32).reshape(3)
    hi = _c(bmax, np.float32).reshape(3)
    m = None if mask is None else _c(mask, np.uint8)
    shape = np.zeros(3, np.int32) if m is None else np.array(m.shape, np.int32)
    offs = np.zeros(R + 1, np.int32)
    tn = np.zeros(R, np.float32)
    tf = np.zeros(R, np.float32)
    L = lib()
    L.orc_sample_rays.restype = C.c_int64
    args = (C.c_int32(R), _ptr(o), _ptr(d), _ptr(lo), _ptr(hi), C.c_float(near), C.c_float(step), C.c_float(voxel),
            C.c_int32(max_per_ray), _ptr(m), _ptr(shape), _ptr(offs), _ptr(tn), _ptr(tf))
    S = int(L.orc_sample_rays(*args, None, None, None, None))
    xyz = np.zeros((S, 3), np.float32)
    dl, sm, sl = (np.zeros(S, np.float32) for _ in range(3))
    L.orc_sample_rays(*args, _ptr(xyz), _ptr(dl), _ptr(sm), _ptr(sl))
    return dict(ray_offsets=offs, t_near=tn, t_far=tf, xyz=xyz, delta=dl, s_mid=sm, s_len=sl)


def sample_ndc(origins, dirs, bmin, bmax, fx, fy, near, planes, step, max_per_ray=4096, mask=None):
    """Forward-facing NDC plane sampling (orc_sample_ndc).  Returns a dict with ray_offsets
    [R+1] int32 and the float32 samples xyz [S,3] (NDC points), delta, s_mid, s_len."""
    o = _c(origins, np.float32).reshape(-1, 3)
    d = _c(dirs, np.float32).reshape(-1, 3)
    R = o.shape[0]
    lo = _c(bmin, np.float32).reshape(3)
    hi = _c(bmax, np.float32).reshape(3)
    m = None if mask is None else _c(mask, np.uint8)
    shape = np.zeros(3, np.int32) if m is None else np.array(m.shape, np.int32)
    offs = np.zeros(R + 1, np.int32)
    L = lib()
    L.orc_sample_ndc.restype = C.c_int64
    args = (C.c_int32(R), _ptr(o), _ptr(d), _ptr(lo), _ptr(hi), C.c_float(fx), C.c_float(fy), C.c_float(near),
            C.c_int32(planes), C.c_float(step), C.c_int32(max_per_ray), _ptr(m), _ptr(shape), _ptr(offs))
    S = int(L.orc_sample_ndc(*args, None, None, None, None))
    xyz = np.zeros((S, 3), np.float32)
    dl, sm, sl = (np.zeros(S, np.float32) for _ in range(3))
    L.orc_sample_ndc(*args, _ptr(xyz), _ptr(dl), _ptr(sm), _ptr(sl))
    return dict(ray_offsets=offs, xyz=xyz, delta=dl, s_mid=sm, s_len=sl)


def r16_round(x):
    """Round to 11 significant bits, to nearest even (the FP16 operands of the cheaper head)."""
    a = _c(x, np.float64)
    out = np.zeros_like(a)
    lib().orc_r16_round(C.c_int64(a.size), _ptr(a), _ptr(out))
    return out


def mlp_magnitudes(mlp, offs, dirs, feat, grad_rgb, F=4, half=False):
    """Conditioning magnitudes of the colour head's outputs (orc_mlp_magnitudes): returns
    (mag_rgb [S,3], mag_feat [S,C], [W1, W2, W3] magnitudes, [b1, b2, b3] magnitudes)."""
    keep = _Keep()
    feat = keep(_c(feat, np.float64))
    P = _mlp_struct(mlp, keep, feat.shape[1], F, half)
    offs = keep(_c(offs, np.int32))
    dirs = keep(_c(dirs, np.float32))
    gr = keep(_c(grad_rgb, np.float64))
    sizes = [mlp.W[0].size, mlp.b[0].size, mlp.W[1].size, mlp.b[1].size, mlp.W[2].size, mlp.b[2].size]
    mr = np.zeros((feat.shape[0], 3))
    mf = np.zeros_like(feat)
    mp = np.zeros(sum(sizes))
    lib().orc_mlp_magnitudes(C.byref(P), C.c_int32(offs.shape[0] - 1), _ptr(offs), _ptr(dirs), _ptr(feat), _ptr(gr),
                             _ptr(mr), _ptr(mf), _ptr(mp))
    parts = np.split(mp, np.cumsum(sizes)[:-1])
    W = [parts[0].reshape(mlp.W[0].shape), parts[2].reshape(mlp.W[1].shape), parts[4].reshape(mlp.W[2].shape)]
    return mr, mf, W, [parts[1], parts[3], parts[5]]
