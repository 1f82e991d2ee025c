"""Seeded synthetic scenes, rays and ragged sample batches (numpy only).

The paper's workloads are real captures (Synthetic-NeRF, Tanks&Temples, LLFF,
mip-NeRF 360, section 5).  None of them is available here, so Gaussian-blob scenes
with the paper's shapes stand in for them:

* dense grids of 160^3 and 320^3 vertices (section 5.1, section 5.4),
* 8192 rays with 256 points each per iteration (section 1),
* the unbounded-scene parameterisation of Eq. 4 with p = inf for the ragged case.

Every array is produced in float32 (or int32 for offsets) from
``numpy.random.Generator(PCG64(1000 * config + stream))`` so that the HIP path and
the FP64 oracle read bit-identical inputs.  Streams: 0 density, 1 colour/features,
2 MLP weights, 3 rays, 4 live mask and ray lengths, 5 targets, 6 held-out rays,
7 proposal weights.

Geometry used only to *produce* inputs lives here too: the ray/box slab test and
uniform placement of samples between the clipped near and far distances, and, for
the unbounded case, disparity-linear placement followed by the Eq. 4 contraction.
These produce the ragged batch the training step consumes; the step itself never
computes them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

F32 = np.float32


def _rng(cfg: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * cfg + stream))


# --------------------------------------------------------------------------- data


@dataclass
class Grid:
    """Dense vertex grid, channel-last: ``data[nx, ny, nz, C]`` (float32, C-contiguous).

    Vertices sit on the box corners: vertex i along an axis is at
    ``xyz_min + i * (xyz_max - xyz_min) / (n - 1)``.  ``warp`` says how points address
    the box: 0 directly, 1 / 2 through the unbounded-scene contraction (Eq. 4) with
    p = inf / 2 and parameter ``warp_b``.
    """
    data: np.ndarray
    xyz_min: np.ndarray
    xyz_max: np.ndarray
    warp: int = 0
    warp_b: float = 1.0

    @property
    def shape(self):
        return self.data.shape[:3]

    @property
    def channels(self):
        return self.data.shape[3]

    def voxel_size(self) -> float:
        return float((self.xyz_max[0] - self.xyz_min[0]) / (self.data.shape[0] - 1))


@dataclass
class Rays:
    origins: np.ndarray   # [R,3] f32
    dirs: np.ndarray      # [R,3] f32, unit length
    t_near: np.ndarray    # [R] f32 (0 for rays that miss)
    t_far: np.ndarray     # [R] f32
    hit: np.ndarray       # [R] bool


@dataclass
class Samples:
    """Flattened ragged batch: ray r owns samples ``ray_offsets[r]:ray_offsets[r+1]``."""
    ray_offsets: np.ndarray  # [R+1] int32
    xyz: np.ndarray          # [S,3] f32
    delta: np.ndarray        # [S] f32, interval length in voxel units
    s_mid: np.ndarray        # [S] f32, normalised midpoint, non-decreasing within a ray
    s_len: np.ndarray        # [S] f32, normalised interval length

    @property
    def n_rays(self) -> int:
        return int(self.ray_offsets.shape[0] - 1)

    @property
    def n_samples(self) -> int:
        return int(self.ray_offsets[-1])

    def lengths(self) -> np.ndarray:
        return np.diff(self.ray_offsets)


@dataclass
class MLPWeights:
    """Fully connected layers, ``W[l]`` is ``[out, in]`` like torch's Linear."""
    W: list
    b: list

    def n_params(self) -> int:
        return int(sum(w.size for w in self.W) + sum(b.size for b in self.b))


@dataclass
class Workload:
    name: str
    density: Grid
    color: Optional[Grid]            # colour grid (C=3) for the grid-colour mode
    feat: Optional[Grid]             # feature grid (C=12) for the MLP-colour mode
    mlp: Optional[MLPWeights]
    rays: Rays
    samples: Samples
    target: np.ndarray               # [R,3] f32
    bg: tuple = (1.0, 1.0, 1.0)
    dist_weight: float = 0.01        # section 5.3 / 5.4: distortion loss weight 1e-2
    alpha_init: float = 1e-4         # section 5.4
    delta_ref: float = 0.5           # section 5.4: 0.5-voxel step
    halt_T: float = 0.0              # 0 disables halting (parity runs); the paper uses 1e-3
    extra: dict = field(default_factory=dict)


# ----------------------------------------------------------------------- grids


def _axis(n, lo, hi):
    return lo + (hi - lo) * np.arange(n, dtype=np.float64) / (n - 1)


def _shape3(n):
    return (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)


def blob_density(rng, n, xyz_min=-1.0, xyz_max=1.0, n_blobs=8, center_box=0.6, return_blobs=False):
    """Density logits N(0,1) + sum of Gaussian blobs (amplitude U[6,14], sigma U[0.05,0.2]).
    n: vertices per axis, or a 3-tuple.  With return_blobs, also returns the blob term alone."""
    lo = np.full(3, xyz_min, np.float64)
    hi = np.full(3, xyz_max, np.float64)
    shp = _shape3(n)
    base = rng.standard_normal(shp, dtype=np.float32)
    mu = rng.uniform(-center_box, center_box, size=(n_blobs, 3))
    sd = rng.uniform(0.05, 0.2, size=n_blobs)
    amp = rng.uniform(6.0, 14.0, size=n_blobs)
    axes = [_axis(shp[a], lo[a], hi[a]) for a in range(3)]
    acc = np.zeros(shp, np.float32)
    for b in range(n_blobs):
        g = [np.exp(-(axes[a] - mu[b, a]) ** 2 / (2 * sd[b] ** 2)).astype(F32) for a in range(3)]
        acc += F32(amp[b]) * (g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :])
    data = (base + acc).astype(F32)[..., None]
    g = Grid(np.ascontiguousarray(data), lo.astype(F32), hi.astype(F32))
    return (g, acc) if return_blobs else g


def normal_grid(rng, n, C, xyz_min=-1.0, xyz_max=1.0) -> Grid:
    data = rng.standard_normal(_shape3(n) + (C,), dtype=np.float32)
    return Grid(data, np.full(3, xyz_min, F32), np.full(3, xyz_max, F32))


def uniform_grid(rng, n, C, xyz_min=-1.0, xyz_max=1.0) -> Grid:
    data = rng.random((n, n, n, C), dtype=np.float32)
    return Grid(data, np.full(3, xyz_min, F32), np.full(3, xyz_max, F32))


# ------------------------------------------------------------------------ rays


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _sphere(rng, n):
    return _unit(rng.standard_normal((n, 3)))


def slab_interval(o, d, bmin, bmax):
    """Ray/box clip by the slab method (float64).  Returns t_near, t_far, hit."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(np.abs(d) > 1e-12, 1.0 / d, 1e12)
        t0 = (bmin[None] - o) * inv
        t1 = (bmax[None] - o) * inv
    tmin = np.minimum(t0, t1).max(axis=1)
    tmax = np.maximum(t0, t1).min(axis=1)
    tn = np.maximum(tmin, 0.0)
    hit = tmax > tn + 1e-9
    return np.where(hit, tn, 0.0), np.where(hit, tmax, 0.0), hit


def _finish_rays(o, d, bmin, bmax) -> Rays:
    d = _unit(d)
    tn, tf, hit = slab_interval(o, d, np.asarray(bmin, np.float64), np.asarray(bmax, np.float64))
    return Rays(o.astype(F32), d.astype(F32), tn.astype(F32), tf.astype(F32), hit)


def rays_at_box(rng, R, radius=4.0, bmin=(-1, -1, -1), bmax=(1, 1, 1)) -> Rays:
    """Origins uniform on a sphere, aimed at points drawn uniformly inside the box."""
    o = radius * _sphere(rng, R)
    tgt = rng.uniform(np.asarray(bmin, float), np.asarray(bmax, float), size=(R, 3))
    return _finish_rays(o, tgt - o, bmin, bmax)


def pinhole_rays(rng, R, n_cams=100, radius=4.0, H=800, W=800, fov_deg=40.0,
                 bmin=(-1, -1, -1), bmax=(1, 1, 1)) -> Rays:
    """Random pixels of pinhole cameras on a sphere, each looking at the origin."""
    cams = radius * _sphere(rng, n_cams)
    f = 0.5 * W / np.tan(np.deg2rad(fov_deg) / 2)
    cid = rng.integers(0, n_cams, size=R)
    px = rng.integers(0, W, size=R) + 0.5
    py = rng.integers(0, H, size=R) + 0.5
    fwd = _unit(-cams)
    up = np.tile(np.array([0.0, 0.0, 1.0]), (n_cams, 1))
    near_pole = np.abs(fwd[:, 2]) > 0.999
    up[near_pole] = np.array([0.0, 1.0, 0.0])
    right = _unit(np.cross(fwd, up))
    down = np.cross(fwd, right)
    dc = np.stack([(px - 0.5 * W) / f, (py - 0.5 * H) / f, np.ones(R)], axis=1)
    d = dc[:, :1] * right[cid] + dc[:, 1:2] * down[cid] + dc[:, 2:] * fwd[cid]
    return _finish_rays(cams[cid], d, bmin, bmax)


def forward_facing_rays(rng, R, n_cams=20, W=1008, H=756, focal=815.0, spread=0.15, tilt_deg=3.0):
    """Random pixels of n_cams pinhole cameras of a forward-facing capture, in the reference
    camera's frame (looking down -z): centres jittered in the z = 0 plane by +-spread, small
    random tilts.  Returns float32 origins and unit directions."""
    cams = np.zeros((n_cams, 3))
    cams[:, :2] = rng.uniform(-spread, spread, (n_cams, 2))
    ang = np.deg2rad(rng.uniform(-tilt_deg, tilt_deg, (n_cams, 2)))
    cid = rng.integers(0, n_cams, size=R)
    px = rng.integers(0, W, size=R) + 0.5
    py = rng.integers(0, H, size=R) + 0.5
    dc = np.stack([(px - 0.5 * W) / focal, -(py - 0.5 * H) / focal, -np.ones(R)], axis=1)
    ax, ay = ang[cid, 0], ang[cid, 1]
    # tilt about x then y
    y1 = dc[:, 1] * np.cos(ax) - dc[:, 2] * np.sin(ax)
    z1 = dc[:, 1] * np.sin(ax) + dc[:, 2] * np.cos(ax)
    x2 = dc[:, 0] * np.cos(ay) + z1 * np.sin(ay)
    z2 = -dc[:, 0] * np.sin(ay) + z1 * np.cos(ay)
    d = _unit(np.stack([x2, y1, z2], axis=1))
    return cams[cid].astype(F32), d.astype(F32)


def rays_into_ball(rng, R, radius=0.9):
    """Origins on a small sphere inside the unit ball, aimed at uniform points of the ball."""
    o = radius * _sphere(rng, R)
    r = rng.random(R) ** (1.0 / 3.0)
    tgt = r[:, None] * _sphere(rng, R)
    d = _unit(tgt - o)
    return o, d


# --------------------------------------------------------------------- samples


def _flatten(live, *cols):
    counts = live.sum(axis=1)
    offs = np.zeros(live.shape[0] + 1, np.int64)
    np.cumsum(counts, out=offs[1:])
    out = [c[live] for c in cols]
    return offs.astype(np.int32), out


def uniform_samples(rays: Rays, n_per_ray: int, voxel: float, live_frac=None, rng=None) -> Samples:
    """``n_per_ray`` midpoint samples on [t_near, t_far]; optional per-ray Bernoulli live mask.

    s is linear in t per ray: sample k has s_mid = (k + 1/2)/N and s_len = 1/N.  The
    alpha interval ``delta`` is the t-step divided by the voxel size.
    """
    R = rays.origins.shape[0]
    N = n_per_ray
    k = np.arange(N, dtype=np.float64)
    tn = rays.t_near.astype(np.float64)[:, None]
    tf = rays.t_far.astype(np.float64)[:, None]
    step = (tf - tn) / N
    t = tn + (k[None] + 0.5) * step
    live = np.repeat(rays.hit[:, None], N, axis=1)
    if live_frac is not None:
        live &= rng.random((R, N)) < live_frac[:, None]
    xyz = rays.origins.astype(np.float64)[:, None, :] + t[..., None] * rays.dirs.astype(np.float64)[:, None, :]
    delta = np.broadcast_to(step / voxel, (R, N))
    smid = np.broadcast_to((k[None] + 0.5) / N, (R, N))
    slen = np.broadcast_to(np.full((1, 1), 1.0 / N), (R, N))
    offs, (xyz, delta, smid, slen) = _flatten(live, xyz, delta, smid, slen)
    return Samples(offs, xyz.astype(F32).reshape(-1, 3), delta.astype(F32), smid.astype(F32), slen.astype(F32))


def _contract_inf(x, b=1.0):
    """Eq. 4 with p = inf: identity inside the unit cube, squashes the rest into [-1-b, 1+b]."""
    nrm = np.abs(x).max(axis=-1, keepdims=True)
    scale = np.where(nrm <= 1.0, 1.0, (1.0 + b - b / np.maximum(nrm, 1.0)) / np.maximum(nrm, 1e-30))
    return x * scale


def disparity_samples(rng, o, d, lengths, voxel, t_near=0.05, t_far=1e3, jitter=0.4, contract=True):
    """Ragged unbounded-scene batch: s linear in disparity on [t_near, t_far].

    Ray r gets ``lengths[r]`` intervals with boundaries s_0 = 0, s_n = 1 and interior
    boundaries (j + U(-jitter, jitter)) / n, so interval lengths are non-uniform.
    delta is the contracted length (Eq. 4, p = inf, b = 1) of the interval divided by the
    voxel size, as the step is measured in contracted space.  The points are the contracted
    midpoints (contract=True) or the world midpoints, for grids that contract them on lookup.
    """
    R = o.shape[0]
    n = lengths.astype(np.int64)
    offs = np.zeros(R + 1, np.int64)
    np.cumsum(n, out=offs[1:])
    S = int(offs[-1])
    ray = np.repeat(np.arange(R), n)
    j = np.arange(S) - offs[ray]            # interval index within its ray
    nr = n[ray].astype(np.float64)
    # boundaries: left boundary of interval j and right boundary (j+1)
    jit = rng.uniform(-jitter, jitter, size=S)
    left = np.where(j == 0, 0.0, (j + jit) / nr)
    # right boundary of interval j is the left boundary of interval j+1 (or 1 at the end)
    right = np.empty(S)
    right[:-1] = left[1:]
    last = (j == n[ray] - 1)
    right[last] = 1.0
    s_mid = 0.5 * (left + right)
    s_len = right - left

    def t_of(s):
        return 1.0 / ((1.0 - s) / t_near + s / t_far)

    oo = o[ray]
    dd = d[ray]
    xw = oo + t_of(s_mid)[:, None] * dd
    xm = _contract_inf(xw) if contract else xw
    xl = _contract_inf(oo + t_of(left)[:, None] * dd)
    xr = _contract_inf(oo + t_of(right)[:, None] * dd)
    delta = np.linalg.norm(xr - xl, axis=1) / voxel
    return Samples(offs.astype(np.int32), xm.astype(F32), delta.astype(F32),
                   s_mid.astype(F32), s_len.astype(F32))


def random_ragged(rng, lengths, w_scale=1.0):
    """Random ragged weights and sorted intervals for distortion-loss unit tests.

    Returns (ray_offsets int32, w f32, s_mid f32, s_len f32).  Boundaries are sorted
    uniform draws on [0,1] per ray, so midpoints are non-decreasing.
    """
    lengths = np.asarray(lengths, np.int64)
    R = lengths.size
    offs = np.zeros(R + 1, np.int64)
    np.cumsum(lengths, out=offs[1:])
    w, m, l = [], [], []
    for r in range(R):
        nr = int(lengths[r])
        b = np.sort(rng.random(nr + 1))
        w.append(w_scale * rng.random(nr) / max(nr, 1) * 2.0)
        m.append(0.5 * (b[1:] + b[:-1]))
        l.append(b[1:] - b[:-1])
    cat = lambda a: np.concatenate(a).astype(F32) if a else np.zeros(0, F32)  # noqa: E731
    return offs.astype(np.int32), cat(w), cat(m), cat(l)


# ----------------------------------------------------------------------- MLPs


def _mlp(rng, sizes, bias_std=0.0) -> MLPWeights:
    W, b = [], []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        W.append((rng.standard_normal((fo, fi)) / np.sqrt(fi)).astype(F32))
        b.append((bias_std * rng.standard_normal(fo)).astype(F32))
    return MLPWeights(W, b)


def mlp_weights(rng, C=12, n_freq=4, hidden=128, bias_std=0.0) -> MLPWeights:
    """Colour MLP: [features(C), PE(view dir)(3 + 6*n_freq)] -> hidden -> hidden -> 3."""
    return _mlp(rng, [C + 3 + 6 * n_freq, hidden, hidden, 3], bias_std)


def proposal_weights(rng, n_bins=64, hidden=64, n_hidden=3, bias_std=0.0) -> MLPWeights:
    """Proposal MLP: coarse alpha(n_bins) -> hidden x n_hidden -> n_bins logits."""
    return _mlp(rng, [n_bins] + [hidden] * n_hidden + [n_bins], bias_std)


# -------------------------------------------------------------------- configs


def config1(R=1024, N=128, n=32) -> Workload:
    """Plain method, tiny: 32^3 density + 32^3x3 colour, 1024 rays x 128 uniform samples."""
    c = 1
    dens = blob_density(_rng(c, 0), n)
    col = uniform_grid(_rng(c, 1), n, 3)
    rays = rays_at_box(_rng(c, 3), R)
    smp = uniform_samples(rays, N, dens.voxel_size())
    tgt = _rng(c, 5).random((R, 3)).astype(F32)
    return Workload("config1", dens, col, None, None, rays, smp, tgt)


def _batch_rng(cfg: int, stream: int, batch: int) -> np.random.Generator:
    """Stream of batch 0 is the config's own; further batches of the same scene draw from their
    own seeds (1000 cfg + 100 batch + stream)."""
    return _rng(cfg, stream) if batch == 0 else np.random.Generator(np.random.PCG64(1000 * cfg + 100 * batch + stream))


def config2(R=8192, N=256, n=160, C=12, lo=0.2, hi=1.0, mlp_bias_std=0.0, batch=0) -> Workload:
    """Fine-stage shape: 160^3 density + 160^3x12 features + colour MLP, pinhole rays, ragged mask.
    batch > 0: another independently seeded ray batch (rays, mask, targets) of the same scene."""
    c = 2
    dens = blob_density(_rng(c, 0), n)
    feat = normal_grid(_rng(c, 1), n, C)
    mlp = mlp_weights(_rng(c, 2), C, bias_std=mlp_bias_std)
    rays = pinhole_rays(_batch_rng(c, 3, batch), R)
    r4 = _batch_rng(c, 4, batch)
    frac = r4.uniform(lo, hi, size=R)
    smp = uniform_samples(rays, N, dens.voxel_size(), live_frac=frac, rng=r4)
    tgt = _batch_rng(c, 5, batch).random((R, 3)).astype(F32)
    return Workload("config2", dens, None, feat, mlp, rays, smp, tgt)


def config3(R=8192, n=320, C=12, median=256, sigma=0.6, lmin=32, lmax=1024, contract_on_host=False) -> Workload:
    """Unbounded, ragged: [-2,2]^3 grids of 320^3 addressed through the Eq. 4 contraction
    (p = inf, b = 1), lognormal ray lengths in [32,1024].  Points are world points and the
    grids carry the contraction (warp 1), unless contract_on_host: then the points are
    contracted here and the grids take them directly."""
    c = 3
    b = 1.0
    lo, hi = -1.0 - b, 1.0 + b
    dens = blob_density(_rng(c, 0), n, lo, hi)
    feat = normal_grid(_rng(c, 1), n, C, lo, hi)
    if not contract_on_host:
        for g in (dens, feat):
            g.warp, g.warp_b = 1, b
    mlp = mlp_weights(_rng(c, 2), C)
    o, d = rays_into_ball(_rng(c, 3), R)
    r4 = _rng(c, 4)
    lengths = np.clip(np.round(r4.lognormal(np.log(median), sigma, size=R)), lmin, lmax).astype(np.int64)
    smp = disparity_samples(r4, o, d, lengths, dens.voxel_size(), contract=contract_on_host)
    rays = Rays(o.astype(F32), d.astype(F32), np.full(R, 0.05, F32), np.full(R, 1e3, F32), np.ones(R, bool))
    tgt = _rng(c, 5).random((R, 3)).astype(F32)
    return Workload("config3", dens, None, feat, mlp, rays, smp, tgt)


def config4(R=16384, N=512, n=160, C=12) -> Workload:
    """Differentiation/scale check: config-2 grids, 16384 rays x 512 samples, all live."""
    w2 = config2(R=8, n=n, C=C)  # same grids and MLP (streams 0-2 of config 2)
    rays = pinhole_rays(_rng(4, 3), R)
    smp = uniform_samples(rays, N, w2.density.voxel_size())
    tgt = _rng(4, 5).random((R, 3)).astype(F32)
    return Workload("config4", w2.density, None, w2.feat, w2.mlp, rays, smp, tgt)


def config6(R=8192, shape=(384, 384, 256), C=12, W=1008, H=756, focal=815.0) -> Workload:
    """Forward-facing (section 5.3): a multiplane-image-like volume of 256 planes of 384 x 384 in
    normalised device coordinates [-1,1]^3 (density + 12-channel features + colour MLP), and the
    rays of 20 forward-facing pinhole cameras (W x H, focal) in the reference camera's frame.
    The batch is made on the GPU by the NDC sampler (samples is None here)."""
    c = 6
    dens = blob_density(_rng(c, 0), shape)
    feat = normal_grid(_rng(c, 1), shape, C)
    mlp = mlp_weights(_rng(c, 2), C)
    o, d = forward_facing_rays(_rng(c, 3), R, W=W, H=H, focal=focal)
    rays = Rays(o, d, np.zeros(R, F32), np.zeros(R, F32), np.ones(R, bool))
    tgt = _rng(c, 5).random((R, 3)).astype(F32)
    wl = Workload("config6", dens, None, feat, mlp, rays, None, tgt)
    wl.extra["ndc"] = (2.0 * focal / W, 2.0 * focal / H, shape[2])
    return wl


def clear_free_space(density: Grid, blobs, keep_above=1.0, empty=-20.0) -> Grid:
    """Variant of a blob scene whose free space has been emptied, as occupancy masking and
    the distortion loss's compactness leave a trained grid (sections 1 and 2): vertices whose
    blob term is below `keep_above` get the logit `empty`; the blobs keep their noise."""
    data = np.where(blobs[..., None] >= keep_above, density.data, F32(empty)).astype(F32)
    return Grid(np.ascontiguousarray(data), density.xyz_min, density.xyz_max)


def config5(R=8192, n=160, C=12, held_out=False, cleared=False) -> Workload:
    """Proposal: config-2 grids and MLP; rays for training (stream 3) or held-out (stream 6).
    cleared=True empties the free space of the density grid (see clear_free_space)."""
    w2 = config2(R=8, n=n, C=C)
    if cleared:
        dens, blobs = blob_density(_rng(2, 0), n, return_blobs=True)   # config 2's density draw
        w2.density = clear_free_space(dens, blobs)
    rays = pinhole_rays(_rng(5, 6 if held_out else 3), R)
    smp = uniform_samples(rays, 256, w2.density.voxel_size())
    tgt = _rng(5, 5).random((R, 3)).astype(F32)
    wl = Workload("config5", w2.density, None, w2.feat, w2.mlp, rays, smp, tgt)
    wl.extra["proposal"] = proposal_weights(_rng(5, 7))
    return wl


def proposal_rays(R, stream, n=160):
    """Pinhole rays over the config-5 scene: stream 3 trains, 6 tunes, 8 evaluates."""
    box = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    return pinhole_rays(_rng(5, stream), R, bmin=box[0], bmax=box[1])
