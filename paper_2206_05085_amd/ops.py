"""Thin Python binding of libdvgo: one function per C entry point, same names without the
``dvgo_`` prefix.  These functions only check and marshal arguments (torch CUDA tensors ->
device pointers, the current HIP stream); all arithmetic runs in the HIP kernels.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import (COLOR_GRID, COLOR_NONE, COLOR_SAMPLES, MLP_F16, MLP_SPLIT_F16, WARP_CONTRACT_INF, WARP_CONTRACT_L2, WARP_NONE, ColorMLP, Grid,
                   Proposal, Rays, RenderParams, Sampler, Samples, call)

__all__ = ["act_shift", "set_debug", "validate_samples", "SampleBatch", "DeviceGrid", "MLPParams", "Schedule", "ray_schedule", "render_autotune",
           "render_state_size", "render_forward",
           "render_backward", "render_train", "distortion_workspace_size", "distortion_loss", "distortion_loss_noalloc", "grid_adam_step", "counter_add", "grid_gather", "tv_add_grad",
           "grid_scatter", "grid_resample", "bin_workspace_size", "bin_samples", "grid_scatter_binned", "owner_workspace_size", "owner_bin", "grid_scatter_owned", "grid_scatter_adam", "alpha", "mlp_workspace_size", "mlp_prepare", "mlp_forward", "mlp_forward_gather", "mlp_backward",
           "mlp_backward_partials", "mlp_reduce_grads", "loss_head",
           "resample_guarded_offsets", "resample_guarded", "SamplerSpec", "sample_count", "sample_emit", "sample_rays", "occupancy_update",
           "COLOR_GRID", "COLOR_SAMPLES", "WARP_NONE", "WARP_CONTRACT_INF", "WARP_CONTRACT_L2",
           "MLP_SPLIT_F16", "MLP_F16"]


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _p(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _chk(t, name, dtype=torch.float32, numel=None, last=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU (libdvgo has no CPU path)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    if last is not None and (t.dim() == 0 or t.shape[-1] != last):
        raise ValueError(f"{name} must have last dimension {last}")
    return t


def act_shift(alpha_init: float = 1e-4, delta_ref: float = 0.5) -> float:
    """Shift b of sigma = softplus(raw + b) such that raw = 0 gives alpha_init at a step of
    delta_ref voxels (the initial-alpha setting of section 5.4); computed by dvgo_act_shift."""
    import ctypes
    out = ctypes.c_double()
    call("dvgo_act_shift", float(alpha_init), float(delta_ref), ctypes.byref(out))
    return out.value


def set_debug(on: bool) -> bool:
    """Debug mode of the library (batches validated on the device before every render and
    distortion call); returns the previous setting."""
    return bool(_lib.lib().dvgo_set_debug(1 if on else 0))


def validate_samples(batch: "SampleBatch") -> None:
    """Checks ray_offsets (0 first, non-decreasing, n_samples last) and per-ray sorted s_mid on
    the device; raises DvgoError (ERR_SHAPE / ERR_UNSORTED) otherwise.  Synchronises."""
    import ctypes
    s = batch.struct()
    call("dvgo_validate_samples", ctypes.byref(s), _stream())


@dataclass
class SampleBatch:
    """A ragged sample batch resident on the GPU (see dvgo_samples in include/dvgo.h)."""
    ray_offsets: torch.Tensor  # int32 [R+1]
    xyz: torch.Tensor          # [S,3]
    delta: torch.Tensor        # [S]
    s_mid: torch.Tensor        # [S]
    s_len: torch.Tensor        # [S]
    n_rays: int
    n_samples: int

    @classmethod
    def from_arrays(cls, ray_offsets, xyz, delta, s_mid, s_len, device="cuda"):
        def f(a, dt=torch.float32):
            return torch.as_tensor(a).to(device=device, dtype=dt).contiguous()
        offs = f(ray_offsets, torch.int32)
        n_rays = offs.numel() - 1
        n_samples = int(xyz.shape[0]) if hasattr(xyz, "shape") else len(xyz)
        return cls(offs, f(xyz).reshape(-1, 3), f(delta), f(s_mid), f(s_len), n_rays, n_samples)

    def struct(self) -> Samples:
        _chk(self.ray_offsets, "ray_offsets", torch.int32, self.n_rays + 1)
        for name in ("xyz", "delta", "s_mid", "s_len"):
            _chk(getattr(self, name), name, numel=self.n_samples * (3 if name == "xyz" else 1))
        return Samples(C_size(Samples), self.n_rays, self.n_samples, _p(self.ray_offsets), _p(self.xyz),
                       _p(self.delta), _p(self.s_mid), _p(self.s_len))


def C_size(struct_type) -> int:
    import ctypes
    return ctypes.sizeof(struct_type)


@dataclass
class DeviceGrid:
    """A dense channel-last vertex grid [nx, ny, nz, ch_stride] on the GPU plus its box."""
    data: torch.Tensor
    xyz_min: Sequence[float]
    xyz_max: Sequence[float]
    grad: Optional[torch.Tensor] = None
    channels: Optional[int] = None
    warp: int = 0          # WARP_NONE, WARP_CONTRACT_INF or WARP_CONTRACT_L2 (Eq. 4)
    warp_b: float = 1.0

    def struct(self, need_grad=False) -> Grid:
        _chk(self.data, "grid data")
        if self.data.dim() != 4:
            raise ValueError("grid data must be [nx, ny, nz, ch_stride]")
        nx, ny, nz, cs = self.data.shape
        if self.grad is not None:
            _chk(self.grad, "grid grad", numel=self.data.numel())
        elif need_grad:
            raise ValueError("grid grad buffer is required here")
        g = Grid()
        g.struct_size = C_size(Grid)
        g.nx, g.ny, g.nz = nx, ny, nz
        g.channels = cs if self.channels is None else self.channels
        g.ch_stride = cs
        g.xyz_min[:] = [float(v) for v in self.xyz_min]
        g.xyz_max[:] = [float(v) for v in self.xyz_max]
        g.data = _p(self.data)
        g.grad = _p(self.grad)
        g.warp = int(self.warp)
        g.warp_b = float(self.warp_b)
        return g


@dataclass
class MLPParams:
    """Colour MLP weights [out][in] (float32 on the GPU) and their gradient buffers."""
    W: list
    b: list
    gW: Optional[list] = None
    gb: Optional[list] = None
    in_feat: int = 12
    n_freq: int = 4
    precision: int = 0   # MLP_SPLIT_F16 (FP32-grade) or MLP_F16 (one FP16 product per product)

    def struct(self, need_grad=False, prepared=False) -> ColorMLP:
        """prepared: the workspace already holds this call's preparation (the previous MLP
        call on it had the same weights, unchanged since, and the same batch)."""
        for i, (w, b) in enumerate(zip(self.W, self.b)):
            _chk(w, f"W{i + 1}")
            _chk(b, f"b{i + 1}")
        m = ColorMLP()
        m.struct_size = C_size(ColorMLP)
        m.in_feat, m.n_freq, m.hidden = self.in_feat, self.n_freq, int(self.W[1].shape[0])
        m.precision = int(self.precision)
        m.prepared = int(bool(prepared))
        m.W1, m.W2, m.W3 = [_p(w) for w in self.W]
        m.b1, m.b2, m.b3 = [_p(b) for b in self.b]
        if self.gW is not None:
            for t in list(self.gW) + list(self.gb):
                _chk(t, "mlp gradient")
            m.gW1, m.gW2, m.gW3 = [_p(w) for w in self.gW]
            m.gb1, m.gb2, m.gb3 = [_p(b) for b in self.gb]
        elif need_grad:
            raise ValueError("MLP gradient buffers are required here")
        return m


@dataclass
class Schedule:
    """Launch schedule of the render kernels (see dvgo_render_params): an optional device
    list of rays (e.g. longest first), waves per block and a persistent grid size."""
    ray_list: Optional[torch.Tensor] = None
    waves_per_block: int = 0
    grid_waves: int = 0


def _params(act_shift_: float, halt_T: float, bg, color_mode: int, want_dist: bool,
            schedule: Optional[Schedule] = None) -> RenderParams:
    p = RenderParams()
    p.struct_size = C_size(RenderParams)
    p.act_shift = act_shift_
    p.halt_T = halt_T
    p.bg[:] = [float(v) for v in bg]
    p.color_mode = color_mode
    p.want_dist = 1 if want_dist else 0
    if schedule is not None:
        if schedule.ray_list is not None:
            _chk(schedule.ray_list, "ray_list", torch.int32)
            p.ray_list = _p(schedule.ray_list)
            p.n_list = schedule.ray_list.numel()
        p.waves_per_block = schedule.waves_per_block
        p.grid_waves = schedule.grid_waves
    return p


def ray_schedule(ray_offsets, order=None, class_offsets=None):
    """Rays sorted by decreasing chunk count (longest first) and the 65 class offsets."""
    R = ray_offsets.numel() - 1
    _chk(ray_offsets, "ray_offsets", torch.int32)
    order = torch.empty(R, dtype=torch.int32, device=ray_offsets.device) if order is None else order
    class_offsets = torch.empty(65, dtype=torch.int32, device=ray_offsets.device) if class_offsets is None else class_offsets
    call("dvgo_ray_schedule", R, _p(ray_offsets), _p(order), _p(class_offsets), _stream())
    return order, class_offsets


def render_autotune(batch: SampleBatch, density: DeviceGrid, color: Optional[DeviceGrid] = None,
                    sample_rgb: Optional[torch.Tensor] = None, *, act_shift_: float, halt_T: float = 0.0,
                    bg=(1.0, 1.0, 1.0), want_dist: bool = True, ray_list: Optional[torch.Tensor] = None,
                    sample_density_grad: bool = False):
    """Runs the library's autotuner; returns (Schedule, ms per forward + backward).
    sample_density_grad: time the backward that writes per-sample density gradients (the
    variant a caller that scatters them itself runs) instead of the in-kernel scatter."""
    import ctypes
    mode = COLOR_GRID if color is not None else COLOR_SAMPLES
    sched = Schedule(ray_list=ray_list)
    p = _params(act_shift_, halt_T, bg, mode, want_dist, sched)
    s = batch.struct()
    gd = density.struct()
    gc = color.struct() if color is not None else None
    wpb, gw, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_float(0)
    call("dvgo_render_autotune", ctypes.byref(p), ctypes.byref(s), ctypes.byref(gd),
         ctypes.byref(gc) if gc is not None else None, _p(sample_rgb), 1 if sample_density_grad else 0,
         ctypes.byref(wpb), ctypes.byref(gw), ctypes.byref(ms), _stream())
    return Schedule(ray_list, wpb.value, gw.value), ms.value


def _size(fn, *args) -> int:
    import ctypes
    out = ctypes.c_size_t(0)
    call(fn, *args, ctypes.byref(out))
    return int(out.value)


def render_state_size(n_rays: int, n_samples: int) -> int:
    return _size("dvgo_render_state_size", n_rays, n_samples)


def render_forward(batch: SampleBatch, density: DeviceGrid, color: Optional[DeviceGrid] = None,
                   sample_rgb: Optional[torch.Tensor] = None, *, act_shift_: float, halt_T: float = 0.0,
                   bg=(1.0, 1.0, 1.0), want_dist: bool = True, out=None, state: Optional[torch.Tensor] = None,
                   sample_w: Optional[torch.Tensor] = None, density_only: bool = False,
                   schedule: Optional[Schedule] = None):
    """Returns (rgb [R,3], T_final [R], dist [R] or None, state).  sample_w [S], if given,
    receives the per-sample weights; density_only renders with zero sample colours."""
    import ctypes
    mode = COLOR_NONE if density_only else (COLOR_GRID if color is not None else COLOR_SAMPLES)
    R, S = batch.n_rays, batch.n_samples
    dev = batch.xyz.device
    if out is None:
        out = (torch.empty(R, 3, device=dev), torch.empty(R, device=dev), torch.empty(R, device=dev))
    rgb, T, dist = out
    if state is None:
        state = torch.empty(render_state_size(R, S), dtype=torch.uint8, device=dev)
    if sample_rgb is not None:
        _chk(sample_rgb, "sample_rgb", numel=3 * S)
    if sample_w is not None:
        _chk(sample_w, "sample_w", numel=S)
    p = _params(act_shift_, halt_T, bg, mode, want_dist, schedule)
    s = batch.struct()
    gd = density.struct()
    gc = color.struct() if color is not None else None
    call("dvgo_render_forward", ctypes.byref(p), ctypes.byref(s), ctypes.byref(gd),
         ctypes.byref(gc) if gc is not None else None, _p(sample_rgb), _p(rgb), _p(T),
         _p(dist) if want_dist else None, _p(sample_w), _p(state), state.numel(), _stream())
    return rgb, T, (dist if want_dist else None), state


def render_backward(batch: SampleBatch, density: DeviceGrid, color: Optional[DeviceGrid], sample_rgb, T_final,
                    state, grad_rgb, grad_dist=None, grad_T=None, *, act_shift_: float, halt_T: float = 0.0,
                    bg=(1.0, 1.0, 1.0), want_dist: bool = True, grad_sample_rgb=None,
                    schedule: Optional[Schedule] = None, grad_sample_density=None):
    """Accumulates into density.grad (and color.grad); returns grad_sample_rgb (sample mode).
    With grad_sample_density [S], the per-sample density-logit gradient is written there
    instead of being added into density.grad."""
    import ctypes
    mode = COLOR_GRID if color is not None else COLOR_SAMPLES
    R, S = batch.n_rays, batch.n_samples
    _chk(grad_rgb, "grad_rgb", numel=3 * R)
    if grad_dist is not None:
        _chk(grad_dist, "grad_dist", numel=R)
    if grad_T is not None:
        _chk(grad_T, "grad_T", numel=R)
    if mode == COLOR_SAMPLES and grad_sample_rgb is None:
        grad_sample_rgb = torch.empty(S, 3, device=batch.xyz.device)
    p = _params(act_shift_, halt_T, bg, mode, want_dist, schedule)
    s = batch.struct()
    if grad_sample_density is not None:
        _chk(grad_sample_density, "grad_sample_density", numel=S)
    gd = density.struct(need_grad=grad_sample_density is None)
    gc = color.struct(need_grad=True) if color is not None else None
    call("dvgo_render_backward", ctypes.byref(p), ctypes.byref(s), ctypes.byref(gd),
         ctypes.byref(gc) if gc is not None else None, _p(sample_rgb), _p(T_final), _p(state), state.numel(),
         _p(grad_rgb), _p(grad_dist), _p(grad_T), _p(grad_sample_rgb), _p(grad_sample_density), _stream())
    return grad_sample_rgb


def render_train(batch: SampleBatch, density: DeviceGrid, color: Optional[DeviceGrid], sample_rgb, target,
                 dist_weight: float, *, act_shift_: float, halt_T: float = 0.0, bg=(1.0, 1.0, 1.0),
                 want_dist: bool = True, out=None, state: Optional[torch.Tensor] = None, grad_sample_rgb=None,
                 schedule: Optional[Schedule] = None, grad_sample_density=None):
    """render_forward, the loss head's gradients (MSE + dist_weight * distortion) and
    render_backward in one launch.  Returns (rgb, T_final, dist or None, state, grad_sample_rgb)."""
    import ctypes
    mode = COLOR_GRID if color is not None else COLOR_SAMPLES
    R, S = batch.n_rays, batch.n_samples
    dev = batch.xyz.device
    if out is None:
        out = (torch.empty(R, 3, device=dev), torch.empty(R, device=dev), torch.empty(R, device=dev))
    rgb, T, dist = out
    if state is None:
        state = torch.empty(render_state_size(R, S), dtype=torch.uint8, device=dev)
    _chk(target, "target", numel=3 * R)
    if sample_rgb is not None:
        _chk(sample_rgb, "sample_rgb", numel=3 * S)
    if mode == COLOR_SAMPLES and grad_sample_rgb is None:
        grad_sample_rgb = torch.empty(S, 3, device=dev)
    if grad_sample_density is not None:
        _chk(grad_sample_density, "grad_sample_density", numel=S)
    p = _params(act_shift_, halt_T, bg, mode, want_dist, schedule)
    s = batch.struct()
    gd = density.struct(need_grad=grad_sample_density is None)
    gc = color.struct(need_grad=True) if color is not None else None
    call("dvgo_render_train", ctypes.byref(p), ctypes.byref(s), ctypes.byref(gd),
         ctypes.byref(gc) if gc is not None else None, _p(sample_rgb), _p(target), float(dist_weight), _p(rgb), _p(T),
         _p(dist) if want_dist else None, _p(state), state.numel(), _p(grad_sample_rgb), _p(grad_sample_density),
         _stream())
    return rgb, T, (dist if want_dist else None), state, grad_sample_rgb


def distortion_workspace_size(n_rays: int, n_samples: int) -> int:
    return _size("dvgo_distortion_workspace_size", n_rays, n_samples)


def distortion_loss(ray_offsets, w, s_mid, s_len, grad_loss=None, grad_w=None, loss=None, ws=None):
    """Returns loss [R]; with grad_loss, also accumulates dD/dw into grad_w (allocated if None)."""
    R = ray_offsets.numel() - 1
    S = w.numel()
    _chk(ray_offsets, "ray_offsets", torch.int32)
    for t, n in ((w, "w"), (s_mid, "s_mid"), (s_len, "s_len")):
        _chk(t, n, numel=S)
    if loss is None:
        loss = torch.empty(R, device=w.device)
    if grad_loss is not None:
        _chk(grad_loss, "grad_loss", numel=R)
        if grad_w is None:
            grad_w = torch.zeros(S, device=w.device)
        if ws is None:
            ws = torch.empty(distortion_workspace_size(R, S), dtype=torch.uint8, device=w.device)
    call("dvgo_distortion_loss", R, _p(ray_offsets), S, _p(w), _p(s_mid), _p(s_len), _p(loss), _p(grad_loss),
         _p(grad_w), _p(ws), 0 if ws is None else ws.numel(), _stream())
    return loss, grad_w


def distortion_loss_noalloc(ray_offsets, w, s_mid, s_len, grad_loss=None, grad_w=None, loss=None):
    """distortion_loss without a workspace: the backward's checkpoints live in the library's fixed
    device array (no allocation by the library; loss / grad_w are allocated here only when not
    given).  Calls that overlap on one GPU race."""
    R = ray_offsets.numel() - 1
    S = w.numel()
    _chk(ray_offsets, "ray_offsets", torch.int32)
    for t, n in ((w, "w"), (s_mid, "s_mid"), (s_len, "s_len")):
        _chk(t, n, numel=S)
    if loss is None:
        loss = torch.empty(R, device=w.device)
    _chk(loss, "loss", numel=R)
    if grad_loss is not None:
        _chk(grad_loss, "grad_loss", numel=R)
        if grad_w is None:
            grad_w = torch.zeros(S, device=w.device)
        _chk(grad_w, "grad_w", numel=S)
    call("dvgo_distortion_loss_noalloc", R, _p(ray_offsets), S, _p(w), _p(s_mid), _p(s_len), _p(loss), _p(grad_loss),
         _p(grad_w) if grad_loss is not None else None, _stream())
    return loss, grad_w


def grid_adam_step(param, grad, exp_avg, exp_avg_sq, *, lr, beta1=0.9, beta2=0.99, eps=1e-8, step=0,
                   step_dev=None, skip_zero_grad=True, zero_grad_after=False):
    """step: 1-based Adam step, or step_dev: an int32 device tensor holding it."""
    n = param.numel()
    for t, nm in ((param, "param"), (grad, "grad"), (exp_avg, "exp_avg"), (exp_avg_sq, "exp_avg_sq")):
        _chk(t, nm, numel=n)
    if step_dev is not None:
        _chk(step_dev, "step_dev", torch.int32, numel=1)
    call("dvgo_grid_adam_step", _p(param), _p(grad), _p(exp_avg), _p(exp_avg_sq), n, lr, beta1, beta2, eps, step,
         _p(step_dev), 1 if skip_zero_grad else 0, 1 if zero_grad_after else 0, _stream())


def counter_add(counter, delta=1):
    _chk(counter, "counter", torch.int32, numel=1)
    call("dvgo_counter_add", _p(counter), delta, _stream())


def grid_gather(grid: DeviceGrid, xyz, out=None):
    import ctypes
    g = grid.struct()
    S = xyz.numel() // 3
    _chk(xyz, "xyz", numel=3 * S)
    if out is None:
        out = torch.empty(S, g.channels, device=xyz.device)
    _chk(out, "out", numel=S * g.channels)
    call("dvgo_grid_gather", ctypes.byref(g), S, _p(xyz), _p(out), _stream())
    return out


def grid_scatter(grid: DeviceGrid, xyz, grad_out):
    import ctypes
    g = grid.struct(need_grad=True)
    S = xyz.numel() // 3
    _chk(xyz, "xyz", numel=3 * S)
    _chk(grad_out, "grad_out", numel=S * g.channels)
    call("dvgo_grid_scatter", ctypes.byref(g), S, _p(xyz), _p(grad_out), _stream())


def grid_resample(grid: DeviceGrid, shape, out=None):
    """The grid resampled (trilinear) to shape (nx, ny, nz) over the same box: a new
    [nx, ny, nz, ch_stride] tensor (padding channels 0)."""
    nx, ny, nz = (int(v) for v in shape)
    cs = grid.data.shape[3]
    if out is None:
        out = torch.empty(nx, ny, nz, cs, device=grid.data.device)
    _chk(out, "out", numel=nx * ny * nz * cs)
    call("dvgo_grid_resample", ctypes_byref(grid.struct()), nx, ny, nz, _p(out), _stream())
    return out


def bin_workspace_size(grid: DeviceGrid, n_samples: int) -> int:
    return _size("dvgo_bin_workspace_size", ctypes_byref(grid.struct()), int(n_samples))


def bin_samples(grid: DeviceGrid, xyz, ws=None):
    """Sort the samples by the grid's 8^3-cell bricks (for grid_scatter_binned); returns ws."""
    _chk(xyz, "xyz", last=3)
    S = xyz.numel() // 3
    if ws is None:
        ws = torch.empty(max(bin_workspace_size(grid, S), 1), dtype=torch.uint8, device=xyz.device)
    call("dvgo_bin_samples", ctypes_byref(grid.struct()), S, _p(xyz), _p(ws), ws.numel(), _stream())
    return ws


def grid_scatter_binned(grid: DeviceGrid, xyz, grad_out, ws):
    """grid.grad += trilinear^T(grad_out), brick by brick, with the bins of bin_samples."""
    _chk(xyz, "xyz", last=3)
    S = xyz.numel() // 3
    _chk(grad_out, "grad_out", numel=S * grid.struct().channels)
    call("dvgo_grid_scatter_binned", ctypes_byref(grid.struct(need_grad=True)), S, _p(xyz), _p(grad_out), _p(ws),
         ws.numel(), _stream())


def owner_workspace_size(grid: DeviceGrid, n_samples: int) -> int:
    return _size("dvgo_owner_workspace_size", ctypes_byref(grid.struct()), int(n_samples))


def owner_bin(grid: DeviceGrid, xyz, ws=None):
    """Sort the (sample, owning 4x4x32-vertex brick) pairs of the points (for grid_scatter_owned and
    grid_scatter_adam); returns ws."""
    _chk(xyz, "xyz", last=3)
    S = xyz.numel() // 3
    if ws is None:
        ws = torch.empty(max(owner_workspace_size(grid, S), 1), dtype=torch.uint8, device=xyz.device)
    call("dvgo_owner_bin", ctypes_byref(grid.struct()), S, _p(xyz), _p(ws), ws.numel(), _stream())
    return ws


def grid_scatter_owned(grid: DeviceGrid, xyz, grad_out, ws):
    """grid.grad += trilinear^T(grad_out), each vertex updated once by its owning brick (bins of
    owner_bin), with no atomics."""
    _chk(xyz, "xyz", last=3)
    S = xyz.numel() // 3
    _chk(grad_out, "grad_out", numel=S * grid.struct().channels)
    call("dvgo_grid_scatter_owned", ctypes_byref(grid.struct(need_grad=True)), S, _p(xyz), _p(grad_out), _p(ws),
         ws.numel(), _stream())


def grid_scatter_adam(grid: DeviceGrid, xyz, grad_out, ws, exp_avg, exp_avg_sq, *, lr, beta1=0.9, beta2=0.99,
                      eps=1e-8, step=0, step_dev=None):
    """The skipping Adam update of grid.data (in place) with the gradient trilinear^T(grad_out)
    formed per brick on chip (bins of owner_bin); grid.grad is not used."""
    _chk(xyz, "xyz", last=3)
    S = xyz.numel() // 3
    g = grid.struct()
    _chk(grad_out, "grad_out", numel=S * g.channels)
    n = grid.data.numel()
    for t, nm in ((exp_avg, "exp_avg"), (exp_avg_sq, "exp_avg_sq")):
        _chk(t, nm, numel=n)
    if step_dev is not None:
        _chk(step_dev, "step_dev", torch.int32, numel=1)
    call("dvgo_grid_scatter_adam", ctypes_byref(g), S, _p(xyz), _p(grad_out), _p(ws), ws.numel(), _p(grid.data),
         _p(exp_avg), _p(exp_avg_sq), lr, beta1, beta2, eps, step, _p(step_dev), _stream())


def ctypes_byref(x):
    import ctypes
    return ctypes.byref(x)


def tv_add_grad(grid: DeviceGrid, weight: float, delta: float = 1.0, dense: bool = True):
    """grid.grad += gradient of the total-variation regulariser (Huber to the six axis
    neighbours, mean over vertices and channels, scaled by weight); dense=False updates only
    vertices whose incoming gradient is non-zero."""
    import ctypes
    g = grid.struct(need_grad=True)
    call("dvgo_tv_add_grad", ctypes.byref(g), float(weight), float(delta), 1 if dense else 0, _stream())


def alpha(density: DeviceGrid, xyz, delta, act_shift_: float, out=None):
    import ctypes
    g = density.struct()
    S = delta.numel()
    _chk(xyz, "xyz", numel=3 * S)
    _chk(delta, "delta", numel=S)
    if out is None:
        out = torch.empty(S, device=delta.device)
    call("dvgo_alpha", ctypes.byref(g), S, _p(xyz), _p(delta), act_shift_, _p(out), _stream())
    return out


def mlp_workspace_size(mlp: MLPParams, n_rays: int, n_samples: int) -> int:
    import ctypes
    return _size("dvgo_mlp_workspace_size", ctypes.byref(mlp.struct()), n_rays, n_samples)


def _mlp_ws(mlp, R, S, ws, dev):
    need = mlp_workspace_size(mlp, R, S)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    return ws


def mlp_prepare(mlp: MLPParams, ray_offsets, dirs, n_samples, ws):
    """Write the colour MLP's preparation for this batch into ws (then pass prepared=True)."""
    import ctypes
    R = ray_offsets.numel() - 1
    _chk(ray_offsets, "ray_offsets", torch.int32)
    _chk(dirs, "dirs", numel=3 * R)
    call("dvgo_mlp_prepare", ctypes.byref(mlp.struct()), R, _p(ray_offsets), _p(dirs), int(n_samples), _p(ws),
         ws.numel(), _stream())
    return ws


def mlp_forward(mlp: MLPParams, ray_offsets, dirs, feat, rgb=None, ws=None, prepared=False):
    """prepared=True: ws already holds this batch's preparation (mlp_prepare or a preceding
    MLP call with the same weights and batch)."""
    import ctypes
    R = ray_offsets.numel() - 1
    S = feat.shape[0]
    _chk(ray_offsets, "ray_offsets", torch.int32)
    _chk(dirs, "dirs", numel=3 * R)
    _chk(feat, "feat", numel=S * mlp.in_feat)
    if prepared and ws is None:
        raise ValueError("prepared=True needs the workspace of the preceding call")
    if rgb is None:
        rgb = torch.empty(S, 3, device=feat.device)
    ws = _mlp_ws(mlp, R, S, ws, feat.device)
    m = mlp.struct(prepared=prepared)
    call("dvgo_mlp_forward", ctypes.byref(m), R, _p(ray_offsets), _p(dirs), S, _p(feat), _p(rgb), _p(ws),
         ws.numel(), _stream())
    return rgb


def mlp_forward_gather(mlp: MLPParams, ray_offsets, dirs, feat_grid: DeviceGrid, xyz, feat_out=None, rgb=None,
                       ws=None, prepared=False):
    """Colour MLP forward whose features are looked up in feat_grid at xyz inside the kernel (the
    same values grid_gather gives, bit for bit); feat_out [S, in_feat] (optional) receives them."""
    import ctypes
    R = ray_offsets.numel() - 1
    S = xyz.shape[0]
    _chk(ray_offsets, "ray_offsets", torch.int32)
    _chk(dirs, "dirs", numel=3 * R)
    _chk(xyz, "xyz", numel=3 * S)
    if feat_out is not None:
        _chk(feat_out, "feat_out", numel=S * mlp.in_feat)
    if prepared and ws is None:
        raise ValueError("prepared=True needs the workspace of the preceding call")
    if rgb is None:
        rgb = torch.empty(S, 3, device=xyz.device)
    ws = _mlp_ws(mlp, R, S, ws, xyz.device)
    call("dvgo_mlp_forward_gather", ctypes.byref(mlp.struct(prepared=prepared)), R, _p(ray_offsets), _p(dirs), S,
         ctypes.byref(feat_grid.struct()), _p(xyz), _p(feat_out), _p(rgb), _p(ws), ws.numel(), _stream())
    return rgb


def mlp_backward(mlp: MLPParams, ray_offsets, dirs, feat, grad_rgb, grad_feat=None, ws=None, prepared=False):
    """prepared=True reuses the preparation a preceding mlp_forward on the same ws wrote
    (same weights and batch); it needs an explicit ws."""
    return _mlp_backward_call("dvgo_mlp_backward", mlp, ray_offsets, dirs, feat, grad_rgb, grad_feat, ws, prepared)


def _mlp_backward_call(entry, mlp, ray_offsets, dirs, feat, grad_rgb, grad_feat, ws, prepared):
    import ctypes
    if prepared and ws is None:
        raise ValueError("prepared=True needs the workspace of the preceding call")
    R = ray_offsets.numel() - 1
    S = feat.shape[0]
    _chk(grad_rgb, "grad_rgb", numel=3 * S)
    if grad_feat is None:
        grad_feat = torch.empty(S, mlp.in_feat, device=feat.device)
    ws = _mlp_ws(mlp, R, S, ws, feat.device)
    m = mlp.struct(need_grad=True, prepared=prepared)
    call(entry, ctypes.byref(m), R, _p(ray_offsets), _p(dirs), S, _p(feat), _p(grad_rgb),
         _p(grad_feat), _p(ws), ws.numel(), _stream())
    return grad_feat


def mlp_backward_partials(mlp: MLPParams, ray_offsets, dirs, feat, grad_rgb, ws, grad_feat=None, prepared=False):
    """mlp_backward with the weight and bias gradients left in ws as per-block partials;
    mlp_reduce_grads on the same ws adds them into the gradient buffers."""
    return _mlp_backward_call("dvgo_mlp_backward_partials", mlp, ray_offsets, dirs, feat, grad_rgb, grad_feat, ws,
                              prepared)


def mlp_reduce_grads(mlp: MLPParams, n_rays: int, n_samples: int, ws):
    """Add the partials a preceding mlp_backward_partials left in ws into mlp.gW / mlp.gb."""
    import ctypes
    call("dvgo_mlp_reduce_grads", ctypes.byref(mlp.struct(need_grad=True)), int(n_rays), int(n_samples), _p(ws),
         ws.numel(), _stream())


def loss_head(rgb, target, dist, dist_weight, loss=None, grad_rgb=None, grad_dist=None, want_loss=True,
              want_grad=True):
    """want_loss / want_grad = False leave that part out (its outputs are then None): the
    gradients alone take a many-block launch, the loss a one-block reduction."""
    R = rgb.shape[0]
    _chk(rgb, "rgb", numel=3 * R)
    _chk(target, "target", numel=3 * R)
    if dist is not None:
        _chk(dist, "dist", numel=R)
    if not (want_loss or want_grad):
        raise ValueError("loss_head: nothing requested")
    dev = rgb.device
    loss = (torch.empty(1, device=dev) if loss is None else loss) if want_loss else None
    if want_grad:
        grad_rgb = torch.empty(R, 3, device=dev) if grad_rgb is None else grad_rgb
        if grad_dist is None and dist is not None:
            grad_dist = torch.empty(R, device=dev)
    else:
        grad_rgb = grad_dist = None
    call("dvgo_loss_head", R, _p(rgb), _p(target), _p(dist), dist_weight, _p(loss), _p(grad_rgb), _p(grad_dist),
         _stream())
    return loss, grad_rgb, grad_dist


# --------------------------------------------------------------- proposal stage


@dataclass
class RayBatch:
    """Bounded-scene rays on the GPU (see dvgo_rays)."""
    origins: torch.Tensor
    dirs: torch.Tensor
    t_near: torch.Tensor
    t_far: torch.Tensor

    @classmethod
    def from_arrays(cls, origins, dirs, t_near, t_far, device="cuda"):
        f = lambda a: torch.as_tensor(a).to(device=device, dtype=torch.float32).contiguous()  # noqa: E731
        return cls(f(origins).reshape(-1, 3), f(dirs).reshape(-1, 3), f(t_near), f(t_far))

    @property
    def n_rays(self):
        return int(self.t_near.numel())

    def struct(self) -> Rays:
        R = self.n_rays
        for t, n, k in ((self.origins, "origins", 3), (self.dirs, "dirs", 3), (self.t_near, "t_near", 1),
                        (self.t_far, "t_far", 1)):
            _chk(t, n, numel=k * R)
        return Rays(C_size(Rays), R, _p(self.origins), _p(self.dirs), _p(self.t_near), _p(self.t_far))


@dataclass
class ProposalParams:
    """Proposal MLP float32 master weights (4 layers, 64 wide) and gradient buffers."""
    W: list
    b: list
    gW: Optional[list] = None
    gb: Optional[list] = None

    def struct(self, need_grad=False) -> Proposal:
        import ctypes
        q = Proposal()
        q.struct_size = C_size(Proposal)
        q.n_bins, q.hidden, q.n_layers = int(self.W[-1].shape[0]), int(self.W[0].shape[0]), len(self.W)
        for i, (w, b) in enumerate(zip(self.W, self.b)):
            _chk(w, f"proposal W{i}")
            _chk(b, f"proposal b{i}")
            q.W[i], q.b[i] = _p(w), _p(b)
        if self.gW is not None:
            for i, (w, b) in enumerate(zip(self.gW, self.gb)):
                _chk(w, f"proposal gW{i}")
                _chk(b, f"proposal gb{i}")
                q.gW[i], q.gb[i] = _p(w), _p(b)
        elif need_grad:
            raise ValueError("proposal gradient buffers are required here")
        del ctypes
        return q


def proposal_coarse(rays: RayBatch, density: DeviceGrid, *, act_shift_: float, voxel: float, eps: float = 1e-4,
                    feat=None, w_coarse=None):
    import ctypes
    R = rays.n_rays
    dev = rays.t_near.device
    feat = torch.empty(R, 64, device=dev) if feat is None else feat
    r = rays.struct()
    g = density.struct()
    call("dvgo_proposal_coarse", ctypes.byref(r), ctypes.byref(g), act_shift_, voxel, eps, _p(feat), _p(w_coarse),
         _stream())
    return feat, w_coarse


def proposal_forward(prop: ProposalParams, feat, logits=None, prob=None, entropy=None):
    import ctypes
    R = feat.shape[0]
    _chk(feat, "feat", numel=64 * R)
    dev = feat.device
    logits = torch.empty(R, 64, device=dev) if logits is None else logits
    prob = torch.empty(R, 64, device=dev) if prob is None else prob
    entropy = torch.empty(R, device=dev) if entropy is None else entropy
    q = prop.struct()
    call("dvgo_proposal_forward", ctypes.byref(q), R, _p(feat), _p(logits), _p(prob), _p(entropy), _stream())
    return logits, prob, entropy


def proposal_workspace_size(prop: ProposalParams, n_rays: int) -> int:
    import ctypes
    return _size("dvgo_proposal_workspace_size", ctypes.byref(prop.struct()), n_rays)


def proposal_backward(prop: ProposalParams, feat, target, loss=None, ws=None):
    import ctypes
    R = feat.shape[0]
    _chk(feat, "feat", numel=64 * R)
    _chk(target, "target", numel=64 * R)
    loss = torch.empty(1, device=feat.device) if loss is None else loss
    need = proposal_workspace_size(prop, R)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=feat.device)
    q = prop.struct(need_grad=True)
    call("dvgo_proposal_backward", ctypes.byref(q), R, _p(feat), _p(target), _p(loss), _p(ws), ws.numel(), _stream())
    return loss


def histogram(ray_offsets, w, s_mid, n_bins=64, min_mass=1e-4, hist=None):
    R = ray_offsets.numel() - 1
    _chk(ray_offsets, "ray_offsets", torch.int32)
    _chk(w, "w")
    _chk(s_mid, "s_mid", numel=w.numel())
    hist = torch.empty(R, n_bins, device=w.device) if hist is None else hist
    call("dvgo_histogram", R, _p(ray_offsets), _p(w), _p(s_mid), n_bins, min_mass, _p(hist), _stream())
    return hist


def resample_offsets(rays: RayBatch, entropy, tau, n_fine=48, n_plain=256, ray_offsets=None):
    import ctypes
    R = rays.n_rays
    _chk(entropy, "entropy", numel=R)
    ray_offsets = torch.empty(R + 1, dtype=torch.int32, device=entropy.device) if ray_offsets is None else ray_offsets
    r = rays.struct()
    call("dvgo_resample_offsets", ctypes.byref(r), _p(entropy), tau, n_fine, n_plain, _p(ray_offsets), _stream())
    return ray_offsets


def resample(rays: RayBatch, prob, entropy, tau, ray_offsets, n_samples, voxel, n_fine=48, n_plain=256, out=None):
    """Fills a fine batch of n_samples (= ray_offsets[-1]) samples; returns a SampleBatch."""
    import ctypes
    R = rays.n_rays
    _chk(prob, "prob", numel=64 * R)
    dev = prob.device
    if out is None:
        out = (torch.empty(n_samples, 3, device=dev), torch.empty(n_samples, device=dev),
               torch.empty(n_samples, device=dev), torch.empty(n_samples, device=dev))
    xyz, dl, sm, sl = out
    r = rays.struct()
    call("dvgo_resample", ctypes.byref(r), _p(prob), _p(entropy), tau, _p(ray_offsets), n_fine, n_plain, voxel,
         _p(xyz), _p(dl), _p(sm), _p(sl), _stream())
    return SampleBatch(ray_offsets, xyz, dl, sm, sl, R, int(n_samples))


def resample_guarded_offsets(rays: RayBatch, prob, w_coarse, entropy, tau, n_base=4, n_extra=32, w_min=1e-4,
                             ray_offsets=None, counts=None):
    """Guarded resampling layout: occupied coarse bins get n_base + their share of n_extra
    sub-intervals; returns (ray_offsets [R+1], counts [R,64])."""
    import ctypes
    R = rays.n_rays
    _chk(prob, "prob", numel=64 * R)
    _chk(w_coarse, "w_coarse", numel=64 * R)
    _chk(entropy, "entropy", numel=R)
    dev = prob.device
    ray_offsets = torch.empty(R + 1, dtype=torch.int32, device=dev) if ray_offsets is None else ray_offsets
    counts = torch.empty(R, 64, dtype=torch.int32, device=dev) if counts is None else counts
    r = rays.struct()
    call("dvgo_resample_guarded_offsets", ctypes.byref(r), _p(prob), _p(w_coarse), _p(entropy), float(tau),
         int(n_base), int(n_extra), float(w_min), _p(ray_offsets), _p(counts), _stream())
    return ray_offsets, counts


def resample_guarded(rays: RayBatch, ray_offsets, counts, n_samples, voxel, out=None):
    """Fills the guarded fine batch laid out by resample_guarded_offsets; returns a SampleBatch."""
    import ctypes
    R = rays.n_rays
    _chk(counts, "counts", torch.int32, numel=64 * R)
    dev = counts.device
    if out is None:
        out = (torch.empty(n_samples, 3, device=dev), torch.empty(n_samples, device=dev),
               torch.empty(n_samples, device=dev), torch.empty(n_samples, device=dev))
    xyz, dl, sm, sl = out
    r = rays.struct()
    call("dvgo_resample_guarded", ctypes.byref(r), _p(ray_offsets), _p(counts), float(voxel), _p(xyz), _p(dl),
         _p(sm), _p(sl), _stream())
    return SampleBatch(ray_offsets, xyz, dl, sm, sl, R, int(n_samples))


# ------------------------------------------------------------------ sample producer


@dataclass
class SamplerSpec:
    """Scene box, spacing and occupancy mask of the sample producer (dvgo_sampler).  Box mode
    (default): step and voxel in world units.  NDC mode (ndc = (fx, fy, planes), fx = 2 focal / W,
    fy = 2 focal / H): step in planes, near = the camera's near plane, voxel unused."""
    xyz_min: Sequence[float]
    xyz_max: Sequence[float]
    step: float
    voxel: float = 1.0
    near: float = 0.0
    max_per_ray: int = 4096
    mask: Optional[torch.Tensor] = None  # uint8 [nx, ny, nz] on the GPU, or None (all active)
    ndc: Optional[tuple] = None

    def struct(self) -> Sampler:
        sp = Sampler()
        sp.struct_size = C_size(Sampler)
        if self.ndc is not None:
            sp.mode = _lib.SAMPLE_NDC
            sp.ndc_fx, sp.ndc_fy, sp.ndc_planes = float(self.ndc[0]), float(self.ndc[1]), int(self.ndc[2])
        sp.xyz_min[:] = [float(v) for v in self.xyz_min]
        sp.xyz_max[:] = [float(v) for v in self.xyz_max]
        sp.near, sp.step, sp.voxel = float(self.near), float(self.step), float(self.voxel)
        sp.max_per_ray = int(self.max_per_ray)
        if self.mask is not None:
            _chk(self.mask, "mask", torch.uint8)
            if self.mask.dim() != 3:
                raise ValueError("mask must be [nx, ny, nz]")
            sp.mask_shape[:] = list(self.mask.shape)
            sp.mask = _p(self.mask)
        return sp


def _rays(origins, dirs):
    _chk(origins, "origins", last=3)
    R = origins.numel() // 3
    _chk(dirs, "dirs", numel=3 * R)
    return R


def sample_count(spec: SamplerSpec, origins, dirs, ray_offsets=None, t_near=None, t_far=None):
    """Kept samples per ray as ray_offsets [R+1] (int32, exclusive prefix); optional box interval."""
    R = _rays(origins, dirs)
    dev = origins.device
    if ray_offsets is None:
        ray_offsets = torch.empty(R + 1, dtype=torch.int32, device=dev)
    _chk(ray_offsets, "ray_offsets", torch.int32, R + 1)
    for name, t in (("t_near", t_near), ("t_far", t_far)):
        if t is not None:
            _chk(t, name, numel=R)
    call("dvgo_sample_count", spec.struct(), R, _p(origins), _p(dirs), _p(ray_offsets), _p(t_near), _p(t_far),
         _stream())
    return ray_offsets


def sample_emit(spec: SamplerSpec, origins, dirs, ray_offsets, n_samples: int, out=None) -> SampleBatch:
    """Fills the batch laid out by sample_count; n_samples = ray_offsets[R] (the capacity)."""
    R = _rays(origins, dirs)
    dev = origins.device
    _chk(ray_offsets, "ray_offsets", torch.int32, R + 1)
    if out is None:
        out = SampleBatch(ray_offsets, torch.empty(n_samples, 3, device=dev), torch.empty(n_samples, device=dev),
                          torch.empty(n_samples, device=dev), torch.empty(n_samples, device=dev), R, n_samples)
    for name in ("xyz", "delta", "s_mid", "s_len"):
        _chk(getattr(out, name), name, numel=n_samples * (3 if name == "xyz" else 1))
    call("dvgo_sample_emit", spec.struct(), R, _p(origins), _p(dirs), _p(ray_offsets), int(n_samples), _p(out.xyz),
         _p(out.delta), _p(out.s_mid), _p(out.s_len), _stream())
    return out


def sample_rays(spec: SamplerSpec, origins, dirs) -> SampleBatch:
    """Count, read the total (one 4-byte device-to-host copy, which synchronises), emit."""
    offs = sample_count(spec, origins, dirs)
    total = int(offs[-1].item())
    return sample_emit(spec, origins, dirs, offs, total)


def occupancy_update(density: DeviceGrid, act_shift_: float, delta: float, alpha_thr: float, mask):
    """In place: mask &= 27-neighbour dilation of (alpha of the vertex logit at step delta >= alpha_thr)."""
    g = density.struct()
    _chk(mask, "mask", torch.uint8, g.nx * g.ny * g.nz)
    call("dvgo_occupancy_update", g, float(act_shift_), float(delta), float(alpha_thr), _p(mask), _stream())
    return mask
