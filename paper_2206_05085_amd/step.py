"""The per-ray training step on one GPU: every stage is a libdvgo kernel.

Feature-grid mode (hybrid colour, Table 1):
    grid_gather(features) -> mlp_forward (or both in mlp_forward_gather) -> render_forward (density gather, alpha,
    compositing, distortion) -> loss_head -> render_backward (density grad +=, d rgb)
    -> mlp_backward (d features, MLP grads +=) -> grid_scatter (feature grad +=)
    -> grid_adam_step x 3 (density, features, MLP) with zero-gradient skipping on the grids.
Colour-grid mode: render_forward/backward with a 3-channel colour grid, then Adam.

All buffers are allocated once per batch shape, so a step allocates nothing and can be
captured in a HIP graph (``capture``/``replay``).
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import ops


class TrainStep:
    def __init__(self, density, box, *, feat=None, color=None, mlp=None, n_freq=4, act_shift=None, halt_T=0.0,
                 bg=(1.0, 1.0, 1.0), dist_weight=0.01, lr_grid=0.1, lr_mlp=1e-3, betas=(0.9, 0.99), eps=1e-8,
                 tv=None, warp=None, mlp_precision=0, binned_scatter=True, owner_scatter=False, concurrent=True,
                 fused_gather=True, fused_render=True, device="cuda"):
        """density [n,n,n,1]; feat [n,n,n,C] with mlp = ([W1,W2,W3],[b1,b2,b3]) (MLP mode), or
        color [n,n,n,3] (grid mode).  Arrays may be numpy or torch; they are copied to the GPU.
        tv: optional (weight_density, weight_feat_or_color, huber_delta, dense) total-variation
        term, added into the grid gradients after the backward pass.  warp: optional (mode, b):
        every grid is addressed through the Eq. 4 contraction (ops.WARP_CONTRACT_INF or
        ops.WARP_CONTRACT_L2) and the batch holds world points.  mlp_precision: ops.MLP_SPLIT_F16
        (FP32-grade colour head) or ops.MLP_F16 (the cheaper head, FP16 matrix operands).
        binned_scatter: the renderer writes per-sample density gradients, which are scattered
        brick by brick (samples binned once per step) instead of by in-wave aggregated atomics
        inside the render kernel.  owner_scatter (with binned_scatter; off by default, the step measured
        about 1% slower with it): the density gradient is summed by the 4x4x32-vertex bricks that own the vertices (no global atomics), and when no TV
        term joins it, the density's Adam update is fused into that sum (its gradient never reaches
        memory); without it the density uses the atomic brick scatter.  The 12-channel feature
        gradient always takes the in-wave aggregated atomic scatter and the streaming Adam (the
        owner sum of 12 channels measured slower).  concurrent: in the feature-grid mode, run the binning, the
        density scatter, the density and MLP Adam updates and the colour head's preparation for
        the next step on a second stream, overlapped with the feature scatter and feature Adam
        (stream-ordered, graph-capturable).  A concurrent step leaves that preparation in the
        colour head's workspace and sets prepared_ahead, and the next step skips its own; bind(),
        optimise() and the sequential path clear the flag, and an in-place torch write to the MLP
        weights (which bumps their version) makes the next step prepare again.
        fused_gather: look the features up inside the colour head's forward kernel (which also
        writes them for the backward) instead of a separate gather kernel (feature rows whose
        channel count is a multiple of 4).  fused_render: in the concurrent step, the render
        forward, the loss gradient and the render backward run as one launch
        (ops.render_train; bit for bit the same results as the three calls)."""
        def dev(a):
            return torch.as_tensor(a).to(device=device, dtype=torch.float32).contiguous()

        self.device = device
        self.box = (tuple(float(v) for v in box[0]), tuple(float(v) for v in box[1]))
        self.grid_mode = color is not None
        self.shift = ops.act_shift() if act_shift is None else act_shift
        self.halt_T, self.bg, self.lam = halt_T, tuple(bg), dist_weight
        self.tv = None if tv is None else (float(tv[0]), float(tv[1]), float(tv[2]), bool(tv[3]))
        self.binned = bool(binned_scatter)
        self.owner = self.binned and bool(owner_scatter)
        self.concurrent = bool(concurrent)
        self.fused_render = bool(fused_render)
        self.side = None
        self.prepared_ahead = False  # the colour head's workspace holds the preparation for the next step
        self._prep_version = -1  # torch version of the MLP weights that preparation was made from
        self.warp = (0, 1.0) if warp is None else (int(warp[0]), float(warp[1]))
        self.fused_gather = bool(fused_gather) and feat is not None and np.shape(feat)[-1] % 4 == 0
        self.lr_grid, self.lr_mlp, self.betas, self.eps = lr_grid, lr_mlp, betas, eps
        self.t_dev = torch.zeros(1, dtype=torch.int32, device=device)  # Adam step, advanced on the device
        self.density = self._param(dev(density))
        if self.grid_mode:
            self.color = self._param(dev(color))
        else:
            self.feat = self._param(dev(feat))
            Ws, bs = mlp
            flat = torch.cat([dev(w).reshape(-1) for w in Ws] + [dev(b).reshape(-1) for b in bs])
            self.mlp_flat = self._param(flat)
            views, gviews, o = [], [], 0
            for t in [dev(w) for w in Ws] + [dev(b) for b in bs]:
                views.append(self.mlp_flat["p"][o:o + t.numel()].view(t.shape))
                gviews.append(self.mlp_flat["g"][o:o + t.numel()].view(t.shape))
                o += t.numel()
            self.mlp = ops.MLPParams(views[:3], views[3:], gviews[:3], gviews[3:], in_feat=int(self.feat["p"].shape[-1]),
                                     n_freq=n_freq, precision=mlp_precision)
        self.batch = None
        self.schedule = None
        self.successor = None

    def share_parameters(self, other: "TrainStep") -> "TrainStep":
        """Train the parameters (grids, colour head, moments, gradients and the Adam step counter)
        of `other`: two steps bound to different batches then update one model."""
        for name in ("density", "color", "feat", "mlp_flat", "mlp"):
            if hasattr(other, name):
                setattr(self, name, getattr(other, name))
        self.t_dev = other.t_dev
        return self

    def chain(self, successor: "TrainStep") -> "TrainStep":
        """The step that runs after this one (sharing its parameters, bound to another batch): this
        step's tail prepares the colour head for it (from the updated weights and its batch), so
        it skips its own preparation.  Steps (and graphs captured from them) must then run in the
        chained order."""
        self.successor = successor
        return self

    @staticmethod
    def _param(p):
        return {"p": p, "g": torch.zeros_like(p), "m": torch.zeros_like(p), "v": torch.zeros_like(p)}

    def grid(self, which) -> ops.DeviceGrid:
        d = getattr(self, which)
        return ops.DeviceGrid(d["p"], self.box[0], self.box[1], grad=d["g"],
                              channels=3 if which == "color" else None, warp=self.warp[0], warp_b=self.warp[1])

    def bind(self, batch: ops.SampleBatch, dirs, target):
        """Attach a sample batch (already on the GPU) and allocate every per-batch buffer.  A
        schedule tuned for an earlier batch is dropped (its ray list belongs to that batch)."""
        R, S = batch.n_rays, batch.n_samples
        d = self.device
        self.batch = batch
        self.schedule = None
        self.prepared_ahead = False
        self.dirs = torch.as_tensor(dirs).to(d, torch.float32).contiguous()
        self.target = torch.as_tensor(target).to(d, torch.float32).contiguous()
        self.rgb, self.T, self.dist = (torch.empty(R, 3, device=d), torch.empty(R, device=d),
                                       torch.empty(R, device=d))
        self.state = torch.empty(ops.render_state_size(R, S), dtype=torch.uint8, device=d)
        if self.binned:
            # one binning per step serves every grid of the same geometry
            self.g_raw = torch.empty(S, device=d)
            if self.owner:
                self.own_ws = torch.empty(max(ops.owner_workspace_size(self.grid("density"), S), 1),
                                          dtype=torch.uint8, device=d)
            else:
                self.bin_ws = torch.empty(max(ops.bin_workspace_size(self.grid("density"), S), 1),
                                          dtype=torch.uint8, device=d)

        self.loss = torch.zeros(1, device=d)
        self.g_rgb, self.g_dist = torch.empty(R, 3, device=d), torch.empty(R, device=d)
        if not self.grid_mode:
            C = self.mlp.in_feat
            self.feat_s = torch.empty(S, C, device=d)
            self.rgb_s = torch.empty(S, 3, device=d)
            self.g_rgb_s = torch.empty(S, 3, device=d)
            self.g_feat_s = torch.empty(S, C, device=d)
            self.mlp_ws = torch.empty(max(ops.mlp_workspace_size(self.mlp, R, S), 1), dtype=torch.uint8, device=d)
        return self

    def bind_rays(self, spec: ops.SamplerSpec, origins, dirs, target):
        """Produce the batch on the GPU from rays (box clipping + occupancy compaction with
        spec.mask) and bind it.  Reads the sample total back to the host (one small copy)."""
        o = torch.as_tensor(origins).to(self.device, torch.float32).contiguous()
        d = torch.as_tensor(dirs).to(self.device, torch.float32).contiguous()
        return self.bind(ops.sample_rays(spec, o, d), d, target)

    def update_occupancy(self, mask, alpha_thr: float = 1e-3, delta: float = 0.5):
        """Switch off mask vertices whose 3x3x3 neighbourhood has no density logit with alpha
        >= alpha_thr at a step of delta voxels (mask: uint8 over the density grid, in place)."""
        return ops.occupancy_update(self.grid("density"), self.shift, delta, alpha_thr, mask)

    def upscale(self, shape):
        """Progressive grid scaling: resample the density and feature (or colour) grids to
        shape = (nx, ny, nz) over the same box and restart their Adam moments.  Per-batch
        buffers that depend on the grid are re-allocated; a captured graph must be captured
        again."""
        for name in ("density", "color" if self.grid_mode else "feat"):
            d = getattr(self, name)
            new = ops.grid_resample(ops.DeviceGrid(d["p"], self.box[0], self.box[1]), shape)
            setattr(self, name, self._param(new))
        if self.batch is not None:
            self.bind(self.batch, self.dirs, self.target)
        self.graph = None
        return self

    def tune(self, longest_first: bool = True):
        """Pick the render kernels' launch shape with the library's autotuner (on the bound
        batch; call outside graph capture).  Returns (Schedule, ms of render fwd + bwd)."""
        b = self.batch
        order = ops.ray_schedule(b.ray_offsets)[0] if longest_first else None
        colour = self.grid("color") if self.grid_mode else None
        srgb = None if self.grid_mode else self.rgb_s
        self.schedule, ms = ops.render_autotune(b, self.grid("density"), colour, srgb, act_shift_=self.shift,
                                                halt_T=self.halt_T, bg=self.bg, ray_list=order,
                                                sample_density_grad=self.binned)
        return self.schedule, ms

    # --------------------------------------------------------------- stages
    def forward(self, gathered=False, loss_value=True, prepared=False):
        """gathered: the features of the samples are already in feat_s.  loss_value=False:
        the loss head writes only the gradients the backward needs (the caller reduces the
        loss value later, off the backward's path).  prepared: the colour MLP's preparation
        for this step is already in its workspace."""
        b = self.batch
        if self.grid_mode:
            ops.render_forward(b, self.grid("density"), self.grid("color"), None, act_shift_=self.shift,
                               halt_T=self.halt_T, bg=self.bg, want_dist=True, out=(self.rgb, self.T, self.dist),
                               state=self.state, schedule=self.schedule)
        else:
            self._colour_forward(gathered, prepared)
            ops.render_forward(b, self.grid("density"), None, self.rgb_s, act_shift_=self.shift, halt_T=self.halt_T,
                               bg=self.bg, want_dist=True, out=(self.rgb, self.T, self.dist), state=self.state,
                               schedule=self.schedule)
        ops.loss_head(self.rgb, self.target, self.dist, self.lam, loss=self.loss, grad_rgb=self.g_rgb,
                      grad_dist=self.g_dist, want_loss=loss_value)

    def _colour_forward(self, gathered, prepared):
        b = self.batch
        if self.fused_gather and not gathered:
            ops.mlp_forward_gather(self.mlp, b.ray_offsets, self.dirs, self.grid("feat"), b.xyz,
                                   feat_out=self.feat_s, rgb=self.rgb_s, ws=self.mlp_ws, prepared=prepared)
        else:
            if not gathered:
                ops.grid_gather(self.grid("feat"), b.xyz, out=self.feat_s)
            ops.mlp_forward(self.mlp, b.ray_offsets, self.dirs, self.feat_s, rgb=self.rgb_s, ws=self.mlp_ws,
                            prepared=prepared)

    def _render_fwd_bwd(self, gathered=False, prepared=False):
        """The concurrent step's forward and render backward: the colour head's forward, then the
        render forward, the loss gradients and the render backward (per-sample density gradients
        into g_raw, colour gradients into g_rgb_s), as one fused launch or as three."""
        b = self.batch
        if self.fused_render:
            self._colour_forward(gathered, prepared)
            ops.render_train(b, self.grid("density"), None, self.rgb_s, self.target, self.lam, act_shift_=self.shift,
                             halt_T=self.halt_T, bg=self.bg, want_dist=True, out=(self.rgb, self.T, self.dist),
                             state=self.state, grad_sample_rgb=self.g_rgb_s, schedule=self.schedule,
                             grad_sample_density=self.g_raw)
            return
        self.forward(gathered=gathered, loss_value=False, prepared=prepared)
        ops.render_backward(b, self.grid("density"), None, self.rgb_s, self.T, self.state, self.g_rgb, self.g_dist,
                            None, act_shift_=self.shift, halt_T=self.halt_T, bg=self.bg, grad_sample_rgb=self.g_rgb_s,
                            schedule=self.schedule, grad_sample_density=self.g_raw)

    def _bin(self):
        b = self.batch
        if self.owner:
            ops.owner_bin(self.grid("density"), b.xyz, ws=self.own_ws)
        else:
            ops.bin_samples(self.grid("density"), b.xyz, ws=self.bin_ws)

    def _scatter_density(self):
        b = self.batch
        if self.owner:
            ops.grid_scatter_owned(self.grid("density"), b.xyz, self.g_raw, self.own_ws)
        else:
            ops.grid_scatter_binned(self.grid("density"), b.xyz, self.g_raw, self.bin_ws)

    def _scatter_feat(self):
        # the 12-channel feature gradient keeps the in-wave aggregated atomic scatter (owner-brick sums
        # of 12 channels measured slower)
        ops.grid_scatter(self.grid("feat"), self.batch.xyz, self.g_feat_s)

    def _update_density(self):
        """The density gradient from the per-sample values (owner sum), the TV term, and Adam: fused
        into one kernel when there is no TV term."""
        b = self.batch
        if self.tv is None:
            d = self.density
            b1, b2 = self.betas
            ops.grid_scatter_adam(self.grid("density"), b.xyz, self.g_raw, self.own_ws, d["m"], d["v"],
                                  lr=self.lr_grid, beta1=b1, beta2=b2, eps=self.eps, step_dev=self.t_dev)
            return
        ops.grid_scatter_owned(self.grid("density"), b.xyz, self.g_raw, self.own_ws)
        ops.tv_add_grad(self.grid("density"), self.tv[0], self.tv[2], self.tv[3])
        self._adam("density", self.lr_grid, True)

    def _update_feat(self, counted=None):
        self._scatter_feat()
        if self.tv is not None:
            ops.tv_add_grad(self.grid("feat"), self.tv[1], self.tv[2], self.tv[3])
        if counted is not None:
            torch.cuda.current_stream().wait_event(counted)  # this step's Adam counter
        self._adam("feat", self.lr_grid, True)

    def backward(self):
        b = self.batch
        graw = None
        if self.binned:
            self._bin()
            graw = self.g_raw
        if self.grid_mode:
            ops.render_backward(b, self.grid("density"), self.grid("color"), None, self.T, self.state, self.g_rgb,
                                self.g_dist, None, act_shift_=self.shift, halt_T=self.halt_T, bg=self.bg,
                                schedule=self.schedule, grad_sample_density=graw)
        else:
            ops.render_backward(b, self.grid("density"), None, self.rgb_s, self.T, self.state, self.g_rgb,
                                self.g_dist, None, act_shift_=self.shift, halt_T=self.halt_T, bg=self.bg,
                                grad_sample_rgb=self.g_rgb_s, schedule=self.schedule, grad_sample_density=graw)
        if self.binned:
            self._scatter_density()
        if not self.grid_mode:
            self._mlp_backward_and_scatter()
        if self.tv is not None:
            # total-variation gradients go straight into the grid gradients before Adam (section 2)
            w_density, w_other, delta, dense = self.tv
            ops.tv_add_grad(self.grid("density"), w_density, delta, dense)
            ops.tv_add_grad(self.grid("color" if self.grid_mode else "feat"), w_other, delta, dense)

    def optimise(self):
        self.prepared_ahead = False  # the MLP weights change
        ops.counter_add(self.t_dev, 1)
        b1, b2 = self.betas
        groups = [("density", self.lr_grid, True), ("color" if self.grid_mode else "feat", self.lr_grid, True)]
        if not self.grid_mode:
            groups.append(("mlp_flat", self.lr_mlp, False))
        for name, lr, skip in groups:
            d = getattr(self, name)
            ops.grid_adam_step(d["p"], d["g"], d["m"], d["v"], lr=lr, beta1=b1, beta2=b2, eps=self.eps,
                               step_dev=self.t_dev, skip_zero_grad=skip, zero_grad_after=True)

    def _mlp_backward_and_scatter(self):
        b = self.batch
        ops.mlp_backward(self.mlp, b.ray_offsets, self.dirs, self.feat_s, self.g_rgb_s, grad_feat=self.g_feat_s,
                         ws=self.mlp_ws, prepared=True)
        self._scatter_feat()

    def _adam(self, name, lr, skip):
        b1, b2 = self.betas
        d = getattr(self, name)
        ops.grid_adam_step(d["p"], d["g"], d["m"], d["v"], lr=lr, beta1=b1, beta2=b2, eps=self.eps,
                           step_dev=self.t_dev, skip_zero_grad=skip, zero_grad_after=True)

    def step(self):
        if not (self.concurrent and self.binned and not self.grid_mode):
            self.prepared_ahead = False
            self.forward()
            self.backward()
            self.optimise()
            return self.loss
        if self.owner:
            return self._step_owner()
        return self._step_brick()

    def _fork_side(self):
        main = torch.cuda.current_stream()
        if self.side is None:
            self.side = torch.cuda.Stream(device=self.device)
        return main, self.side

    def _prepare_if_stale(self):
        b = self.batch
        # in-place torch writes to the weights (or their views) bump their version; the library's
        # own Adam does not
        if not self.prepared_ahead or self._prep_version != self.mlp_flat["p"]._version:
            ops.mlp_prepare(self.mlp, b.ray_offsets, self.dirs, b.n_samples, self.mlp_ws)

    def _side_tail(self, main, side, density_work, count=False):
        """After the colour-head backward: the side stream takes the colour head's weight-gradient
        reduction and Adam, its preparation for the next step, the loss value and then the density
        work (density_work); main continues with the feature update.  The colour head's short chain goes first:
        behind the density update it would run alone after main's feature Adam, the density Adam
        being slowed by sharing HBM with it (1.1% of the config-2 step).  count: the side first
        advances the Adam step counter (off main's path); the returned event marks it, for main's
        feature Adam."""
        b = self.batch
        side.wait_stream(main)
        counted = None
        with torch.cuda.stream(side):
            if count:
                ops.counter_add(self.t_dev, 1)  # the Adam step, before any update of this step
                counted = torch.cuda.Event()
                counted.record(side)
            ops.mlp_reduce_grads(self.mlp, b.n_rays, b.n_samples, self.mlp_ws)
            self._adam("mlp_flat", self.lr_mlp, False)
            if self.fused_gather:
                # the next step's preparation, from the updated weights (main reads the workspace
                # again only after the join); for a chained successor, with its batch
                nxt = self.successor or self
                nb = nxt.batch
                ops.mlp_prepare(self.mlp, nb.ray_offsets, nxt.dirs, nb.n_samples, nxt.mlp_ws)
            ops.loss_head(self.rgb, self.target, self.dist, self.lam, loss=self.loss, want_grad=False)
            density_work()
        return counted

    def _step_owner(self):
        # Two streams.  main: the colour head (with the feature lookup fused into its forward),
        # render forward and backward (per-sample density gradients), the colour-head backward
        # (weight gradients left as per-block partials), then the feature scatter and Adam (after an
        # event for the counter).  side, after the colour-head backward: the Adam step counter, the
        # colour head's weight-gradient reduction and Adam, its preparation for the next step, the
        # loss value, the owner binning of the samples and the density update (the owner-brick sum
        # of its per-sample gradients fused with its Adam step, or, with a TV term, the sum, the TV
        # gradient and Adam).
        # The binning depends only on the points, but run beside the colour head's forward it slows
        # that kernel by more than it takes; beside the feature scatter it is hidden.  Every Adam
        # launch follows the counter (in stream order, or through the event); each buffer has one
        # writer at a time; the side joins main at the end.
        main, side = self._fork_side()
        b = self.batch
        if self.fused_gather:
            # the Adam step counter advances on the side stream after the colour-head backward
            self._prepare_if_stale()
            self._render_fwd_bwd(prepared=True)
        else:
            side.wait_stream(main)  # the side's first kernels depend on nothing of this step
            ops.grid_gather(self.grid("feat"), b.xyz, out=self.feat_s)  # enqueued first: launched first
            with torch.cuda.stream(side):
                ops.counter_add(self.t_dev, 1)
                ops.mlp_prepare(self.mlp, b.ray_offsets, self.dirs, b.n_samples, self.mlp_ws)
                prepared = torch.cuda.Event()
                prepared.record(side)
            main.wait_event(prepared)
            self._render_fwd_bwd(gathered=True, prepared=True)
        ops.mlp_backward_partials(self.mlp, b.ray_offsets, self.dirs, self.feat_s, self.g_rgb_s, self.mlp_ws,
                                  grad_feat=self.g_feat_s, prepared=True)

        def density_work():
            self._bin()
            self._update_density()

        counted = self._side_tail(main, side, density_work, count=self.fused_gather)
        self._update_feat(counted)
        main.wait_stream(side)
        self._handed_prep()
        return self.loss

    def _handed_prep(self):
        nxt = self.successor or self
        if nxt is not self:
            self.prepared_ahead = False
        nxt.prepared_ahead = self.fused_gather
        nxt._prep_version = self.mlp_flat["p"]._version

    def _step_brick(self):
        # Two streams, atomic scatters.  main: colour head (with the feature gather fused into its
        # forward), render forward and backward, colour-head backward (its weight gradients left as
        # per-block partials), feature scatter, feature Adam (after an event for the counter).  side,
        # after the colour-head backward: the Adam step counter, the reduction of the weight
        # gradients, MLP Adam, the colour head's preparation for the next step, the loss value, the
        # binning and density scatter (+ TV), beside the feature scatter and Adam; after the join,
        # main runs the density Adam.  With the gather apart (features not a multiple of
        # 4 channels) the side also runs the counter, the colour head's preparation and the binning
        # beside the gather.
        main, side = self._fork_side()
        b = self.batch
        if self.fused_gather:
            # the Adam step counter advances on the side stream after the colour-head backward
            self._prepare_if_stale()
            self._render_fwd_bwd(prepared=True)
        else:
            side.wait_stream(main)  # the side's first kernels depend on nothing of this step
            ops.grid_gather(self.grid("feat"), b.xyz, out=self.feat_s)  # enqueued first: launched first
            with torch.cuda.stream(side):
                ops.counter_add(self.t_dev, 1)  # the Adam step, before any update of this step
                ops.mlp_prepare(self.mlp, b.ray_offsets, self.dirs, b.n_samples, self.mlp_ws)
                prepared = torch.cuda.Event()
                prepared.record(side)
                ops.bin_samples(self.grid("density"), b.xyz, ws=self.bin_ws)
                binned = torch.cuda.Event()
                binned.record(side)
            main.wait_event(prepared)  # the colour head's preparation and the step counter
            self._render_fwd_bwd(gathered=True, prepared=True)
            # An edge from the binning into main (long satisfied by now): without one, a graph
            # replay may launch the binning only behind main's last kernels, and the density work
            # with it.
            main.wait_event(binned)
        # the weight-gradient reduction waits on the side stream: only the MLP Adam needs it
        ops.mlp_backward_partials(self.mlp, b.ray_offsets, self.dirs, self.feat_s, self.g_rgb_s, self.mlp_ws,
                                  grad_feat=self.g_feat_s, prepared=True)

        def density_work():
            if self.fused_gather:
                ops.bin_samples(self.grid("density"), b.xyz, ws=self.bin_ws)
            ops.grid_scatter_binned(self.grid("density"), b.xyz, self.g_raw, self.bin_ws)
            if self.tv is not None:
                ops.tv_add_grad(self.grid("density"), self.tv[0], self.tv[2], self.tv[3])

        counted = self._side_tail(main, side, density_work, count=self.fused_gather)
        ops.grid_scatter(self.grid("feat"), b.xyz, self.g_feat_s)
        if self.tv is not None:
            ops.tv_add_grad(self.grid("feat"), self.tv[1], self.tv[2], self.tv[3])
        if counted is not None:
            main.wait_event(counted)  # this step's Adam counter
        self._adam("feat", self.lr_grid, True)
        main.wait_stream(side)
        # the density Adam last, on main: beside the feature Adam (both HBM-bound) it slowed that
        # update by more than it takes alone
        self._adam("density", self.lr_grid, True)
        self._handed_prep()
        return self.loss

    # ----------------------------------------------------------- HIP graphs
    def capture(self, warmup: int = 1) -> Optional[torch.cuda.CUDAGraph]:
        """Capture forward+backward+Adam of the bound batch in a graph.  Each replay is one
        full step: the Adam step counter lives on the device and is advanced inside the
        graph, so replays continue the bias correction exactly like eager steps.  A concurrent
        step captured after the warm-up leaves out its own colour-head preparation and takes the
        one the previous replay (or the warm-up) left in the workspace: capture again after
        bind() or after changing the MLP weights outside the step."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.step()
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g
        return g
