"""The optimisation loop of the method (Sec. 4.1): one photometric loss,
Adam with the 3D Gaussian-splatting settings except a position learning
rate of 1e-5, the schedule stretched to the iteration budget, no
densification.

One step = preprocess -> bin/sort -> render -> L1 + w (1 - SSIM) and its
gradient -> render/preprocess backward -> Adam, every stage a HIP kernel of
libgs4d.so launched on the current stream with no host synchronisation.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import gs4d as G
from .rasterizer import Rasterizer

# Learning rates per parameter row (READING of "standard 3DGS
# hyper-parameters" for this parameterisation; only the position rate is
# given by the paper).
LR_POSITION = 1e-5
LR_DEFAULTS = {
    "mean_xyz": (LR_POSITION, LR_POSITION * 0.01),
    "mean_t": (LR_POSITION, LR_POSITION * 0.01),
    "log_scale": (5e-3, 5e-3),
    "rotors": (1e-3, 1e-3),
    "opacity": (5e-2, 5e-2),
    "rgb": (2.5e-3, 2.5e-3),
    # isotropic, motion-aware form only: the velocity (world units per unit
    # of normalised time); 1e-2 beat 3e-3 and 1e-3 on held-out PSNR after
    # 1,500 scene steps
    "velocity": (1e-2, 1e-4),
    # SCH colour only: the constant (n = 0, l = 0) coefficient at the RGB
    # rate in colour units (the basis value Y_00 = 1 / (2 sqrt(pi)) scales
    # it), every higher coefficient at 1/20 of that (the 3D Gaussian-
    # splatting ratio of its higher spherical-harmonic bands)
    "sch_dc": (2.5e-3 * 2.0 * math.sqrt(math.pi), 2.5e-3 * 2.0 * math.sqrt(math.pi)),
    "sch_rest": (2.5e-3 * 2.0 * math.sqrt(math.pi) / 20, 2.5e-3 * 2.0 * math.sqrt(math.pi) / 20),
}

ROTOR_ROWS = (["mean_xyz"] * 3 + ["mean_t"] + ["log_scale"] * 4 + ["rotors"] * 8 + ["opacity"]
              + ["rgb"] * 3)
ISO_ROWS = (["mean_xyz"] * 3 + ["mean_t"] + ["log_scale"] * 2 + ["velocity"] * 3 + ["opacity"]
            + ["rgb"] * 3)


def to_iso(params: torch.Tensor) -> torch.Tensor:
    """Isotropic, motion-aware parameters [13, n] from rotor-form ones with
    identity rotors and one spatial scale (the heuristic initialisation):
    the same model, at zero velocity."""
    p = params
    return torch.cat([p[0:4], p[4:5], p[7:8], torch.zeros_like(p[0:3]), p[16:17], p[17:20]],
                     dim=0).contiguous()


def adam_config(budget: int, lrs=None, iso: bool = False, rows=None) -> G.gs4d_adam_cfg:
    lrs = dict(LR_DEFAULTS, **(lrs or {}))
    if rows is None:
        rows = ISO_ROWS if iso else ROTOR_ROWS
    cfg = G.gs4d_adam_cfg()
    for k, name in enumerate(rows):
        cfg.lr0[k], cfg.lr1[k] = lrs[name]
    cfg.budget, cfg.rows = int(budget), len(rows)
    cfg.beta1, cfg.beta2, cfg.eps = 0.9, 0.999, 1e-15
    return cfg


def _capture(fn, stream):
    """fn's launches on `stream`, captured as one HIP graph."""
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        fn()
    return g


class Trainer:
    """Single-view training on a fixed set of frames (views [F, 23],
    targets [F, 3, H, W] on the device).  Parameters in rotor form [20, N] or
    in the isotropic, motion-aware form [13, N] (chosen by their rows).
    With sch (a gs4d_sch), rotor-form parameters take their colour from
    sphericylindrical-harmonic coefficients (self.coef [3 K, N], started
    from the parameters' RGB by gs4d_sch_from_rgb and trained with them;
    rows 17-19 of the parameters are then unused)."""

    def __init__(self, params: torch.Tensor, views, targets: torch.Tensor, budget: int = 5000,
                 ssim_weight: float = 0.2, pair_capacity: int | None = None, lrs=None,
                 batch: int = 256, sch=None):
        self.params = params.contiguous()
        dev = self.params.device
        self.n = self.params.shape[1]
        self.views = np.atleast_2d(views)
        self.cviews = [G.make_views(v) for v in self.views]
        self.targets = targets
        self.F = self.views.shape[0]
        self.rast = Rasterizer(self.n, self.views[0], device=dev, pair_capacity=pair_capacity,
                               batch=batch)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=dev)
        self.iso = self.params.shape[0] == G.ISO_FIELDS
        self.cfg = adam_config(budget, lrs, iso=self.iso)
        # parameter gradients (the rasterizer's buffer holds the rotor form's)
        self.dparams = torch.zeros_like(self.params) if self.iso else self.rast.dparams
        self.ssim_w = float(ssim_weight)
        H, W = self.rast.H, self.rast.W
        self.dimg = torch.zeros((1, 3, H, W), device=dev)
        self.loss = torch.zeros(1, device=dev)
        self.ssim_ws = torch.zeros(G.gs4d_photometric_loss_workspace_size(1, 3, H, W),
                                   dtype=torch.uint8, device=dev)
        self.overflow_seen = torch.zeros(1, dtype=torch.int32, device=dev)
        self.sch = sch
        if sch is not None:
            assert not self.iso, "the SCH colour is built on the rotor form"
            rows = G.gs4d_sch_rows(sch.degree, sch.n_freq)
            self.coef = torch.empty((rows, self.n), device=dev)
            G.gs4d_sch_from_rgb(self.params[17:20], sch, self.coef)
            self.dcoef = torch.zeros_like(self.coef)
            self.cm = torch.zeros_like(self.coef)
            self.cv = torch.zeros_like(self.coef)
            # two Adam groups of one row each: the constant coefficients
            # (3 N values) and the higher ones, each with its own step count
            self.coef_groups = [(sl, adam_config(budget, lrs, rows=[name]),
                                 torch.zeros(1, dtype=torch.int32, device=dev))
                                for sl, name in ((slice(0, 3), "sch_dc"),
                                                 (slice(3, rows), "sch_rest"))
                                if sl.stop > sl.start]
            self.rast.set_sch(sch, self.coef)

    def size_pairs(self, frames=None, margin=1.5):
        """Measure the pair count over some frames and size the pair buffers."""
        frames = range(self.F) if frames is None else frames
        peak = 0
        for f in frames:
            self.rast.set_views(self.cviews[f])
            self.rast.preprocess(self.params)
            self.rast.bin_sort(check=True)
            peak = max(peak, int(self.rast.n_pairs.item()))
        cap = int(peak * margin) + 4096
        if cap > self.rast.capacity:
            self.rast._alloc_pairs(cap)
        return peak

    def forward_loss(self, f: int):
        r = self.rast
        r.set_views(self.cviews[f])
        r.preprocess(self.params)
        r.bin_sort(check=False)
        r.render()
        target = self.targets[f:f + 1]
        G.gs4d_photometric_loss(r.image, target, 1.0, self.ssim_w, self.loss, self.dimg,
                                self.ssim_ws)

    def stage_forward(self, f: int):
        self.forward_loss(f)
        torch.maximum(self.overflow_seen, self.rast.overflow, out=self.overflow_seen)
        # the render backward's accumulator, cleared here so that the
        # backward stage is the backward kernel alone
        self.rast.zero_grad2d()

    def stage_render_bwd(self, f: int):
        self.rast.render_bwd_2d(self.dimg, pre_zeroed=True)

    def stage_update(self, f: int):
        r = self.rast
        if self.sch is not None:
            G.gs4d_preprocess_sch_bwd(self.params, self.coef, self.sch, r.touched, r.grad2d,
                                      self.cviews[f], self.dparams, self.dcoef)
            for sl, cfg, step in self.coef_groups:
                flat = lambda t: t[sl].view(1, -1)
                G.gs4d_adam_step(flat(self.coef), flat(self.dcoef), flat(self.cm), flat(self.cv),
                                 cfg, step)
        else:
            bwd = G.gs4d_preprocess_iso_bwd if self.iso else G.gs4d_preprocess_bwd
            bwd(self.params, r.touched, r.grad2d, self.cviews[f], self.dparams)
        G.gs4d_adam_step(self.params, self.dparams, self.m, self.v, self.cfg, self.step_dev)

    def step(self, f: int):
        self.stage_forward(f)
        self.stage_render_bwd(f)
        self.stage_update(f)

    # ------------------------------------------------------------ graphs
    def capture(self, frames):
        """Capture each frame's step as one HIP graph, and again as three:
        [preprocess, bin/sort, render, loss], [render backward], [preprocess
        backward, Adam], so that a caller can time the render backward with
        events between replays.  Every buffer is preallocated, so replays
        allocate nothing."""
        self.graphs = {}
        self.whole = {}
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        for f in frames:
            self.whole[f] = _capture(lambda: self.step(f), side)
            self.graphs[f] = [_capture(lambda st=stage: st(f), side)
                              for stage in (self.stage_forward, self.stage_render_bwd,
                                            self.stage_update)]
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()

    def step_graph(self, f: int, events=None):
        """Replay frame f's captured step; with events=(a, b), a and b are
        recorded around the render backward (three graphs), else the step is
        one graph."""
        if events is None:
            self.whole[f].replay()
            return
        g0, g1, g2 = self.graphs[f]
        g0.replay()
        events[0].record()
        g1.replay()
        events[1].record()
        g2.replay()

    def loss_value(self) -> float:
        """L1 + w (1 - SSIM) of the last forward (synchronises)."""
        return float(self.loss.item())

    def psnr(self, frames) -> float:
        """Mean PSNR over frames (synchronises)."""
        r = self.rast
        sse = torch.zeros(1, dtype=torch.float64, device=self.params.device)
        vals = []
        for f in frames:
            r.set_views(self.cviews[f])
            r.forward(self.params, check=True)
            G.gs4d_fill_f32(sse.view(torch.float32), 0.0)
            G.gs4d_sse(r.image, self.targets[f:f + 1], sse)
            mse = float(sse.item()) / r.image.numel()
            vals.append(-10.0 * math.log10(max(mse, 1e-20)))
        return float(np.mean(vals))


class BatchedTrainer:
    """All views in every launch: one preprocess over (view, Gaussian), one
    sort over view-major tiles, persistent render forward (largest tiles
    first) with the per-view L1 loss and its gradient reduced in-kernel,
    persistent render backward, preprocess backward summed over views, Adam.
    targets: [V, 3, H, W] on the device."""

    def __init__(self, params: torch.Tensor, views, targets: torch.Tensor, budget: int = 5000,
                 pair_capacity: int | None = None, lrs=None, batch: int = 256,
                 persistent: bool = True, n_workgroups: int = 0):
        self.params = params.contiguous()
        dev = self.params.device
        self.n = self.params.shape[1]
        self.views = np.atleast_2d(views)
        self.V = self.views.shape[0]
        self.rast = Rasterizer(self.n, self.views, device=dev, pair_capacity=pair_capacity,
                               batch=batch, persistent=persistent, n_workgroups=n_workgroups)
        self.targets = targets.contiguous()
        self.rast.set_target(self.targets, 1.0)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=dev)
        self.cfg = adam_config(budget, lrs)
        self.overflow_seen = torch.zeros(1, dtype=torch.int32, device=dev)
        self.graphs = None

    def size_pairs(self, margin=1.5):
        self.rast.preprocess(self.params)
        self.rast.bin_sort(check=True)
        peak = int(self.rast.n_pairs.item())
        cap = int(peak * margin) + 4096
        if cap > self.rast.capacity:
            self.rast._alloc_pairs(cap)
        return peak

    def stage_forward(self):
        r = self.rast
        r.preprocess(self.params)
        r.bin_sort(check=False)
        r.render()
        torch.maximum(self.overflow_seen, r.overflow, out=self.overflow_seen)
        r.zero_grad2d()

    def stage_render_bwd(self):
        r = self.rast
        r.render_bwd_2d(r.dL_dimage, pre_zeroed=True)

    def stage_update(self):
        r = self.rast
        G.gs4d_preprocess_bwd(self.params, r.touched, r.grad2d, r.cviews, r.dparams)
        G.gs4d_adam_step(self.params, r.dparams, self.m, self.v, self.cfg, self.step_dev)

    def stage_backward(self):
        self.stage_render_bwd()
        self.stage_update()

    def step(self):
        self.stage_forward()
        self.stage_backward()

    def capture(self):
        """The step as one HIP graph, and again as three ([forward + fused
        loss], [render backward], [preprocess backward + Adam]) so that the
        render backward can be timed with events between replays."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        self.whole = _capture(self.step, side)
        self.graphs = [_capture(stage, side)
                       for stage in (self.stage_forward, self.stage_render_bwd, self.stage_update)]
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()

    def step_graph(self, events=None):
        if events is None:
            self.whole.replay()
            return
        g0, g1, g2 = self.graphs
        g0.replay()
        events[0].record()
        g1.replay()
        events[1].record()
        g2.replay()

    def loss_per_view(self):
        return self.rast.loss_per_view.detach().cpu().numpy()
