"""Device-buffer management around the C ABI, and the autograd Function.

``Rasterizer`` owns every buffer one rasterization needs (records, pairs,
workspaces, image, per-pixel state) so that a training step allocates
nothing; torch provides the memory and the stream only.  The per-pixel
state the backward needs (T_final and the last blended entry) is kept, the
per-entry transmittance is recomputed by the backward kernel.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gs4d as G


class Rasterizer:
    """Buffers for rendering ``n`` Gaussians into ``views`` (numpy [V, 23]).
    With ``forward_only`` no per-pixel state or gradient buffer is kept (the
    forward then writes the image only; backward calls raise)."""

    def __init__(self, n: int, views, device="cuda", pair_capacity: int | None = None,
                 batch: int = 256, count_blends: bool = False, persistent: bool = False,
                 n_workgroups: int = 0, forward_only: bool = False):
        self.forward_only = bool(forward_only)
        self.device = torch.device(device)
        self.views_np = np.atleast_2d(np.asarray(views, dtype=np.float64))
        self.cviews = G.make_views(self.views_np)
        self.V = self.views_np.shape[0]
        self.W, self.H = int(self.views_np[0, 16]), int(self.views_np[0, 17])
        self.tiles_x, self.tiles_y = (self.W + 15) // 16, (self.H + 15) // 16
        self.n_tiles = self.V * self.tiles_x * self.tiles_y
        self.n = int(n)
        self.batch = batch
        dev = self.device
        V, H, W = self.V, self.H, self.W
        self.rec = torch.zeros((V, max(n, 1), G.REC_FLOATS), dtype=torch.float32, device=dev)
        self.rect = torch.zeros((V, max(n, 1), 4), dtype=torch.int32, device=dev)
        self.touched = torch.zeros((V, max(n, 1)), dtype=torch.int32, device=dev)
        self.ranges = torch.zeros((self.n_tiles, 2), dtype=torch.int32, device=dev)
        self.n_pairs = torch.zeros(1, dtype=torch.int64, device=dev)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=dev)
        self.image = torch.zeros((V, 3, H, W), dtype=torch.float32, device=dev)
        if self.forward_only:
            self.T_final = self.last = self.dparams = self.grad2d = None
        else:
            self.T_final = torch.zeros((V, H, W), dtype=torch.float32, device=dev)
            self.last = torch.zeros((V, H, W), dtype=torch.int32, device=dev)
            self.dparams = torch.zeros((G.N_FIELDS, max(n, 1)), dtype=torch.float32, device=dev)
            self.grad2d = torch.zeros((V, max(n, 1), G.GRAD2D_FLOATS), dtype=torch.float32,
                                      device=dev)
        self.counters = torch.zeros(3, dtype=torch.int64, device=dev) if count_blends else None
        # persistent launches: largest-first tile order + one work counter per kernel
        self.persistent = persistent
        self.order_tiles = True      # persistent: largest tiles first (else index order)
        self.n_workgroups = n_workgroups
        self.order = torch.zeros(self.n_tiles, dtype=torch.int32, device=dev)
        self.queues = torch.zeros(2, dtype=torch.int32, device=dev)
        self._bwd_queue_zeroed = False
        # persistent launches: fixed assignment of work-list positions instead
        # of a shared work counter
        self.static_schedule = False
        self.order_ws = torch.zeros(G.gs4d_tile_order_workspace_size(self.n_tiles), dtype=torch.uint8,
                                    device=dev)
        # fused per-view L1 (set_target)
        self.target = None
        self.l1_weight = 1.0
        self.loss_per_view = torch.zeros(V, dtype=torch.float32, device=dev)
        self.dL_dimage = (None if self.forward_only
                          else torch.zeros((V, 3, H, W), dtype=torch.float32, device=dev))
        # bumped by every forward: the state a backward reads belongs to the
        # latest forward only
        self.generation = 0
        # SCH appearance (set_sch): the colour comes from these coefficients
        self.sch = None
        self.coef = None
        self._alloc_pairs(pair_capacity if pair_capacity else max(1 << 16, 8 * n * V))

    def set_views(self, views):
        """Point the rasterizer at other views (same count and image size)."""
        if isinstance(views, __import__("ctypes").Array):
            assert len(views) == self.V
            self.cviews = views
            return
        v = np.atleast_2d(np.asarray(views, dtype=np.float64))
        assert v.shape[0] == self.V and int(v[0, 16]) == self.W and int(v[0, 17]) == self.H
        self.views_np = v
        self.cviews = G.make_views(v)

    def _alloc_pairs(self, cap: int):
        self.capacity = int(cap)
        dev = self.device
        self.keys = torch.zeros(self.capacity, dtype=torch.int64, device=dev)
        self.vals = torch.zeros(self.capacity, dtype=torch.int32, device=dev)
        ws = G.gs4d_bin_sort_workspace_size(self.n, self.V, self.capacity)
        self.ws = torch.zeros(ws, dtype=torch.uint8, device=dev)

    def set_sch(self, sch, coef):
        """Take the colour of rotor-form parameters from sphericylindrical-
        harmonic coefficients coef [3 K, n] (gs4d_preprocess_sch) instead of
        their rows 17-19; sch=None returns to the RGB colour."""
        if sch is not None:
            assert tuple(coef.shape) == (G.gs4d_sch_rows(sch.degree, sch.n_freq), self.n)
        self.sch, self.coef = sch, coef

    # ------------------------------------------------------------------ stages
    def preprocess(self, params: torch.Tensor):
        """Rotor-form parameters [20, n], or the isotropic, motion-aware form
        [13, n] (gs4d_preprocess_iso); the outputs are the same.  With
        set_sch, rotor-form parameters take their colour from the SCH
        coefficients."""
        if self.sch is not None:
            assert params.shape[0] == G.N_FIELDS
            G.gs4d_preprocess_sch(params, self.coef, self.sch, self.cviews, self.rec, self.rect,
                                  self.touched)
        elif params.shape[0] == G.ISO_FIELDS:
            G.gs4d_preprocess_iso(params, self.cviews, self.rec, self.rect, self.touched)
        else:
            G.gs4d_preprocess(params, self.cviews, self.rec, self.rect, self.touched)

    def bin_sort(self, check: bool = True):
        """Sort into tiles.  With ``check`` the host reads the pair count and
        grows the pair buffers (and re-sorts) if they overflowed."""
        while True:
            G.gs4d_bin_sort(self.rec, self.rect, self.touched, self.n, self.cviews, self.capacity,
                            self.keys, self.vals, self.ranges, self.n_pairs, self.overflow, self.ws)
            if not check:
                return
            if int(self.overflow.item()) == 0:
                return
            need = int(self.n_pairs.item())
            self._alloc_pairs(int(need * 1.25) + 1024)

    def set_target(self, target, l1_weight=1.0):
        """Fuse the per-view L1 loss into the forward: render() then also
        writes loss_per_view (zeroed first) and dL_dimage."""
        self.target = target
        self.l1_weight = float(l1_weight)

    def _opts(self, queue_index):
        o = G.gs4d_render_opts()
        o.batch = self.batch
        if self.persistent:
            o.persistent = 2 if self.static_schedule else 1
            o.n_workgroups = self.n_workgroups
            o.order = self.order.data_ptr() if self.order_tiles else 0
            o.queue = self.queues.data_ptr() + 4 * queue_index
        return o

    def tile_order(self):
        # also zeroes both work counters, so the next backward needs no reset
        G.gs4d_tile_order(self.ranges, self.order, self.queues, self.order_ws)
        self._bwd_queue_zeroed = True

    def _bwd_queue(self):
        """A zero work counter for a persistent backward: left zero by the tile
        ordering of the forward just before it, else reset here."""
        if not self._bwd_queue_zeroed:
            G.gs4d_fill_u32(self.queues[1:2], 0)
        self._bwd_queue_zeroed = False

    def render(self, opts=None):
        if opts is None:
            opts = self._opts(0)
            if self.persistent:
                if self.order_tiles:
                    self.tile_order()
                else:
                    G.gs4d_fill_u32(self.queues, 0)
                    self._bwd_queue_zeroed = True
        if self.counters is not None:
            G.gs4d_fill_u32(self.counters.view(torch.int32), 0)
            opts.counters = self.counters.data_ptr()
        if self.target is not None:
            G.gs4d_fill_f32(self.loss_per_view, 0.0)
            opts.target = self.target.data_ptr()
            opts.l1_weight = self.l1_weight
            opts.loss_per_view = self.loss_per_view.data_ptr()
            opts.dL_dimage = self.dL_dimage.data_ptr() if self.dL_dimage is not None else 0
        G.gs4d_render_fwd(self.rec, self.n, self.vals, self.ranges, self.cviews, self.image,
                          self.T_final, self.last, opts)

    def zero_grad2d(self):
        """Clear the 2D-gradient accumulator ahead of time: the next
        render_bwd_2d(pre_zeroed=True) then launches the backward kernel only."""
        G.gs4d_fill_f32(self.grad2d, 0.0)

    def render_bwd_2d(self, dL_dimage, pre_zeroed=False):
        if self.forward_only:
            raise RuntimeError("forward-only rasterizer: no state for a backward")
        if self.persistent:
            self._bwd_queue()
        opts = self._opts(1)
        if pre_zeroed:
            opts.flags = G.RENDER_GRAD2D_ZEROED
        G.gs4d_render_bwd_2d(self.rec, self.n, self.vals, self.ranges, self.cviews, dL_dimage,
                             self.T_final, self.last, self.grad2d, opts)

    def forward(self, params: torch.Tensor, check: bool = True, opts=None):
        assert params.shape in ((G.N_FIELDS, self.n), (G.ISO_FIELDS, self.n))
        assert params.dtype == torch.float32
        self.generation += 1
        self.preprocess(params)
        self.bin_sort(check)
        self.render(opts)
        return self.image

    def backward(self, params: torch.Tensor, dL_dimage: torch.Tensor):
        if self.forward_only:
            raise RuntimeError("forward-only rasterizer: no state for a backward")
        if params.shape[0] != G.N_FIELDS or self.sch is not None:
            raise ValueError("backward() takes rotor-form RGB parameters; for the isotropic "
                             "form or the SCH colour use render_bwd_2d and the form's "
                             "preprocess backward")
        if self.persistent:
            self._bwd_queue()
        G.gs4d_render_bwd(params, self.rec, self.touched, self.vals, self.ranges, self.cviews,
                          dL_dimage.contiguous(), self.T_final, self.last, self.dparams,
                          grad2d=self.grad2d, opts=self._opts(1))
        return self.dparams

    def pairs(self):
        P = int(self.n_pairs.item())
        return self.keys[:P], self.vals[:P]


class GS4DRasterize(torch.autograd.Function):
    """image = GS4DRasterize.apply(params [20, N], rasterizer).

    The backward runs gs4d_render_bwd on the state the forward left in the
    rasterizer's buffers; if another forward ran through the same rasterizer
    in between (its generation moved on), backward raises instead of
    returning gradients of the wrong state."""

    @staticmethod
    def forward(ctx, params, rast):
        rast.forward(params.detach().contiguous())
        ctx.rast = rast
        ctx.generation = rast.generation
        ctx.save_for_backward(params)
        return rast.image.clone()

    @staticmethod
    def backward(ctx, dimg):
        if ctx.rast.generation != ctx.generation:
            raise RuntimeError("GS4DRasterize.backward: the rasterizer ran another forward "
                               "after this one; its buffers no longer hold this forward's state")
        (params,) = ctx.saved_tensors
        d = ctx.rast.backward(params.detach().contiguous(), dimg.contiguous())
        return d.clone(), None
