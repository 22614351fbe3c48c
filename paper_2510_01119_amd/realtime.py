"""Forward-only rendering at display resolutions, and its frame rate.

Novel views of a set of 4D Gaussians at a camera and a time t, rendered with
the same preprocess, binning and compositing kernels as training but with no
state kept for a backward (the paper compares methods by rendering speed in
frames per second at 480x270 and 854x480-class resolutions, Sec. 4 and its
efficiency tables).  Each frame's launches are captured once as a HIP graph
and replayed.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import gs4d as G
from .rasterizer import Rasterizer
from .train import _capture

# display sizes of the frame-rate benchmark (width, height)
DISPLAY_SIZES = ((480, 270), (854, 480), (860, 480))


def rescale_view(view, width: int, height: int) -> np.ndarray:
    """The same camera at another image size: the focal lengths and the
    principal point scale with the image (a pixel keeps its viewing ray up to
    the change of pixel pitch)."""
    v = np.array(view, dtype=np.float64, copy=True)
    sx, sy = width / float(v[16]), height / float(v[17])
    v[12:16] = np.float32(np.array([v[12] * sx, v[13] * sy, v[14] * sx, v[15] * sy]))
    v[16], v[17] = int(width), int(height)
    return v


class FrameRenderer:
    """Renders the frames of ``views`` (numpy [F, 23], one image size) of
    fixed parameters, forward only, on persistent largest-first launches.
    ``frames_per_launch`` consecutive frames share one launch of each kernel
    (the multi-view path: one preprocess, one sort over view-major tiles, one
    compositing launch), which fills the GPU at small image sizes at the
    cost of latency; F must be a multiple of it."""

    def __init__(self, params: torch.Tensor, views, margin: float = 1.3, batch: int = 256,
                 frames_per_launch: int = 1):
        self.params = params.contiguous()
        self.views = np.atleast_2d(views)
        B = int(frames_per_launch)
        assert B >= 1 and len(self.views) % B == 0
        self.B = B
        self.cviews = [G.make_views(self.views[i:i + B]) for i in range(0, len(self.views), B)]
        self.rast = Rasterizer(self.params.shape[1], self.views[0:B], device=self.params.device,
                               batch=batch, persistent=True, forward_only=True)
        # The parameters do not change, so each frame's pair count is fixed:
        # buffers sized from the measured peak cannot overflow on replay.
        peak = 0
        for cv in self.cviews:
            self.rast.set_views(cv)
            self.rast.preprocess(self.params)
            self.rast.bin_sort(check=True)
            peak = max(peak, int(self.rast.n_pairs.item()))
        cap = int(peak * margin) + 4096
        if cap > self.rast.capacity:
            self.rast._alloc_pairs(cap)
        self.peak_pairs = peak
        self.graphs = None

    @property
    def image(self) -> torch.Tensor:
        """[frames_per_launch, 3, H, W]: the last launch's frames."""
        return self.rast.image

    def render(self, f: int) -> torch.Tensor:
        """Launch f's frames (f * frames_per_launch ...), eager; the images
        land in ``self.image``."""
        r = self.rast
        r.set_views(self.cviews[f])
        r.preprocess(self.params)
        r.bin_sort(check=False)
        r.render()
        return r.image

    def capture(self):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        self.graphs = [_capture(lambda f=f: self.render(f), side) for f in range(len(self.cviews))]
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()

    def replay(self, f: int):
        self.graphs[f].replay()

    def frame_rate(self, frames: int = 200, warmup: int = 20) -> dict:
        """Frames per second over ``frames`` frames (graph replays cycling
        through the launches), bracketed by device synchronisations."""
        if self.graphs is None:
            self.capture()
        F = len(self.graphs)
        launches = max(1, frames // self.B)
        for k in range(warmup):
            self.replay(k % F)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(launches):
            self.replay(k % F)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n = launches * self.B
        return {"fps": round(n / dt, 1), "ms_per_frame": round(1e3 * dt / n, 4),
                "frames": n, "views": F * self.B, "frames_per_launch": self.B,
                "peak_pairs": self.peak_pairs}
