"""Forward-only rendering at display sizes (the frame-rate path).

* a forward-only rasterizer (no T_final / last / gradient buffers) writes
  the same image bits as the training forward, and refuses a backward;
* FrameRenderer at 480x270 (a 960x540 camera rescaled): every frame's graph
  replay equals its eager launches bit for bit, and the image matches the
  oracle's compositing to 1e-4 except at pixels next to an alpha / clamp /
  transmittance threshold; three frames per launch give the same bits.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_01119_amd import synth
from paper_2510_01119_amd.rasterizer import Rasterizer
from paper_2510_01119_amd.realtime import FrameRenderer, rescale_view

from gpu_helpers import check_image, decision_bounds, gpu_forward, need_gpu

pytestmark = pytest.mark.gpu


def test_forward_only_image_equals_training_forward():
    need_gpu()
    p = synth.small_set(2000, 0)
    view = synth.front_view(64, 64, 64.0)
    r1, P = gpu_forward(p, view)
    r2 = Rasterizer(2000, view, forward_only=True)
    r2.forward(P)
    torch.cuda.synchronize()
    assert r2.T_final is None and r2.last is None
    assert torch.equal(r1.image, r2.image)
    with pytest.raises(RuntimeError):
        r2.render_bwd_2d(torch.zeros_like(r2.image))


def test_frame_renderer_display_size():
    need_gpu()
    p = synth.small_set(6000, 5, log_s_xyz=(-3.5, 0.5))
    base = [synth.front_view(960, 540, 800.0, 3.0, t) for t in (0.25, 0.5, 0.75)]
    views = np.stack([rescale_view(v, 480, 270) for v in base])
    P = torch.from_numpy(p).cuda()
    fr = FrameRenderer(P, views)
    fr.capture()
    for f in range(len(views)):
        fr.replay(f)
        torch.cuda.synchronize()
        img = fr.image.clone()
        fr.render(f)
        torch.cuda.synchronize()
        assert torch.equal(img, fr.image)
        o = oracle.forward(p, views[f], "f32")
        flag, img_b, _, _ = decision_bounds(p, views[f][None], o["rec"].astype(np.float64),
                                            o["vals"], o["ranges"], np.zeros((1, 3, 270, 480)))
        check_image(f"frame renderer 480x270 frame {f}", img.cpu().numpy(), o["image"], flag, img_b)
    rate = fr.frame_rate(frames=30, warmup=3)
    assert rate["fps"] > 0 and rate["peak_pairs"] > 0
    # three frames per launch: the same image bits as one frame per launch
    fr3 = FrameRenderer(P, views, frames_per_launch=3)
    fr3.capture()
    fr3.replay(0)
    torch.cuda.synchronize()
    for f in range(len(views)):
        fr.render(f)
        torch.cuda.synchronize()
        assert torch.equal(fr3.image[f], fr.image[0])
