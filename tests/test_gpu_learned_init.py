"""The learned initialisation end to end on a held-out synthetic scene
(seed 900; the network was trained on scenes 100-199):

* the rotor-form parameters it writes read back (gs4d_motion_of) as the
  network's predictions, and the rest of each column is the heuristic one;
* its gain: after the same number of batched training steps from the
  heuristic and from the learned initialisation, the learned one is ahead
  on the held-out frames.
"""
import json

import numpy as np
import pytest
import torch

from paper_2510_01119_amd import learned_init as LI
from paper_2510_01119_amd.pipeline import init_gain
from paper_2510_01119_amd.scene import build_scene

from gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def held_out():
    need_gpu()
    sc, images, p0, info, pruned = build_scene(seed=900, keep_pruned=True)
    return sc, images, p0, pruned, LI.InitModel.load()


def test_apply_round_trip(held_out):
    sc, images, p0, pruned, model = held_out
    p = LI.apply(p0.clone(), pruned, model)
    feat = LI.features(pruned, model.shift, model.scale)
    pred = LI.predict(model, feat)
    back = LI.motion_targets(p)
    keep = [0, 1, 2, 3, 16, 17, 18, 19]
    assert torch.equal(p[keep], p0[keep])
    assert torch.allclose(back[0], pred[0], atol=1e-3)
    assert torch.allclose(back[1:], pred[1:], atol=1e-3 * (1 + float(pred[1:].abs().max())))
    assert bool(torch.isfinite(p).all())


def test_learned_init_gain(held_out):
    sc, images, p0, pruned, model = held_out
    res = init_gain(sc, images, p0, pruned, model, budget=150, lr_mult=2.0)
    print("gain:", json.dumps(res), flush=True)
    h, l = res["heuristic"]["psnr"], res["learned"]["psnr"]
    assert l[-1] > h[-1], (h, l)
