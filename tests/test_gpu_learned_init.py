"""The learned initialisation end to end on held-out synthetic scenes
(seeds 900-902; the network was trained on scenes 100-189, its settings
chosen on 190-199 and 950-951):

* the rotor-form parameters it writes read back (gs4d_motion_of) as the
  network's predictions on the dynamic points, the static points keep the
  heuristic initialisation, and the rest of each column is the heuristic
  one;
* its gain: after the same fixed budget of batched steps (8 views per
  step) from the heuristic and from the learned initialisation, the
  learned one is ahead on the held-out frames of every scene, by a margin
  on average.
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
    assert model.meta.get("classes") == "dynamic"
    p = LI.apply(p0.clone(), pruned, model)
    feat = LI.features(pruned, model.shift, model.scale)
    pred = LI.predict(model, feat)
    back = LI.motion_targets(p)
    keep = [0, 1, 2, 3, 16, 17, 18, 19]
    assert torch.equal(p[keep], p0[keep])
    dyn = pruned[2]
    assert torch.equal(p[:, ~dyn], p0[:, ~dyn])
    assert torch.allclose(back[0, dyn], pred[0, dyn], atol=1e-3)
    assert torch.allclose(back[1:, dyn], pred[1:, dyn],
                          atol=1e-3 * (1 + float(pred[1:, dyn].abs().max())))
    assert bool(torch.isfinite(p).all())


def test_learned_init_gain(held_out):
    """Held-out PSNR after 300 batched steps of 8 views (rates x6 decayed to
    0.03x), learned against heuristic initialisation, on three scenes."""
    from paper_2510_01119_amd.pipeline import BATCHED_DECAY, BATCHED_LR_MULT
    gains = []
    for seed in (900, 901, 902):
        if seed == 900:
            sc, images, p0, pruned, model = held_out
        else:
            sc, images, p0, _, pruned = build_scene(seed=seed, keep_pruned=True)
            model = held_out[4]
        res = init_gain(sc, images, p0, pruned, model, budget=300, lr_mult=BATCHED_LR_MULT,
                        group=8, decay=BATCHED_DECAY)
        print(f"gain[{seed}]:", json.dumps(res), flush=True)
        gains.append(res["learned"]["psnr"][-1] - res["heuristic"]["psnr"][-1])
        del sc, images, p0, pruned
        torch.cuda.empty_cache()
    print(f"fixed-budget gains (dB): {np.round(gains, 3).tolist()}", flush=True)
    assert min(gains) > 0.0 and float(np.mean(gains)) >= 0.1, gains
