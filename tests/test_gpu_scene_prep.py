"""Upstream of pruning, the paper's way (Sec. 3.2), on a small synthetic
scene: the Otsu split of the (noisy, 8x8-averaged, upsampled) motion
probability map recovers the ground-truth motion mask (mean IoU >= 0.75 over
frames), the recorded scene scale equals the mean over frames of each
frame's mean back-projected depth over the focal length, and the adaptive
voxel edges lambda (1/N) sum_i mean(D_i) / f prune the cloud."""
import numpy as np
import pytest
import torch

from paper_2510_01119_amd.scene import Scene

from gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu


def test_otsu_mask_and_adaptive_voxel():
    need_gpu()
    sc = Scene(seed=3, n_gt=200_000, frames=12, width=480, height=270, focal=400.0)
    images, cloud = sc.render_ground_truth(motion="otsu")
    xyz, attr, cls = cloud
    assert sc.mask_iou is not None and sc.mask_iou >= 0.75, sc.mask_iou
    t, d = attr[3].double().cpu().numpy(), attr[4].double().cpu().numpy()
    ref = float(np.mean([d[t == u].mean() for u in np.unique(t)])) / 400.0
    assert abs(sc.depth_over_f - ref) <= 1e-5 * ref
    assert 0 < int(cls.sum().item()) < cls.numel()
    vs, vd = 4.0 * sc.depth_over_f, 4.0 * sc.depth_over_f
    pxyz, pattr, dyn, count = sc.prune(cloud, vs, voxel_dynamic=vd)
    assert 0 < pxyz.shape[1] < xyz.shape[1] // 5
    assert int(count.sum().item()) == xyz.shape[1]
    assert 0 < int(dyn.sum().item()) < pxyz.shape[1]


def test_lite_and_full_presets():
    """The paper's two settings (Sec. 4.1) on one small scene: Lite prunes
    both classes at 4 mean(D / f); Full prunes static points at 1 mean(D / f)
    and keeps every dynamic point as its own Gaussian, whose spatial scale is
    then the footprint of its pixel (depth / f)."""
    need_gpu()
    from paper_2510_01119_amd.scene import build_scene
    out = {}
    for preset in ("lite", "full"):
        sc, _, params, info, pruned = build_scene(seed=3, n_gt=200_000, frames=12, width=480,
                                                  height=270, preset=preset, keep_pruned=True)
        out[preset] = (sc, params, info, pruned)
    (sl, pl, il, _), (sf, pf, inf, (fxyz, fattr, fdyn, fcount)) = out["lite"], out["full"]
    assert sl.depth_over_f == sf.depth_over_f and il["mask_iou"] == inf["mask_iou"]
    assert il["voxel_static"] == pytest.approx(4.0 * sl.depth_over_f, rel=1e-6)
    assert il["voxel_dynamic"] == pytest.approx(4.0 * sl.depth_over_f, rel=1e-6)
    assert inf["voxel_static"] == pytest.approx(sf.depth_over_f, rel=1e-6)
    assert inf["voxel_dynamic"] == 0.0
    assert torch.all(fcount[fdyn] == 1)
    assert inf["n_dynamic"] > 4 * il["n_dynamic"] and inf["n_gaussians"] > il["n_gaussians"]
    # unpruned dynamic points: spatial log-scale = log(depth / f); pruned
    # static ones: the voxel edge
    d = fdyn.cpu().numpy()
    ls = pf[4].double().cpu().numpy()
    depth = fattr[4].double().cpu().numpy()
    assert np.allclose(ls[d], np.log(depth[d] / sf.f), atol=1e-5)
    assert np.allclose(ls[~d], np.log(inf["voxel_static"]), atol=1e-5)
    assert torch.isfinite(pl).all() and torch.isfinite(pf).all()


def test_pseudo_frames_repair_the_sequence_ends():
    """The sliding-window motion maps see half a window at the first and
    last frames, whose moving objects then fall below the sequence's Otsu
    threshold; pseudo-frames at both ends (Sec. 3.2) restore them, and the
    interior frames stay as they were."""
    need_gpu()
    ious = {}
    for pf in (False, True):
        sc = Scene(seed=3, n_gt=200_000, frames=12, width=480, height=270, focal=400.0)
        sc.render_ground_truth(motion="otsu", pseudo_frames=pf)
        ious[pf] = np.array(sc.mask_iou_frames)
        del sc
        torch.cuda.empty_cache()
    ends = [0, len(ious[True]) - 1]
    print(f"mask IoU per frame without pseudo-frames {np.round(ious[False], 3).tolist()}, "
          f"with {np.round(ious[True], 3).tolist()}", flush=True)
    assert ious[True][ends].min() >= 0.75
    assert ious[True][ends].mean() >= ious[False][ends].mean() + 0.1
    assert abs(ious[True][2:-2].mean() - ious[False][2:-2].mean()) <= 0.05
