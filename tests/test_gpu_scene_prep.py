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
