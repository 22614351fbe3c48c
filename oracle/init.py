"""TEST INFRASTRUCTURE: oracle of the scene preparation around grid pruning
(plain numpy, FP64).  Only tests, the smoke check and the benchmark's CPU
baseline may import it; it shares no code with the HIP path.

* back projection on consistent depth (Sec. 3.2, back-projection equation):
  X = G o pi^-1(p, D, K^-1) -- the pixel centre p = (x + 1/2, y + 1/2) at
  depth D through the inverse intrinsics into the camera frame, then the
  camera-to-world transform (the inverse of the view's world-to-camera
  [R | t]);
* the heuristic initialisation of Sec. 4.1: temporal scale 2/fps for dynamic
  points and the whole video for static ones (time normalised to [0, 1], so
  2 / frames and 1), position, time and colour from the pruned points,
  identity rotation; the spatial scale is the voxel edge of the point's
  class, or the footprint D / f of one back-projected pixel for a class that
  is not pruned, and the opacity 0.1 (readings: the paper inherits both from
  its baseline without values).
"""
from __future__ import annotations

import numpy as np

OPACITY0 = 0.1


def backproject(depth_acc, cover, view, min_cover=0.5):
    """Points of the pixels with cover > min_cover, in row-major pixel order:
    (xyz [3, m], depth [m], pixel index [m] = y W + x), FP64.  D is the
    alpha-weighted depth depth_acc / cover."""
    view = np.asarray(view, np.float64)
    W, H = int(view[16]), int(view[17])
    R = view[:12].reshape(3, 4)[:, :3]
    t = view[:12].reshape(3, 4)[:, 3]
    fx, fy, cx, cy = view[12:16]
    cov = np.asarray(cover, np.float64).reshape(H * W)
    acc = np.asarray(depth_acc, np.float64).reshape(H * W)
    pix = np.nonzero(cov > min_cover)[0]
    D = acc[pix] / cov[pix]
    y, x = np.divmod(pix, W)
    # pi^-1: the homogeneous pixel through K^-1, scaled by the depth
    K = np.array([[fx, 0.0, cx], [0.0, fy, cy], [0.0, 0.0, 1.0]])
    ph = np.stack([x + 0.5, y + 0.5, np.ones_like(D)])
    xc = np.linalg.solve(K, ph) * D
    # camera -> world: the inverse of x_cam = R X + t
    X = np.linalg.solve(R, xc - t[:, None])
    return X, D, pix.astype(np.int64)


def heuristic_init(xyz, rgb, t, dynamic, voxel_static, voxel_dynamic, frames, depth=None,
                   focal=None):
    """Rotor-form parameters [20, k] (FP64) of the pruned points."""
    xyz = np.asarray(xyz, np.float64)
    k = xyz.shape[1]
    dyn = np.zeros(k, bool) if dynamic is None else np.asarray(dynamic).astype(bool)
    p = np.zeros((20, k))
    p[0:3] = xyz
    p[3] = np.asarray(t, np.float64)
    scale = np.where(dyn, voxel_dynamic, voxel_static).astype(np.float64)
    unpruned = ~(scale > 0)
    if unpruned.any():
        scale = np.where(unpruned, np.asarray(depth, np.float64) / float(focal), scale)
    p[4:7] = np.log(scale)[None]
    p[7] = np.where(dyn, np.log(2.0 / frames), np.log(1.0))
    p[8] = 1.0
    p[12] = 1.0
    p[16] = np.log(OPACITY0 / (1.0 - OPACITY0))
    p[17:20] = np.asarray(rgb, np.float64)
    return p
