"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only draws random numbers and builds camera matrices; it holds
none of the rasterizer's arithmetic.  Every float it hands out is rounded to
FP32 first, so that the CPU oracle (which reads FP64 views) and the GPU path
(which reads FP32 views) see identical values.

Parameter layout: ``params`` is float32 ``[20, N]`` (one plane per field):
  0..3   mean (x, y, z, t)
  4..7   log scale (x, y, z, t)
  8..11  left unit quaternion (w, x, y, z)    (normalised on use)
  12..15 right unit quaternion (w, x, y, z)   (normalised on use)
  16     opacity logit
  17..19 rgb

View layout: float64 ``[23]`` (FP32-representable values):
  0..11 world-to-camera [R | t], row-major 3x4, camera axes x right, y down,
        z forward; 12 fx; 13 fy; 14 cx; 15 cy; 16 width; 17 height;
  18 render time t; 19 near plane; 20..22 background rgb.
"""
from __future__ import annotations

import numpy as np

N_FIELDS = 20
VIEW_LEN = 23


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def make_view(Rt, fx, fy, cx, cy, width, height, t, near=0.2, bg=(0.0, 0.0, 0.0)):
    v = np.zeros(VIEW_LEN, dtype=np.float64)
    v[0:12] = _f32(np.asarray(Rt, dtype=np.float64).reshape(12))
    v[12:16] = _f32([fx, fy, cx, cy])
    v[16] = int(width)
    v[17] = int(height)
    v[18] = _f32(t)
    v[19] = _f32(near)
    v[20:23] = _f32(bg)
    return v


def look_at(eye, target, up=(0.0, 1.0, 0.0)):
    """World-to-camera [R|t] (3x4) for a camera at ``eye`` looking at ``target``.

    Camera axes: x right, y down, z forward (towards the target)."""
    eye = np.asarray(eye, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    up = np.asarray(up, dtype=np.float64)
    zc = target - eye
    zc /= np.linalg.norm(zc)
    xc = np.cross(zc, up)
    if np.linalg.norm(xc) < 1e-9:
        xc = np.cross(zc, np.array([1.0, 0.0, 0.0]))
    xc /= np.linalg.norm(xc)
    yc = np.cross(zc, xc)
    R = np.stack([xc, yc, zc], axis=0)
    t = -R @ eye
    return np.concatenate([R, t[:, None]], axis=1)


def front_view(width=64, height=64, f=64.0, dist=3.0, t=0.5, near=0.2, bg=(0.0, 0.0, 0.0)):
    """Camera with identity rotation at distance ``dist`` in front of the origin."""
    Rt = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, dist]], dtype=np.float64)
    return make_view(Rt, f, f, width / 2.0, height / 2.0, width, height, t, near, bg)


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def small_set(n=2000, seed=0, log_s_xyz=(-3.0, 0.5), log_s_t=(-2.0, 0.5)):
    """The 2,000-Gaussian plain single-view set: means uniform in [-1,1]^3 x
    t in [0,1]; log scales N(-3, 0.5) (xyz, independent per axis) and
    N(-2, 0.5) (t); two random unit quaternions; opacity logit N(0,1);
    rgb U(0,1)."""
    rng = np.random.default_rng(seed)
    p = np.zeros((N_FIELDS, n), dtype=np.float64)
    p[0:3] = rng.uniform(-1.0, 1.0, (3, n))
    p[3] = rng.uniform(0.0, 1.0, n)
    p[4:7] = rng.normal(log_s_xyz[0], log_s_xyz[1], (3, n))
    p[7] = rng.normal(log_s_t[0], log_s_t[1], n)
    p[8:12] = _unit_quats(rng, n)
    p[12:16] = _unit_quats(rng, n)
    p[16] = rng.normal(0.0, 1.0, n)
    p[17:20] = rng.uniform(0.0, 1.0, (3, n))
    return p.astype(np.float32)


def perturb(params, seed=1):
    """Seeded perturbation used to make an L1 target from a copy of a set."""
    rng = np.random.default_rng(seed)
    p = params.astype(np.float64).copy()
    n = p.shape[1]
    p[0:4] += rng.normal(0.0, 0.02, (4, n))
    p[4:8] += rng.normal(0.0, 0.1, (4, n))
    p[8:16] += rng.normal(0.0, 0.05, (8, n))
    p[16] += rng.normal(0.0, 0.2, n)
    p[17:20] = np.clip(p[17:20] + rng.normal(0.0, 0.05, (3, n)), 0.0, 1.0)
    return p.astype(np.float32)


def clustered_set(n=1_000_000, seed=4, n_blobs=20, blob_sigma=0.1, shell=(4.0, 5.0),
                  frac_blobs=0.8):
    """Means clustered as Gaussian blobs plus a uniform background shell;
    the other attributes are drawn as in :func:`small_set`."""
    rng = np.random.default_rng(seed)
    p = small_set(n, seed + 1000).astype(np.float64)
    nb = int(round(frac_blobs * n))
    centres = rng.uniform(-1.0, 1.0, (n_blobs, 3))
    which = rng.integers(0, n_blobs, nb)
    p[0:3, :nb] = (centres[which] + rng.normal(0.0, blob_sigma, (nb, 3))).T
    ns = n - nb
    d = rng.standard_normal((3, ns))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    r = rng.uniform(shell[0], shell[1], ns)
    p[0:3, nb:] = d * r
    return p.astype(np.float32)


def linear_loss_weights(n_views, height, width, seed=7):
    """Random upstream gradient dL/dimage for a linear loss sum(w * C)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (n_views, 3, height, width)).astype(np.float32)


def batched_set(n=500_000, seed=3, frac_dynamic=0.2, rotations="motion"):
    """Many-view set.  Means uniform in [-1,1]^3 x [0,1]; spatial log scales
    N(-5, 0.5) per axis (the views zoom in, so splats stay a few pixels);
    opacity logit N(0,1); rgb U(0,1).

    rotations="motion": the structure of the paper's motion-aware model
    (Sec. 3.3): a static majority with identity orientation (no space-time
    coupling) and a long temporal scale (log s_t ~ N(0.5, 0.3)), and a
    dynamic part that lives briefly (log s_t ~ N(-2.5, 0.3)) and moves
    (rotors within ~0.1 rad of identity, so the velocity a/c is ~0.1 per
    unit time).

    rotations="random": the 2,000-Gaussian set's shapes -- two random unit
    quaternions (a random 4D rotation) per Gaussian, log s_t ~ N(0, 0.3),
    so s_t is ~150 times s_xyz and the conditional covariance is the
    ill-conditioned difference of two large blocks."""
    rng = np.random.default_rng(seed)
    if rotations == "random":
        p = small_set(n, seed, log_s_xyz=(-5.0, 0.5)).astype(np.float64)
        p[7] = np.random.default_rng(seed + 7).normal(0.0, 0.3, n)
        return p.astype(np.float32)
    if rotations != "motion":
        raise ValueError(rotations)
    p = np.zeros((N_FIELDS, n), dtype=np.float64)
    p[0:3] = rng.uniform(-1.0, 1.0, (3, n))
    p[3] = rng.uniform(0.0, 1.0, n)
    p[4:7] = rng.normal(-5.0, 0.5, (3, n))
    dyn = rng.uniform(0.0, 1.0, n) < frac_dynamic
    p[7] = np.where(dyn, rng.normal(-2.5, 0.3, n), rng.normal(0.5, 0.3, n))
    for base in (8, 12):
        q = np.zeros((4, n))
        q[0] = 1.0
        q[1:4] = np.where(dyn, rng.normal(0.0, 0.05, (3, n)), 0.0)
        p[base:base + 4] = q / np.linalg.norm(q, axis=0, keepdims=True)
    p[16] = rng.normal(0.0, 1.0, n)
    p[17:20] = rng.uniform(0.0, 1.0, (3, n))
    return p.astype(np.float32)


def frustum_count(params, view):
    """Number of Gaussian means inside a view's image and in front of its
    near plane (plain pinhole geometry; used to pick camera intrinsics)."""
    Rt = np.asarray(view[:12]).reshape(3, 4)
    X = Rt[:, :3] @ params[0:3].astype(np.float64) + Rt[:, 3:4]
    z = X[2]
    ok = z > view[19]
    u = view[12] * X[0] / np.where(ok, z, 1.0) + view[14]
    v = view[13] * X[1] / np.where(ok, z, 1.0) + view[15]
    ok &= (u >= 0) & (u < view[16]) & (v >= 0) & (v < view[17])
    return int(ok.sum())


def batched_views(params, targets=(57_000, 115_000, 175_000, 235_000, 295_000, 355_000, 410_000,
                                   460_000), width=960, height=540, dist=3.0, seed=5):
    """One camera per target count, around the set at distance `dist`, time
    t spread over [0.1, 0.9]; each focal length is bisected until the view
    frustum holds about `target` Gaussian means."""
    rng = np.random.default_rng(seed)
    views = []
    for i, target in enumerate(targets):
        a = 2 * np.pi * i / len(targets) + rng.uniform(-0.2, 0.2)
        eye = dist * np.array([np.sin(a), rng.uniform(-0.3, 0.3), -np.cos(a)])
        Rt = look_at(eye, (0.0, 0.0, 0.0), up=(0.0, -1.0, 0.0))
        t = 0.1 + 0.8 * i / max(len(targets) - 1, 1)
        lo, hi = 50.0, 20000.0          # focal length bracket (pixels)
        for _ in range(40):
            f = np.sqrt(lo * hi)
            v = make_view(Rt, f, f, width / 2, height / 2, width, height, t)
            if frustum_count(params, v) > target:
                lo = f
            else:
                hi = f
        views.append(make_view(Rt, np.sqrt(lo * hi), np.sqrt(lo * hi), width / 2, height / 2,
                               width, height, t))
    return np.stack(views)
