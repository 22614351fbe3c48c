"""Seeded synthetic dynamic scene at scene scale, built on the GPU.

Stand-in for the paper's video datasets (their frames, depth and camera
recovery are not available here).  Recipe:

* ground truth: about 1M Gaussians -- three textured background planes
  (back wall, floor, side wall; procedural checker/stripe/noise colours)
  and three rigid objects (ellipsoidal shells with striped colours) that
  move along Catmull-Rom spline trajectories while spinning;
* a smooth monocular camera path, fx = fy = 800 at 960x540, 200 frames with
  timestamps t_f = f / (frames - 1);
* each frame is rendered by this package's own rasterizer; a second pass
  with the colour channels replaced by (camera depth, 1, dynamic flag)
  gives the alpha-weighted depth, the coverage and a ground-truth motion
  mask;
* every pixel with coverage > 0.5 is back-projected (gs4d_backproject) to a
  world point with its colour, timestamp and motion class (Sec. 3.2, back
  projection), plus
  its depth and optical-flow magnitude (a further pass renders each
  ground-truth Gaussian's pixel displacement to the next frame: the stand-in
  for an optical-flow estimate), inputs of the learned initialisation;
* the motion class of a point is either the ground-truth mask or (motion =
  "otsu") the paper's segmentation: low-resolution motion-probability maps
  (motion_probability: a sliding-window stand-in for the SLAM's H/8 x W/8
  maps, with pseudo-frames at both ends of the sequence), bilinearly
  upsampled and split by one Otsu threshold over the whole sequence
  (gs4d_otsu_mask on the pooled maps, gs4d_threshold_mask per frame);
* the voxel edge is fixed, or (voxel = "adaptive") S_v = lambda (1/N) sum_i
  D_i / f with D_i the mean back-projected depth of frame i (Sec. 3.2), one
  lambda for static and one for dynamic points;
* gs4d_grid_prune merges the points per voxel (Sec. 3.2, grid pruning);
* the heuristic initialisation (Sec. 4.1, gs4d_heuristic_init): centroid
  position, mean timestamp and colour, temporal scale 2 / frames for
  dynamic points (two frame intervals, i.e. 2 / fps with time normalised to
  [0, 1]) and the whole video (1.0) for static ones, spatial scale = the
  voxel edge, opacity 0.1, identity rotors.
"""
from __future__ import annotations

import math
import sys

import numpy as np
import torch

from . import gs4d as G
from . import synth
from .rasterizer import Rasterizer


def _catmull_rom(P, u):
    """Closed Catmull-Rom spline through control points P [k, 3] at u in [0, 1)."""
    k = P.shape[0]
    x = u * k
    i = np.floor(x).astype(int)
    t = (x - i)[:, None]
    p0, p1, p2, p3 = (P[(i + d) % k] for d in (-1, 0, 1, 2))
    return 0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t ** 2
                  + (-p0 + 3 * p1 - 3 * p2 + p3) * t ** 3)


def pseudo_frame(j: int, frames: int) -> int:
    """The real frame that slot j of a sequence extended by pseudo-frames at
    both ends holds (Sec. 3.2, motion probability estimation): the
    extension mirrors the sequence about its first and last frame, so frame
    -d is frame d and frame (F-1)+d is frame (F-1)-d."""
    F = frames
    if F <= 1:
        return 0          # a single frame mirrors onto itself
    while j < 0 or j > F - 1:
        j = -j if j < 0 else 2 * (F - 1) - j
    return j


def motion_probability(dyn_low, window=2, noise=0.2, pseudo_frames=True, gen=None):
    """Stand-in for the SLAM's low-resolution motion-probability maps
    (dyn_low [F, h, w]: each frame's ground-truth dynamic fraction at H/8 x
    W/8), as a sliding-window estimator: frame i's map is the mean over its
    2 * window neighbour slots j = i-window..i+window (j != i) of a per-pair
    evidence clamp(s_i + noise * eps, 0, 1), with eps seeded N(0, 1), one
    draw per unordered pair of real frames.  A slot outside the sequence
    holds no evidence (0): the first and last frames see half a window, and
    their moving objects come out at half the interior's probability.  With
    pseudo_frames the sequence is first extended at both ends
    (pseudo_frame), so every slot holds a frame -- a pseudo-frame is a copy,
    so its pair repeats its mirror's evidence, and a slot holding a copy of
    frame i itself shows no motion (0) -- and the first and last frames'
    maps are on the interior's scale."""
    F = dyn_low.shape[0]
    dev = dyn_low.device
    if gen is None:
        gen = torch.Generator(device=dev)
        gen.manual_seed(0)
    # eps[a, d - 1]: the pair (a, a + d)
    eps = torch.randn((F, window) + tuple(dyn_low.shape[1:]), generator=gen, device=dev)
    out = torch.zeros_like(dyn_low)
    for i in range(F):
        acc = torch.zeros_like(dyn_low[i])
        for d in range(1, window + 1):
            for j in (i - d, i + d):
                if not 0 <= j < F:
                    if not pseudo_frames:
                        continue
                    j = pseudo_frame(j, F)
                if j == i:
                    continue
                a, b = min(i, j), max(i, j)
                acc += (dyn_low[i] + noise * eps[a, b - a - 1]).clamp(0.0, 1.0)
        out[i] = acc / (2 * window)
    return out


def _rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


class Scene:
    def __init__(self, seed=0, n_gt=1_000_000, frames=200, width=960, height=540, focal=800.0,
                 device="cuda", scale=0.195):
        self.seed, self.frames, self.W, self.H, self.f = seed, frames, width, height, focal
        # world scale of the whole scene (geometry, trajectories, camera path);
        # projection is scale-free, so the frames look alike at any scale,
        # while the number of occupied 0.01 voxels grows as scale^2
        self.scale = float(scale)
        self.device = torch.device(device)
        rng = np.random.default_rng(seed)
        n_obj = n_gt // 20            # three objects, 5% each
        n_planes = n_gt - 3 * n_obj
        self.static = self._apply_scale(self._planes(rng, n_planes))
        obj, self.obj_id = self._objects(rng, n_obj)
        self.obj_local = self._apply_scale(obj)
        # object trajectories: closed splines inside the room
        self.ctrl = [self.scale * np.stack([rng.uniform(-1.4, 1.4, 5), rng.uniform(-0.4, 0.9, 5),
                                            rng.uniform(0.0, 2.2, 5)], axis=1) for _ in range(3)]
        self.spin = rng.uniform(-3.0, 3.0, 3)
        self.cams = self._camera_path(rng)

    # ------------------------------------------------------------ geometry
    def _apply_scale(self, p):
        p = p.copy()
        p[0:3] *= self.scale
        p[4:7] += math.log(self.scale)
        return p

    def _planes(self, rng, n):
        # (normal axis, plane coordinate, extents of the two other axes)
        specs = [(2, 3.0, (-3.0, 3.0), (-2.2, 1.5)),    # back wall z = 3 (x, y)
                 (1, 1.5, (-3.0, 3.0), (-1.5, 3.0)),    # floor y = 1.5 (x, z)
                 (0, -3.0, (-2.2, 1.5), (-1.5, 3.0))]   # left wall x = -3 (y, z)
        areas = np.array([(a[1] - a[0]) * (b[1] - b[0]) for _, _, a, b in specs])
        counts = np.floor(n * areas / areas.sum()).astype(int)
        counts[0] += n - counts.sum()
        out = np.zeros((20, n))
        o = 0
        for (ax, c, ea, eb), m in zip(specs, counts):
            u = rng.uniform(ea[0], ea[1], m)
            v = rng.uniform(eb[0], eb[1], m)
            others = [k for k in range(3) if k != ax]
            xyz = np.zeros((3, m))
            xyz[ax] = c + rng.normal(0, 0.002, m)
            xyz[others[0]] = u
            xyz[others[1]] = v
            spacing = math.sqrt(areas[[s[0] for s in specs].index(ax)] / m)
            ls = np.full((3, m), math.log(1.2 * spacing))
            ls[ax] = math.log(0.15 * spacing)
            # procedural texture: checker x stripes x noise, tinted per plane
            chk = ((np.floor(u * 2.5) + np.floor(v * 2.5)) % 2)
            stripes = 0.5 + 0.5 * np.sin(7.0 * u + 3.0 * v)
            tint = rng.uniform(0.3, 1.0, 3)
            col = np.clip((0.35 + 0.4 * chk[None] + 0.25 * stripes[None]) * tint[:, None]
                          + rng.normal(0, 0.04, (3, m)), 0, 1)
            sl = slice(o, o + m)
            out[0:3, sl] = xyz
            out[3, sl] = 0.5
            out[4:7, sl] = ls
            out[7, sl] = math.log(100.0)          # static in time
            out[8, sl] = 1.0
            out[12, sl] = 1.0
            out[16, sl] = 3.0
            out[17:20, sl] = col
            o += m
        return out

    def _objects(self, rng, n_obj):
        locs, ids = [], []
        radii = [(0.35, 0.25, 0.3), (0.25, 0.4, 0.25), (0.3, 0.3, 0.2)]
        for k in range(3):
            d = rng.standard_normal((3, n_obj))
            d /= np.linalg.norm(d, axis=0, keepdims=True)
            r = np.array(radii[k])[:, None]
            xyz = d * r * (1 + rng.normal(0, 0.01, (1, n_obj)))
            base = rng.uniform(0.2, 1.0, 3)
            band = (np.floor((d[1] + 1) * 4) % 2)[None]
            col = np.clip(base[:, None] * (0.5 + 0.5 * band) + rng.normal(0, 0.03, (3, n_obj)), 0, 1)
            area = 4 * math.pi * np.mean(radii[k]) ** 2
            sp = math.sqrt(area / n_obj)
            p = np.zeros((20, n_obj))
            p[0:3] = xyz
            p[3] = 0.5
            p[4:7] = math.log(1.3 * sp)
            p[7] = math.log(100.0)
            p[8] = 1.0
            p[12] = 1.0
            p[16] = 3.0
            p[17:20] = col
            locs.append(p)
            ids.append(np.full(n_obj, k))
        return np.concatenate(locs, axis=1), np.concatenate(ids)

    def _camera_path(self, rng):
        cams = []
        for f in range(self.frames):
            u = f / max(self.frames - 1, 1)
            eye = self.scale * np.array([-0.8 + 1.6 * u, -0.3 + 0.15 * math.sin(2 * math.pi * u),
                                         -3.2 + 0.4 * u])
            target = self.scale * np.array([0.2 * math.sin(math.pi * u), 0.2, 1.2])
            Rt = synth.look_at(eye, target, up=(0.0, -1.0, 0.0))
            cams.append(synth.make_view(Rt, self.f, self.f, self.W / 2, self.H / 2, self.W, self.H, u))
        return np.stack(cams)

    def object_pose(self, k, t):
        pos = _catmull_rom(self.ctrl[k], np.array([t % 1.0]))[0]
        return _rot_y(self.spin[k] * t), pos

    def gt_params(self, t):
        """Ground-truth set at time t (objects moved rigidly), float32 [20, N] on the device."""
        if not hasattr(self, "_static_dev"):
            self._static_dev = torch.from_numpy(self.static.astype(np.float32)).to(self.device)
            self._obj_dev = torch.from_numpy(self.obj_local.astype(np.float32)).to(self.device)
            self._obj_sel = [torch.from_numpy(np.nonzero(self.obj_id == k)[0]).to(self.device)
                             for k in range(3)]
        obj = self._obj_dev.clone()
        for k in range(3):
            R, pos = self.object_pose(k, t)
            sel = self._obj_sel[k]
            Rd = torch.from_numpy(R.astype(np.float32)).to(self.device)
            pd = torch.from_numpy(pos.astype(np.float32)).to(self.device)
            obj[0:3, sel] = Rd @ self._obj_dev[0:3, sel] + pd[:, None]
        obj[3] = t
        return torch.cat([self._static_dev, obj], dim=1).contiguous()

    # ------------------------------------------------------------ synthesis
    def _flow(self, f):
        """Per ground-truth Gaussian, the pixel displacement of its centre
        from frame f to the next frame (from the previous one for the last
        frame): the optical-flow magnitude, camera and object motion
        together."""
        a, b = (f, f + 1) if f + 1 < self.frames else (f - 1, f)
        px = []
        for k in (a, b):
            v = self.cams[k]
            mu = self.gt_params(float(v[18]))[0:3]
            Rt = torch.from_numpy(v[:12].reshape(3, 4)).to(self.device).float()
            xc = Rt[:, :3] @ mu + Rt[:, 3:4]
            z = xc[2].clamp_min(1e-3)
            px.append(torch.stack([float(v[12]) * xc[0] / z + float(v[14]),
                                   float(v[13]) * xc[1] / z + float(v[15])]))
        return torch.linalg.norm(px[1] - px[0], dim=0)

    def render_ground_truth(self, verbose=False, motion="gt", motion_noise=0.2,
                            pseudo_frames=True, motion_window=2):
        """Renders every frame; returns (images [F,3,H,W] on device, point
        cloud (xyz [3,M], attr [6,M] = rgb, t, depth, optical-flow
        magnitude; cls [M]) on device).  Also records
        self.depth_over_f (the mean over frames of each frame's mean
        back-projected depth, over the focal length: S_v's scene scale)
        and, with motion="otsu", self.mask_iou_frames (per frame, the Otsu
        mask's intersection over union with the ground-truth mask on the
        back-projected pixels) and self.mask_iou (their mean)."""
        import torch.nn.functional as F
        dev = self.device
        n_back, ious = 0, []
        if motion == "otsu":
            otsu_ws = torch.zeros(G.gs4d_otsu_workspace_size(), dtype=torch.uint8, device=dev)
            otsu_mask = torch.zeros(self.H * self.W, dtype=torch.uint8, device=dev)
            otsu_thr = torch.zeros(1, device=dev)
            gen = torch.Generator(device=dev)
            gen.manual_seed(1000 + self.seed)
            lows, pixs, gt_dyns = [], [], []
        n = self.static.shape[1] + self.obj_local.shape[1]
        r = Rasterizer(n, self.cams[0], device=dev, pair_capacity=1 << 24)
        # back projection (gs4d_backproject): at most every pixel of a frame
        hw = self.H * self.W
        bp_xyz = torch.empty((3, hw), device=dev)
        bp_depth = torch.empty(hw, device=dev)
        bp_pix = torch.empty(hw, dtype=torch.int32, device=dev)
        bp_n = torch.zeros(1, dtype=torch.int64, device=dev)
        bp_sum = torch.zeros(1, dtype=torch.float64, device=dev)
        bp_ws = torch.empty(G.gs4d_backproject_workspace_size(hw), dtype=torch.uint8, device=dev)
        mean_depth = []
        dyn_flag = torch.zeros(n, device=dev)
        dyn_flag[self.static.shape[1]:] = 1.0
        images = torch.empty((self.frames, 3, self.H, self.W), device=dev)
        pts, attrs, clss = [], [], []
        for f in range(self.frames):
            view = self.cams[f]
            r.set_views(view)
            p = self.gt_params(float(view[18]))
            r.forward(p)
            images[f] = r.image[0]
            # second pass: (depth, coverage, dynamic) as colours
            rec = r.rec[0]
            rec[:, 8] = rec[:, 6]
            rec[:, 9] = (r.touched[0] > 0).float()
            rec[:, 10] = dyn_flag
            r.render()
            aux = r.image[0].clone()
            cov2 = aux[1]
            cov = cov2.reshape(-1)
            # back projection of the pixels with coverage > 0.5 (Sec. 3.2)
            G.gs4d_fill_f32(bp_sum.view(torch.float32), 0.0)
            G.gs4d_backproject(aux[0], aux[1], view, 0.5, hw, bp_xyz, bp_depth, bp_pix, bp_n, bp_ws,
                               depth_sum=bp_sum)
            m = int(bp_n.item())
            pix = bp_pix[:m].long()
            depth = bp_depth[:m]
            world = bp_xyz[:, :m].clone()
            mean_depth.append(float(bp_sum.item()) / max(m, 1))
            # third pass: optical-flow magnitude (pixels per frame) as a colour
            rec[:, 8] = self._flow(f)
            rec[:, 9] = 0.0
            rec[:, 10] = 0.0
            r.render()
            flow = r.image[0][0].reshape(-1)[pix] / cov[pix]
            pts.append(world)
            col = images[f].reshape(3, -1)[:, pix]
            attrs.append(torch.cat([col, torch.full((1, m), float(view[18]), device=dev),
                                    depth[None], flow[None]]))
            n_back += m
            gt_dyn = aux[2].reshape(-1)[pix] / cov[pix] > 0.5
            if motion == "otsu":
                # the class is decided once every frame's map is known
                frac = torch.where(cov2 > 0, aux[2] / cov2.clamp_min(1e-6), torch.zeros_like(cov2))
                lows.append(F.avg_pool2d(frac[None, None], 8, ceil_mode=True)[0, 0])
                pixs.append(bp_pix[:m].clone())
                gt_dyns.append(gt_dyn)
            else:
                clss.append(gt_dyn.to(torch.uint8))
            if verbose and f % 50 == 0:
                print(f"scene: frame {f}/{self.frames} pairs={int(r.n_pairs.item())}",
                      file=sys.stderr, flush=True)
        if motion == "otsu":
            # one Otsu threshold over the whole sequence's maps, applied to
            # each frame's bilinearly upsampled map
            low = motion_probability(torch.stack(lows), motion_window, motion_noise,
                                     pseudo_frames, gen).contiguous()
            G.gs4d_otsu_mask(low.reshape(-1), otsu_thr, None, otsu_ws)
            for f in range(self.frames):
                prob = F.interpolate(low[f][None, None], size=(self.H, self.W), mode="bilinear",
                                     align_corners=False)[0, 0].contiguous()
                G.gs4d_threshold_mask(prob, otsu_thr, otsu_mask)
                dyn = otsu_mask[pixs[f].long()].bool()
                gt_dyn = gt_dyns[f]
                inter = float((dyn & gt_dyn).sum().item())
                union = float((dyn | gt_dyn).sum().item())
                ious.append(inter / union if union > 0 else 1.0)
                clss.append(dyn.to(torch.uint8))
            del lows, pixs, gt_dyns
        xyz = torch.cat(pts, dim=1).contiguous()
        attr = torch.cat(attrs, dim=1).contiguous()
        cls = torch.cat(clss).contiguous()
        # S_v's scene scale (Sec. 3.2): the mean over frames of each frame's
        # mean depth, over the focal length
        self.depth_over_f = float(np.mean(mean_depth)) / self.f if mean_depth else 0.0
        self.mask_iou_frames = ious if ious else None
        self.mask_iou = float(np.mean(ious)) if ious else None
        return images, (xyz, attr, cls)

    def prune(self, cloud, voxel=0.01, min_count=1, voxel_dynamic=None):
        """gs4d_grid_prune of the cloud; an edge <= 0 leaves that class
        unpruned (every point kept)."""
        xyz, attr, cls = cloud
        dev = self.device
        m = xyz.shape[1]
        vd = voxel if voxel_dynamic is None else voxel_dynamic
        cap = m if not (voxel > 0 and vd > 0) else min(m, 4_000_000)
        out_xyz = torch.empty((3, cap), device=dev)
        out_attr = torch.empty((attr.shape[0], cap), device=dev)
        out_count = torch.empty(cap, dtype=torch.int32, device=dev)
        out_key = torch.empty(cap, dtype=torch.int64, device=dev)
        n_out = torch.zeros(1, dtype=torch.int64, device=dev)
        status = torch.zeros(1, dtype=torch.int32, device=dev)
        ws = torch.empty(G.gs4d_grid_prune_workspace_size(m, attr.shape[0]), dtype=torch.uint8,
                         device=dev)
        G.gs4d_grid_prune(xyz, attr, cls, voxel, vd, min_count, cap, out_xyz, out_attr,
                          out_count, out_key, n_out, status, ws)
        st, k = int(status.item()), int(n_out.item())
        if st != 0:
            raise RuntimeError(f"grid prune status {st} (voxels {k}, capacity {cap})")
        del ws
        dyn = (out_key[:k] < 0)          # class bit 63 set -> negative as int64
        return out_xyz[:, :k], out_attr[:, :k], dyn, out_count[:k]

    def heuristic_init(self, pruned, voxel=0.01, voxel_dynamic=None):
        """Sec. 4.1's initialisation of the pruned points (gs4d_heuristic_init):
        centroid, mean timestamp and colour; s_t = 2 / frames for dynamic and
        1 for static points; s_xyz = the class's voxel edge (the footprint of
        one pixel at its depth for a class that is not pruned); identity
        rotors; opacity 0.1."""
        xyz, attr, dyn, _ = pruned
        k = xyz.shape[1]
        vd = voxel if voxel_dynamic is None else voxel_dynamic
        p = torch.empty((20, k), device=self.device)
        G.gs4d_heuristic_init(xyz, attr[0:3], attr[3], attr[4], dyn.to(torch.uint8), k, voxel, vd,
                              self.f, self.frames, p)
        return p


# The paper's two initialisation settings (Sec. 4.1, implementation
# details): Lite prunes static and dynamic points on adaptive voxels with
# lambda_s = lambda_d = 4; Full uses lambda_s = 1 and leaves the dynamic
# points unpruned.  Both take the motion class from the Otsu split (Sec.
# 3.2).
PRESETS = {
    "lite": dict(motion="otsu", voxel="adaptive", lambda_static=4.0, lambda_dynamic=4.0),
    "full": dict(motion="otsu", voxel="adaptive", lambda_static=1.0, lambda_dynamic=None),
}


def build_scene(seed=0, n_gt=1_000_000, frames=200, width=960, height=540, voxel=0.01,
                device="cuda", verbose=False, keep_pruned=False, motion="gt",
                lambda_static=4.0, lambda_dynamic=4.0, preset=None, pseudo_frames=True):
    """Ground-truth frames and the pruned, heuristically initialised set
    (with keep_pruned, also the pruned cloud: xyz, attr, dynamic flag,
    count).  voxel: an edge length, or "adaptive" for S_v = lambda mean(D / f)
    with lambda_static / lambda_dynamic (None: that class is not pruned);
    motion: "gt" (ground-truth mask) or "otsu" (the paper's split); preset
    "lite" or "full" sets motion, voxel and both lambdas as the paper's
    settings of those names (PRESETS)."""
    if preset is not None:
        cfg = PRESETS[preset]
        motion, voxel = cfg["motion"], cfg["voxel"]
        lambda_static, lambda_dynamic = cfg["lambda_static"], cfg["lambda_dynamic"]
    sc = Scene(seed, n_gt, frames, width, height, device=device)
    images, cloud = sc.render_ground_truth(verbose, motion=motion, pseudo_frames=pseudo_frames)
    n_raw = cloud[0].shape[1]
    if voxel == "adaptive":
        vs = lambda_static * sc.depth_over_f if lambda_static is not None else 0.0
        vd = lambda_dynamic * sc.depth_over_f if lambda_dynamic is not None else 0.0
    else:
        vs = vd = float(voxel)
    pruned = sc.prune(cloud, vs, voxel_dynamic=vd)
    del cloud
    params = sc.heuristic_init(pruned, vs, vd)
    info = dict(n_raw_points=n_raw, n_gaussians=params.shape[1],
                n_dynamic=int(pruned[2].sum().item()), voxel_static=vs, voxel_dynamic=vd,
                depth_over_f=sc.depth_over_f, motion=motion, mask_iou=sc.mask_iou,
                preset=preset)
    if keep_pruned:
        return sc, images, params, info, pruned
    return sc, images, params, info
