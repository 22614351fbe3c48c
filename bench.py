"""Benchmark: training iterations/s of the 4D Gaussian-splatting optimisation
step on one MI355X, with Gaussian-pixel blends/s and the roofline of the
dominant kernel, next to the CPU oracle on the host cores.

Workload (default, "scene"): the scene-scale plain training configuration --
a seeded synthetic dynamic scene (textured planes + 3 rigid objects on
spline paths, 1M ground-truth Gaussians, 200 frames at 960x540) rendered by
this package, back-projected, grid-pruned at voxel 0.01 and heuristically
initialised; each step trains on one random frame with L1 + 0.2 (1 - SSIM).
"--workload small" runs the 2,000-Gaussian 64x64 single-view case instead.

A step = preprocess, bin/sort, render forward, loss + gradient, render and
preprocess backward, Adam: every stage a libgs4d.so kernel on the current
stream.  All inputs are in HBM before the timed region starts.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd train iters/s and Gaussian-pixel blends/s vs roofline; time-to-PSNR"
HBM_PEAK_GBS = 8000.0
# timed steps between two that bracket the render backward with HIP events
EVENT_EVERY = 4
# FP32 vector peak without packed FP32 (the library is built with packed FP32
# disabled): 256 CUs x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz = 78.6
# TFLOP/s; the published figure counts packed FP32: 157.3 TFLOP/s
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
ALU_PEAK_PUBLISHED_TFLOPS = 157.3
# Algorithmic FP32 flops of compositing (FMA = 2; exp and division 1 each).
# Per evaluated (pixel, entry): offset (2), quadratic form (9), exp and the
# product with o_t (2).  Per forward blend: 1 - alpha and the transmittance
# product (2), alpha T and the three colour FMAs (7).  Per backward blend:
# transmittance recovery (2), colour gradients (7), dC/dalpha (9), colour
# behind (6), opacity (2), exponent gradient (1), conic (11), mean (10).
FLOPS_EVAL = 13
FLOPS_BLEND_FWD = 9
FLOPS_BLEND_BWD = 48


class ProfileRegion:
    """roctxProfilerResume(0) / roctxProfilerPause(0) around a timed region:
    under `rocprofv3 --marker-trace --selected-regions` only what runs inside
    is collected, so a profile covers exactly the launches a bench line
    times.  Counter runs cannot trace markers, so the region is also
    bracketed by one short torch spin kernel on each side (drained before
    the region's clock starts): in a `--pmc` dispatch list the launches
    between the two spin kernels are the region's.  Without a profiler (or
    the ROCTx library) the calls do nothing."""

    def __init__(self, active):
        self.lib = None
        self.active = active
        if active:
            import ctypes
            for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so"):
                try:
                    self.lib = ctypes.CDLL(name)
                    break
                except OSError:
                    continue
            if self.lib is not None:
                self.lib.roctxProfilerResume.argtypes = [ctypes.c_uint64]
                self.lib.roctxProfilerPause.argtypes = [ctypes.c_uint64]
                self.lib.roctxProfilerResume.restype = ctypes.c_int
                self.lib.roctxProfilerPause.restype = ctypes.c_int
            else:
                log("bench: ROCTx library not found; profiling regions are not marked")

    def _sentinel(self):
        import torch
        spin = getattr(torch.cuda, "_sleep", None)
        if spin is not None:
            spin(64)
        torch.cuda.synchronize()

    def __enter__(self):
        if self.active:
            self._sentinel()
        if self.lib is not None:
            rc = self.lib.roctxProfilerResume(0)
            if rc:
                log(f"bench: roctxProfilerResume returned {rc}")
        return self

    def __exit__(self, *exc):
        if self.lib is not None:
            rc = self.lib.roctxProfilerPause(0)
            if rc:
                log(f"bench: roctxProfilerPause returned {rc}")
        if self.active:
            self._sentinel()
        return False


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_workload(name, device, cache=None):
    """Inputs of the workload, in HBM.  With `cache`, the synthesised scene is
    saved to / loaded from that file (a profiled run then contains only the
    training kernels)."""
    import torch
    if cache and name == "scene" and os.path.exists(cache):
        d = torch.load(cache, map_location=device, weights_only=True)
        info = json.loads(d["info"])
        pruned = (d["pruned_xyz"], d["pruned_attr"], d["pruned_dyn"]) if "pruned_xyz" in d else None
        return d["params"], d["views"].cpu().numpy(), d["images"], info, pruned
    out = _build_workload(name, device)
    if cache and name == "scene":
        params, views, images, info, pruned = out
        torch.save({"params": params, "views": torch.from_numpy(np.asarray(views)),
                    "images": images, "info": json.dumps(info), "pruned_xyz": pruned[0],
                    "pruned_attr": pruned[1], "pruned_dyn": pruned[2]}, cache)
    return out


def _build_workload(name, device):
    import torch
    from paper_2510_01119_amd import synth
    if name == "small":
        params = torch.from_numpy(synth.small_set(2000, 0)).to(device)
        target_p = torch.from_numpy(synth.perturb(synth.small_set(2000, 0), 1)).to(device)
        view = synth.front_view(64, 64, 64.0, 3.0, 0.5)
        from paper_2510_01119_amd.rasterizer import Rasterizer
        r = Rasterizer(2000, view, device=device)
        r.forward(target_p)
        images = r.image.clone()
        info = dict(workload="plain single-view 2k Gaussians 64x64", n_gaussians=2000, frames=1,
                    width=64, height=64)
        return params, view[None], images, info, None
    from paper_2510_01119_amd.scene import build_scene
    t0 = time.time()
    sc, images, params, info, pruned = build_scene(seed=0, device=device, verbose=True,
                                                   keep_pruned=True)
    info.update(workload="scene-scale plain training: synthetic dynamic scene, 200 frames 960x540, "
                         "1M-Gaussian ground truth, grid-pruned at 0.01",
                frames=sc.frames, width=sc.W, height=sc.H, synth_s=round(time.time() - t0, 2))
    return params, sc.cams, images, info, pruned[:3]


def host_cores():
    """(cores this process may use, capped at 16 -- the host share of one
    GPU --, nproc, CPU model)."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return min(usable, 16), os.cpu_count(), model


def cpu_baseline(params_np, views, targets_np, budget_s=20.0):
    """The oracle's training step (FP32-decided preprocess, FP64 compositing
    and chain rule, numpy loss and Adam), as it stands: one single-threaded
    oracle process per usable host core, each repeating steps on its own
    frame for budget_s seconds; the rate is the sum of their steps over the
    wall time."""
    import subprocess
    import tempfile
    cores, nproc, model = host_cores()
    with tempfile.TemporaryDirectory(prefix="gs4d_cpu_") as d:
        np.save(os.path.join(d, "params.npy"), params_np.astype(np.float32))
        np.save(os.path.join(d, "views.npy"), np.asarray(views, np.float64))
        np.save(os.path.join(d, "targets.npy"), np.asarray(targets_np, np.float64))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        t0 = time.perf_counter()
        procs = [subprocess.Popen([sys.executable, "-m", "oracle.bench_worker", d, str(i),
                                   str(budget_s)], cwd=ROOT, env=env, stdout=subprocess.PIPE,
                                  stderr=subprocess.PIPE, text=True) for i in range(cores)]
        outs = [p.communicate() for p in procs]
        wall = time.perf_counter() - t0
    steps = 0
    for p, (out, err) in zip(procs, outs):
        if p.returncode != 0:
            raise RuntimeError(f"oracle worker failed: {err[-500:]}")
        steps += json.loads(out.strip().splitlines()[-1])["steps"]
    return steps / wall, steps, wall, cores, nproc, model


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="scene", choices=["scene", "small", "batched"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 8-view batched leg (500k Gaussians, 960x540)")
    ap.add_argument("--no-ttp", action="store_true", help="skip the time-to-PSNR leg")
    ap.add_argument("--no-fps", action="store_true",
                    help="skip the forward-only frame-rate leg at display sizes")
    ap.add_argument("--no-iso", action="store_true",
                    help="skip the isotropic, motion-aware form's leg (throughput and ablation)")
    ap.add_argument("--no-sch", action="store_true",
                    help="skip the SCH colour's leg (throughput and the w/o-RGB ablation)")
    ap.add_argument("--no-scene-prep", action="store_true",
                    help="skip the leg that builds the scene with the Otsu split and adaptive voxels")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of graph replays")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters); it "
                         "runs inside the profiled region")
    ap.add_argument("--profile-region", default="scene", choices=["scene", "batched", "none"],
                    help="the timed region bracketed for rocprofv3 --selected-regions")
    ap.add_argument("--scene-cache", default=None,
                    help="save/load the synthesised scene here (e.g. /tmp/gs4d_scene.pt)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; --gpus must be 1 (sharding the "
                                   "step over GPUs by view is not implemented)"}))
        sys.exit(2)

    import torch
    from paper_2510_01119_amd import gs4d as G
    from paper_2510_01119_amd.train import Trainer

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    G.lib()
    dev = torch.device("cuda:0")
    if args.workload == "batched":
        out = run_batched(args, dev, ProfileRegion(args.profile_region == "batched"))
        print(json.dumps(out), flush=True)
        return
    log(f"bench: building workload {args.workload}")
    params, views, images, info, pruned = build_workload(args.workload, dev, args.scene_cache)
    n = params.shape[1]
    log(f"bench: {info}")
    tr = Trainer(params.clone(), views, images, budget=5000)
    peak = tr.size_pairs(range(0, len(views), max(1, len(views) // 20)), margin=2.0)
    log(f"bench: pair peak over sampled frames {peak}, capacity {tr.rast.capacity}")
    rng = np.random.default_rng(args.seed)
    seq = rng.integers(0, len(views), args.warmup + args.steps)

    for i in range(args.warmup):
        tr.step(int(seq[i]))
    torch.cuda.synchronize()
    # autotune the render kernels on a warmed-up frame (untimed)
    from paper_2510_01119_amd import autotune
    tr.forward_loss(int(seq[0]))
    choice = autotune.tune(tr.rast, tr.params, tr.dimg)
    log(f"bench: autotune {json.dumps(choice)}")
    for i in range(2):
        tr.step(int(seq[i]))
    torch.cuda.synchronize()

    r = tr.rast
    stages = ["preprocess", "bin_sort", "render_fwd", "loss", "render_bwd", "preprocess_bwd", "adam"]

    # ---- timed region: exactly `steps` training steps --------------------
    # Graph mode: each frame's step was captured as one HIP graph and again
    # as three ([forward + loss + clearing the 2D-gradient accumulator],
    # [render backward kernel], [preprocess backward + Adam]).  Every
    # EVENT_EVERY-th step replays the three, with HIP events on the launch
    # stream bracketing the render backward; the others replay the single
    # graph.
    use_graph = not args.eager
    if use_graph:
        t_cap = time.perf_counter()
        tr.capture(sorted(set(int(f) for f in seq)))
        log(f"bench: captured {len(tr.graphs)} frames x (1 + 3) graphs in "
            f"{time.perf_counter() - t_cap:.1f} s")
        for i in range(3):
            tr.step_graph(int(seq[i]))
            tr.step_graph(int(seq[i]), events=(torch.cuda.Event(enable_timing=True),
                                               torch.cuda.Event(enable_timing=True)))
    bwd_ev = []
    region = ProfileRegion(args.profile_region == "scene")
    if args.calib_copy:
        # a plain copy of known size inside the profiled region: its
        # FETCH_SIZE / WRITE_SIZE per byte calibrates the counters read for
        # the gs4d kernels
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        with region:
            dst.copy_(src)
            torch.cuda.synchronize()
        del src, dst
        log("bench: calibration copy 256 MiB done")
    torch.cuda.synchronize()
    with region:
        t0 = time.perf_counter()
        for i in range(args.steps):
            f = int(seq[args.warmup + i])
            if use_graph and i % EVENT_EVERY:
                tr.step_graph(f)
                continue
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            if use_graph:
                tr.step_graph(f, events=(a, b))
            else:
                tr.stage_forward(f)
                a.record()
                tr.stage_render_bwd(f)
                b.record()
                tr.stage_update(f)
            bwd_ev.append((a, b))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    if int(tr.overflow_seen.item()) != 0:
        raise RuntimeError("pair capacity overflowed during the timed region")
    elapsed = t1 - t0
    its = args.steps / elapsed
    bwd_ms_timed = float(np.mean([x.elapsed_time(y) for x, y in bwd_ev]))
    # blends per step in the state of the timed region: the forward counters
    # over its first (up to) 50 frames, untimed
    counts = count_blends(r, tr.params, [tr.cviews[int(f)] for f in seq[args.warmup:]][:50])
    pairs_per_step = counts.pop("pairs")

    # ---- per-stage breakdown: eager replay of the same frames with events --
    ev = {s_: [] for s_ in stages}

    def staged_step(f):
        def mark(name, fn):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            ev[name].append((a, b))
        r.set_views(tr.cviews[f])
        mark("preprocess", lambda: r.preprocess(tr.params))
        mark("bin_sort", lambda: r.bin_sort(check=False))
        mark("render_fwd", lambda: r.render())
        mark("loss", lambda: G.gs4d_photometric_loss(r.image, tr.targets[f:f + 1], 1.0, tr.ssim_w,
                                                     tr.loss, tr.dimg, tr.ssim_ws))
        r.zero_grad2d()
        mark("render_bwd", lambda: tr.stage_render_bwd(f))
        mark("preprocess_bwd", lambda: G.gs4d_preprocess_bwd(tr.params, r.touched, r.grad2d,
                                                             tr.cviews[f], r.dparams))
        mark("adam", lambda: G.gs4d_adam_step(tr.params, r.dparams, tr.m, tr.v, tr.cfg, tr.step_dev))

    for i in range(min(args.steps, 50)):
        staged_step(int(seq[args.warmup + i]))
    torch.cuda.synchronize()
    # median: a host hiccup between two recorded events would inflate a mean
    stage_ms = {s_: float(np.median([a.elapsed_time(b) for a, b in ev[s_]])) for s_ in stages}
    log(f"bench: {its:.1f} it/s ({'graph' if use_graph else 'eager'}); render_bwd timed "
        f"{bwd_ms_timed:.4f} ms; eager stage ms {json.dumps({k: round(v, 4) for k, v in stage_ms.items()})}")

    # roofline of the dominant kernel
    dominant = max(stage_ms, key=stage_ms.get)
    HW = info["width"] * info["height"]
    dom_ms = bwd_ms_timed if dominant == "render_bwd" else stage_ms[dominant]
    roof = roofline_for(dominant, dom_ms, n, pairs_per_step, counts, HW)
    roof["ms_per_launch"] = round(dom_ms, 4)
    roof["timing"] = (f"HIP events around every {EVENT_EVERY}th launch in the timed region (the "
                      f"render backward kernel alone)"
                      if dominant == "render_bwd" else "HIP events, eager replay of the timed frames")
    roof["units"] = (f"{FLOPS_EVAL} flops per evaluated (pixel, entry) + {FLOPS_BLEND_BWD} per blend "
                     f"(FMA = 2), per launch; peak = unpacked FP32 FMA rate")

    line = {
        "metric": METRIC,
        "value": round(its, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": info["workload"], "n_gaussians": n, "width": info["width"],
                   "height": info["height"], "frames": info["frames"],
                   "loss": "L1 + 0.2(1-SSIM)", "n_raw_points": info.get("n_raw_points"),
                   "state": f"parameters after {args.warmup} warm-up + 2 autotune steps; timed "
                            f"frames seed {args.seed}"},
        "blends_per_s": round(counts["blends"] * its, 1),
        "evaluated_per_s": round(counts["evaluated"] * its, 1),
        "blends_per_step": round(counts["blends"], 1),
        "evaluated_per_step": round(counts["evaluated"], 1),
        "evaluated_to_last_blend_per_step": round(counts["evaluated_to_last"], 1),
        "pairs_per_step": round(pairs_per_step, 1),
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "launch": ("hip graphs" if use_graph else "eager") + f", {choice.get('mode', 'grid')} (autotuned)",
        "autotune": {"fwd_batch": choice["batch"], "bwd_pixels_per_lane": choice["bwd_pixels_per_lane"],
                     "mode": choice.get("mode"), "mode_ms": choice.get("mode_ms"),
                     "workgroups_per_cu": choice.get("workgroups_per_cu"),
                     "wg_ms": choice.get("wg_ms")},
        "roofline": roof,
    }
    if args.workload == "scene" and not args.no_fps:
        line["render_fps"] = render_fps_leg(tr.params, views)

    if not args.no_cpu_baseline:
        p_np = tr.params.detach().cpu().numpy()
        fsel = [int(f) for f in seq[args.warmup:args.warmup + 16]]
        tgt = images[fsel].cpu().numpy()
        v_np = np.stack([views[f] for f in fsel])
        log("bench: cpu baseline (oracle workers) ...")
        rate, steps_done, secs, cores, nproc, model = cpu_baseline(p_np, v_np, tgt)
        line["cpu_baseline"] = {
            "value": round(rate, 6), "unit": "iters/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps_done} full training steps of the same workload ({n} Gaussians, one "
                      f"960x540 frame each) in {secs:.1f} s wall, one single-threaded oracle process "
                      f"per core on {cores} cores",
            "host": {"nproc": nproc, "usable_cores": cores, "cpu": model}}
        del p_np
    if not args.no_batched:
        torch.cuda.empty_cache()
        line["batched"] = run_batched(args, dev, ProfileRegion(args.profile_region == "batched"))
        torch.cuda.empty_cache()
    if args.workload == "scene" and not args.no_ttp and pruned is not None:
        line["time_to_psnr"] = time_to_psnr_leg(params, views, images, pruned)
    if args.workload == "scene" and not args.no_iso:
        line["iso_form"] = iso_leg(params, views, images, args.seed)
    if args.workload == "scene" and not args.no_sch:
        line["sch_form"] = sch_leg(params, views, images, args.seed)
    if args.workload == "scene" and not args.no_scene_prep:
        line["scene_prep"] = scene_prep_leg(params, views, images, args.seed)
    print(json.dumps(line), flush=True)


def count_blends(r, params, cviews):
    """Forward counters over the given frames (untimed): per step averages of
    evaluated (pixel, entry) pairs, blends, evaluated pairs up to each
    pixel's last blend (what the backward re-evaluates), and pairs."""
    import torch
    r.counters = torch.zeros(3, dtype=torch.int64, device=params.device)
    tot = np.zeros(3)
    pairs = []
    for cv in cviews:
        r.set_views(cv)
        r.preprocess(params)
        r.bin_sort(check=False)
        r.render()
        tot += r.counters.cpu().numpy()
        pairs.append(int(r.n_pairs.item()))
    r.counters = None
    k = max(len(cviews), 1)
    return {"evaluated": tot[0] / k, "blends": tot[1] / k, "evaluated_to_last": tot[2] / k,
            "pairs": float(np.mean(pairs))}


def iso_leg(params, views, images, seed, steps=200, warmup=20, budget=1500):
    """The paper's isotropic, motion-aware parameterisation (13 floats per
    Gaussian) on the same scene, from the same heuristic initialisation:
    training iterations/s (whole steps replayed from graphs, render launches
    autotuned as for the rotor form), and a synthetic analogue of the
    paper's ablation at a fixed budget of `budget` single-frame steps:
    PSNR on held-out frames (every 10th) of the rotor form ("w/o
    isotropic"), the isotropic form with its velocity trained, and with the
    velocity frozen at zero ("w/o motion-aware")."""
    import torch
    from paper_2510_01119_amd import autotune
    from paper_2510_01119_amd.train import Trainer, to_iso
    F = len(views)
    rng = np.random.default_rng(seed + 7)
    sample = range(0, F, max(1, F // 20))
    tr = Trainer(to_iso(params.clone()), views, images, budget=5000)
    tr.size_pairs(sample, margin=2.0)
    seq = rng.integers(0, F, warmup + steps)
    for i in range(warmup):
        tr.step(int(seq[i]))
    tr.forward_loss(int(seq[0]))
    autotune.tune(tr.rast, tr.params, tr.dimg)
    tr.capture(sorted(set(int(f) for f in seq[warmup:])))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        tr.step_graph(int(seq[warmup + i]))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if int(tr.overflow_seen.item()) != 0:
        raise RuntimeError("pair capacity overflowed in the isotropic form's timed steps")
    out = {"iters_per_s": round(steps / dt, 1), "ms_per_step": round(1e3 * dt / steps, 4),
           "floats_per_gaussian": 13}
    del tr
    torch.cuda.empty_cache()
    held = list(range(5, F, 10))
    train = [f for f in range(F) if f % 10 != 5]
    order = rng.choice(train, size=budget)
    variants = {
        "rotor (w/o isotropic)": (params, None),
        "isotropic + velocity": (to_iso(params), None),
        "isotropic, velocity frozen (w/o motion-aware)": (to_iso(params), {"velocity": (0.0, 0.0)}),
    }
    psnr = {}
    for name, (p0, lrs) in variants.items():
        t = Trainer(p0.clone(), views, images, budget=budget, lrs=lrs)
        t.size_pairs(sample, margin=2.0)
        for f in order:
            t.step(int(f))
        psnr[name] = (round(t.psnr(held), 3)
                      if int(t.overflow_seen.item()) == 0 else None)
        del t
        torch.cuda.empty_cache()
    out["ablation"] = {"steps": budget, "heldout_frames": len(held), "psnr_db": psnr}
    log(f"bench: isotropic form {json.dumps(out)}")
    return out


def sch_leg(params, views, images, seed, steps=200, warmup=20, budget=1500, degree=3, n_freq=2,
            period=2.0):
    """The sphericylindrical-harmonic colour the paper ablates (Sec. 4.4,
    "w/o RGB"; Sec. 3.1, SCH equation) on the same scene and heuristic
    initialisation, coefficients started from its RGB: training
    iterations/s (graph replays, render launches autotuned as for the RGB
    form) and, at a fixed budget of `budget` single-frame steps in the same
    frame order, held-out PSNR (every 10th frame) of RGB against SCH of
    degree `degree` with `n_freq` temporal frequencies (period `period`,
    twice the sequence in normalised time)."""
    import torch
    from paper_2510_01119_amd import autotune
    from paper_2510_01119_amd import gs4d as G
    from paper_2510_01119_amd.train import Trainer
    F = len(views)
    rng = np.random.default_rng(seed + 11)
    sample = range(0, F, max(1, F // 20))
    sch = G.make_sch(degree, n_freq, period)
    rows = G.gs4d_sch_rows(degree, n_freq)
    tr = Trainer(params.clone(), views, images, budget=5000, sch=sch)
    tr.size_pairs(sample, margin=2.0)
    seq = rng.integers(0, F, warmup + steps)
    for i in range(warmup):
        tr.step(int(seq[i]))
    tr.forward_loss(int(seq[0]))
    autotune.tune(tr.rast, tr.params, tr.dimg)
    tr.capture(sorted(set(int(f) for f in seq[warmup:])))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        tr.step_graph(int(seq[warmup + i]))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if int(tr.overflow_seen.item()) != 0:
        raise RuntimeError("pair capacity overflowed in the SCH form's timed steps")
    out = {"iters_per_s": round(steps / dt, 1), "ms_per_step": round(1e3 * dt / steps, 4),
           "degree": degree, "n_freq": n_freq, "period": period,
           "floats_per_gaussian": 17 + rows}
    del tr
    torch.cuda.empty_cache()
    held = list(range(5, F, 10))
    order = rng.choice([f for f in range(F) if f % 10 != 5], size=budget)
    psnr = {}
    for name, s in (("rgb (the paper's)", None),
                    (f"SCH degree {degree}, {n_freq} temporal frequencies (w/o RGB)", sch)):
        t = Trainer(params.clone(), views, images, budget=budget, sch=s)
        t.size_pairs(sample, margin=2.0)
        for f in order:
            t.step(int(f))
        psnr[name] = round(t.psnr(held), 3) if int(t.overflow_seen.item()) == 0 else None
        del t
        torch.cuda.empty_cache()
    out["ablation"] = {"steps": budget, "heldout_frames": len(held), "psnr_db": psnr}
    log(f"bench: SCH form {json.dumps(out)}")
    return out


def scene_prep_leg(params_gt, views, images_gt, seed, steps=1500):
    """The same synthetic scene prepared the paper's ways (Sec. 3.2, Sec.
    4.1): the motion class from the Otsu split of a noisy low-resolution
    motion-probability map, adaptive voxel edges S_v = lambda mean(D / f),
    and the two settings -- Lite (lambda 4 for static and dynamic points)
    and Full (lambda 1 for static points, dynamic points unpruned).  Per
    preset: build time, S_v, the mask's IoU with the ground truth, the
    Gaussian counts, training iterations/s and the held-out PSNR after
    `steps` single-frame steps (one frame order for all), beside the default
    preparation (ground-truth mask, 0.01 voxels)."""
    import torch
    from paper_2510_01119_amd.scene import build_scene
    from paper_2510_01119_amd.train import Trainer
    F = len(views)
    rng = np.random.default_rng(seed + 9)
    held = list(range(5, F, 10))
    order = rng.choice([f for f in range(F) if f % 10 != 5], size=steps)

    def train(p0, imgs):
        t = Trainer(p0.clone(), views, imgs, budget=steps)
        t.size_pairs(range(0, F, max(1, F // 20)), margin=2.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in order:
            t.step(int(f))
        torch.cuda.synchronize()
        rate = steps / (time.perf_counter() - t0)
        ok = int(t.overflow_seen.item()) == 0
        psnr = round(t.psnr(held), 3) if ok else None
        del t
        torch.cuda.empty_cache()
        return psnr, round(rate, 1)

    out = {"psnr_db_after_steps": steps, "presets": {}}
    for preset in ("lite", "full"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sc, images, params, info = build_scene(seed=0, device="cuda", preset=preset)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        iou_frames = np.array(sc.mask_iou_frames)
        del sc
        psnr, rate = train(params, images)
        out["presets"][preset] = {
            "build_s": round(build_s, 2), "voxel_static": round(info["voxel_static"], 6),
            "voxel_dynamic": round(info["voxel_dynamic"], 6), "mask_iou": round(info["mask_iou"], 4),
            "n_gaussians": info["n_gaussians"], "n_dynamic": info["n_dynamic"],
            "iters_per_s": rate, "psnr_db": psnr}
        out["depth_over_f"] = round(info["depth_over_f"], 7)
        out["n_raw_points"] = info["n_raw_points"]
        del images, params
        torch.cuda.empty_cache()
    # the motion maps' sequence ends with and without pseudo-frames (the
    # presets use them): mask IoU of the first and last frames, and of the
    # rest
    from paper_2510_01119_amd.scene import Scene
    sc = Scene(0, device="cuda")
    sc.render_ground_truth(motion="otsu", pseudo_frames=False)
    plain = np.array(sc.mask_iou_frames)
    del sc
    torch.cuda.empty_cache()
    out["pseudo_frames"] = {
        "mask_iou_ends": round(float(iou_frames[[0, -1]].mean()), 4),
        "mask_iou_ends_without": round(float(plain[[0, -1]].mean()), 4),
        "mask_iou_interior": round(float(iou_frames[1:-1].mean()), 4),
        "mask_iou_interior_without": round(float(plain[1:-1].mean()), 4)}
    psnr, rate = train(params_gt, images_gt)
    out["default"] = {"motion": "ground-truth mask", "voxel": 0.01,
                      "n_gaussians": int(params_gt.shape[1]), "iters_per_s": rate,
                      "psnr_db": psnr}
    log(f"bench: scene prep {json.dumps(out)}")
    return out


def render_fps_leg(params, views, frames=200):
    """Forward-only frame rate of the parameters as they stand after the
    timed training steps, at display sizes: 16 of the scene's cameras (the
    960x540 intrinsics rescaled), each launch one graph replay of preprocess,
    binning, tile ordering and compositing -- one frame per launch (the
    latency mode), and 8 consecutive frames per launch ("_x8", playback
    throughput)."""
    import torch
    from paper_2510_01119_amd.realtime import DISPLAY_SIZES, FrameRenderer, rescale_view
    sel = np.linspace(0, len(views) - 1, 16).round().astype(int)
    out = {}
    for W, H in DISPLAY_SIZES:
        vs = np.stack([rescale_view(views[f], W, H) for f in sel])
        for B in (1, 8):
            fr = FrameRenderer(params, vs, frames_per_launch=B)
            out[f"{W}x{H}" + ("" if B == 1 else f"_x{B}")] = fr.frame_rate(frames=frames)
            del fr
            torch.cuda.empty_cache()
    log(f"bench: forward-only frame rate {json.dumps(out)}")
    return out


def time_to_psnr_leg(params, views, images, pruned):
    """Wall time to the plain single-view form's PSNR: plain training (one
    frame per step, 5,000 steps) fixes the reference on the held-out frames;
    the batched form (4 frames per step, its validated schedule) from the
    heuristic and from the learned initialisation trains until it is within
    0.1 dB.  Also the learned initialisation's fixed-budget gain on this
    scene: held-out PSNR after 300 batched steps of 8 frames from either
    initialisation."""
    import types
    import torch
    from paper_2510_01119_amd import learned_init as LI
    from paper_2510_01119_amd.pipeline import (BATCHED_DECAY, BATCHED_LR_MULT, init_gain,
                                               time_to_psnr)
    log("bench: time-to-PSNR (plain 5000 steps, then batched from both initialisations)")
    sc = types.SimpleNamespace(frames=len(views), cams=np.asarray(views))
    model = LI.InitModel.load() if os.path.exists(LI.MODEL_PATH) else None
    r = time_to_psnr(sc, images, params, pruned, model)
    torch.cuda.empty_cache()
    out = {k: v for k, v in r.items() if k not in ("heuristic", "learned")}
    for name in ("heuristic", "learned"):
        if name in r:
            out[name] = {k: v for k, v in r[name].items() if k != "history"}
    out["held_out"] = "every 10th frame; the others train"
    if model is not None:
        g = init_gain(sc, images, params, pruned, model, budget=300, lr_mult=BATCHED_LR_MULT,
                      group=8, decay=BATCHED_DECAY)
        torch.cuda.empty_cache()
        out["fixed_budget"] = {"steps": 300, "views_per_step": 8,
                               "psnr_heuristic": g["heuristic"]["psnr"][-1],
                               "psnr_learned": g["learned"]["psnr"][-1],
                               "gain_db": round(g["learned"]["psnr"][-1] - g["heuristic"]["psnr"][-1], 3)}
    log(f"bench: time-to-PSNR {json.dumps(out)}")
    return out


def profiled_field(path, field):
    """A machine-read field of a committed rocprofv3 summary, or None if there
    is none or the profiled kernel's source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", path)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "|", " ")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    src = fields.get("kernel_source")
    if not src or field not in fields:
        return None
    digest = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()[:16]
    if digest != fields.get("kernel_source_sha256_16"):
        return None
    return float(fields[field])


def profiled_traffic(kernel):
    """HBM bytes per launch from the committed counter summary (or None)."""
    return profiled_field(f"{kernel}_scene_960x540_traffic.md", "traffic_bytes_per_launch")


def run_batched(args, dev, region):
    """The batched configuration: 8 views per launch from 500k Gaussians
    (uneven visible counts), fused per-view L1, persistent largest-first
    launches, autotuned batch size and block shape, each step replayed from
    HIP graphs; `args.steps` steps timed after `args.warmup`.  Returns its
    figures (iterations/s, views/s, blends/s, the render backward's
    roofline)."""
    import torch
    from paper_2510_01119_amd import autotune, synth
    from paper_2510_01119_amd.rasterizer import Rasterizer
    from paper_2510_01119_amd.train import BatchedTrainer
    t0 = time.time()
    p_np = synth.batched_set(500_000, seed=3)
    views = synth.batched_views(p_np)
    params = torch.from_numpy(p_np).to(dev)
    rt = Rasterizer(params.shape[1], views, device=dev, pair_capacity=1 << 25)
    rt.forward(torch.from_numpy(synth.perturb(p_np, 4)).to(dev))
    targets = rt.image.clone()
    del rt
    tr = BatchedTrainer(params.clone(), views, targets, budget=5000)
    peak = tr.size_pairs(margin=1.3)
    vis = (tr.rast.touched > 0).sum(dim=1).cpu().numpy().tolist()
    log(f"bench: batched set ready in {time.time() - t0:.1f} s; visible per view {vis}; pairs {peak}")
    for _ in range(args.warmup):
        tr.step()
    torch.cuda.synchronize()
    choice = autotune.tune(tr.rast, tr.params, tr.rast.dL_dimage)
    log(f"bench: batched autotune {json.dumps(choice)}")
    tr.capture()
    for _ in range(3):
        tr.step_graph()
    ev = []
    torch.cuda.synchronize()
    with region:
        t1 = time.perf_counter()
        for i in range(args.steps):
            if i % EVENT_EVERY:
                tr.step_graph()
                continue
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            tr.step_graph(events=(a, b))
            ev.append((a, b))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    if int(tr.overflow_seen.item()) != 0:
        raise RuntimeError("pair capacity overflowed during the timed region")
    its = args.steps / (t2 - t1)
    bwd_ms = float(np.mean([x.elapsed_time(y) for x, y in ev]))
    r = tr.rast
    counts = count_blends(r, tr.params, [r.cviews])
    pairs = counts.pop("pairs")
    roof = roofline_for("render_bwd", bwd_ms, params.shape[1], pairs, counts, 960 * 540 * len(views))
    roof["ms_per_launch"] = round(bwd_ms, 4)
    roof["timing"] = (f"HIP events around every {EVENT_EVERY}th render-backward graph replay in "
                      "the timed region (the render backward kernel alone)")
    roof["traffic"] = None          # the HBM counters were taken on the scene workload
    roof.pop("traffic_GBps", None)
    out = {
        "workload": "batched: 8 views per persistent launch, 500k 4D Gaussians, 960x540, "
                    "fused per-view L1",
        "iters_per_s": round(its, 3), "ms_per_step": round(1000.0 * (t2 - t1) / args.steps, 4),
        "steps": args.steps, "warmup": args.warmup,
        "views_per_s": round(its * len(views), 2),
        "n_gaussians": int(params.shape[1]), "views": len(views), "visible_per_view": vis,
        "width": 960, "height": 540,
        "blends_per_s": round(counts["blends"] * its, 1),
        "blends_per_step": round(counts["blends"], 1),
        "pairs_per_step": round(pairs, 1),
        "launch": f"hip graphs, {choice.get('mode', 'grid')} (autotuned)",
        "autotune": {"fwd_batch": choice["batch"], "bwd_pixels_per_lane": choice["bwd_pixels_per_lane"],
                     "mode": choice.get("mode"), "workgroups_per_cu": choice.get("workgroups_per_cu")},
        "loss_per_view": [round(float(x), 5) for x in tr.loss_per_view()],
        "roofline": roof,
    }
    log(f"bench: batched {its:.1f} it/s, render_bwd {bwd_ms:.4f} ms")
    del tr
    return out


def roofline_for(kernel, ms, n, pairs, counts, hw):
    """Algorithmic work of one launch of `kernel` over its measured time.

    render_fwd / render_bwd are bound by the FP32 vector ALU: algorithmic
    flops (FMA = 2, exp and division 1) of the forward, FLOPS_EVAL per
    evaluated (pixel, entry) and FLOPS_BLEND_FWD per blend; of the backward,
    FLOPS_EVAL per (pixel, entry) it re-evaluates (those up to each pixel's
    last blend) and FLOPS_BLEND_BWD per blend -- counts from the forward's
    counters over the same frames -- against the unpacked FP32 FMA rate.
    Other kernels: algorithmic HBM bytes against 8 TB/s."""
    s = ms / 1000.0
    if kernel in ("render_fwd", "render_bwd"):
        if kernel == "render_fwd":
            flops = FLOPS_EVAL * counts["evaluated"] + FLOPS_BLEND_FWD * counts["blends"]
        else:
            flops = FLOPS_EVAL * counts["evaluated_to_last"] + FLOPS_BLEND_BWD * counts["blends"]
        achieved = flops / s / 1e12
        traffic = profiled_traffic(kernel)
        # the issue-rate view: the kernel's VALU instructions per launch
        # (committed SQ-counter summary of the same kernel source, scene
        # state) over the SIMDs' wave64 issue capacity in the measured time
        # (1,024 SIMDs, 4 cycles per wave64 instruction, 2.4 GHz)
        valu = (profiled_field("render_scene_960x540_valu_lds.md", f"{kernel}_valu_instructions_per_launch")
                if hw == 960 * 540 else None)
        issue = None
        if valu is not None:
            issue = {"valu_instructions": round(valu),
                     "issue_frac": round(valu * 4 / (1024 * 2.4e9 * s), 4),
                     "lane_instructions_per_evaluation": round(
                         valu * 64 / (counts["evaluated_to_last"] if kernel == "render_bwd"
                                      else counts["evaluated"]), 1)}
        # LDS against its peak: the kernel's LDS wave instructions per launch
        # (committed counter summary) over one per compute unit per cycle
        lds_n = (profiled_field("render_scene_960x540_lds.md", f"{kernel}_lds_instructions_per_launch")
                 if hw == 960 * 540 else None)
        lds = None
        if lds_n is not None:
            lds = {"lds_instructions": round(lds_n),
                   "issue_frac": round(lds_n / (256 * 2.4e9 * s), 4),
                   "bank_conflict_share": profiled_field("render_scene_960x540_lds.md",
                                                         f"{kernel}_lds_conflict_share")}
        return {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3),
                "peak": round(ALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                "frac": round(achieved / ALU_PEAK_TFLOPS, 4),
                "peak_published": ALU_PEAK_PUBLISHED_TFLOPS,
                "frac_published": round(achieved / ALU_PEAK_PUBLISHED_TFLOPS, 4),
                "flops_per_launch": round(flops),
                "traffic": None if traffic is None else round(traffic),
                "traffic_GBps": None if traffic is None else round(traffic / s / 1e9, 1),
                "valu_issue": issue, "lds": lds}
    bytes_per = {
        "preprocess": 80.0 * n + 68.0 * n,
        "bin_sort": 40.0 * pairs + 64.0 * n,
        "preprocess_bwd": 80.0 * n + 36.0 * n + 80.0 * n,
        "adam": 20 * 4.0 * n * 5,
        "loss": 36.0 * hw * 3,
    }.get(kernel, 0.0)
    achieved = bytes_per / s / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}


if __name__ == "__main__":
    main()
