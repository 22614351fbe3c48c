"""Scene-level optimisation runs: the plain single-view form of the method
(Sec. 4.1: one random training frame per step, L1 + 0.2 (1 - SSIM), Adam,
5,000 iterations) and the batched form (eight training frames per step in
one persistent launch per stage, the same loss over the eight images), both
replayed from HIP graphs, with PSNR on held-out frames and wall time that
excludes the evaluations.

Held-out frames: every 10th frame of the sequence (frame 0, 10, ...); the
others train.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import gs4d as G
from .rasterizer import Rasterizer
from .train import Trainer, _capture, adam_config


def split_frames(n_frames: int):
    held = [f for f in range(n_frames) if f % 10 == 0]
    train = [f for f in range(n_frames) if f % 10 != 0]
    return train, held


class Evaluator:
    """Mean PSNR of a parameter set over held-out frames (forward only)."""

    def __init__(self, n, views, targets, frames, device="cuda"):
        self.views = np.atleast_2d(views)
        self.targets = targets
        self.frames = list(frames)
        self.rast = Rasterizer(n, self.views[self.frames[0]], device=device)
        self.sse = torch.zeros(1, dtype=torch.float64, device=device)

    def psnr(self, params) -> float:
        r = self.rast
        vals = []
        for f in self.frames:
            r.set_views(self.views[f])
            r.forward(params, check=True)
            G.gs4d_fill_f32(self.sse.view(torch.float32), 0.0)
            G.gs4d_sse(r.image, self.targets[f:f + 1], self.sse)
            mse = float(self.sse.item()) / r.image.numel()
            vals.append(-10.0 * math.log10(max(mse, 1e-20)))
        return float(np.mean(vals))


class GroupTrainer:
    """Batched training: the training frames are split (seeded) into fixed
    groups of `group` frames; each step renders one group in one launch per
    stage (persistent, largest tiles first), applies L1 + w (1 - SSIM) over
    the group's images, back-propagates through all views at once and takes
    one Adam step.  Each group's step is captured as three HIP graphs."""

    def __init__(self, params, views, targets, frames, group=8, budget=5000, ssim_weight=0.2,
                 seed=0, lrs=None, batch=256):
        self.params = params.contiguous()
        dev = self.params.device
        self.n = self.params.shape[1]
        self.views = np.atleast_2d(views)
        rng = np.random.default_rng(seed)
        order = list(rng.permutation(list(frames)))
        while len(order) % group:
            order.append(order[len(order) % len(frames)])
        self.groups = [order[i:i + group] for i in range(0, len(order), group)]
        self.targets = [targets[g].contiguous() for g in self.groups]
        self.V = group
        self.rast = Rasterizer(self.n, self.views[self.groups[0]], device=dev, batch=batch,
                               persistent=True)
        H, W = self.rast.H, self.rast.W
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=dev)
        self.cfg = adam_config(budget, lrs)
        self.ssim_w = float(ssim_weight)
        self.dimg = torch.zeros((group, 3, H, W), device=dev)
        self.loss = torch.zeros(1, device=dev)
        self.ws = torch.zeros(G.gs4d_photometric_loss_workspace_size(group, 3, H, W),
                              dtype=torch.uint8, device=dev)
        self.overflow_seen = torch.zeros(1, dtype=torch.int32, device=dev)
        self.cviews = [G.make_views(self.views[g]) for g in self.groups]
        self.graphs = None

    def size_pairs(self, margin=1.5):
        peak = 0
        for k in range(len(self.groups)):
            self.rast.set_views(self.cviews[k])
            self.rast.preprocess(self.params)
            self.rast.bin_sort(check=True)
            peak = max(peak, int(self.rast.n_pairs.item()))
        cap = int(peak * margin) + 4096
        if cap > self.rast.capacity:
            self.rast._alloc_pairs(cap)
        return peak

    def stage_forward(self, k):
        r = self.rast
        r.set_views(self.cviews[k])
        r.preprocess(self.params)
        r.bin_sort(check=False)
        r.render()
        G.gs4d_photometric_loss(r.image, self.targets[k], 1.0, self.ssim_w, self.loss, self.dimg,
                                self.ws)
        torch.maximum(self.overflow_seen, r.overflow, out=self.overflow_seen)

    def stage_render_bwd(self, k):
        self.rast.render_bwd_2d(self.dimg)

    def stage_update(self, k):
        r = self.rast
        G.gs4d_preprocess_bwd(self.params, r.touched, r.grad2d, self.cviews[k], r.dparams)
        G.gs4d_adam_step(self.params, r.dparams, self.m, self.v, self.cfg, self.step_dev)

    def step(self, k):
        self.stage_forward(k)
        self.stage_render_bwd(k)
        self.stage_update(k)

    def capture(self, groups=None):
        """Capture every group's step as one HIP graph (the argument is
        accepted for symmetry with Trainer.capture and ignored)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        self.graphs = [_capture(lambda k=k: self.step(k), side) for k in range(len(self.groups))]
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()

    def step_graph(self, k):
        self.graphs[k].replay()


def run(trainer, schedule, evaluator, eval_every, budget, graph=True, target_psnr=None,
        log=None):
    """Run `budget` steps of `trainer` over the index sequence `schedule`
    (frame or group per step), evaluating every `eval_every` steps.
    Returns the history [(step, train wall seconds, psnr)] and, with
    target_psnr, the first (step, seconds) at which it was reached."""
    hist = []
    reached = None
    wall = 0.0
    done = 0
    if graph:
        trainer.capture(sorted(set(int(k) for k in schedule)))
    while done < budget:
        todo = min(eval_every, budget - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(done, done + todo):
            k = schedule[i % len(schedule)]
            if graph:
                trainer.step_graph(k)
            else:
                trainer.step(k)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        done += todo
        if int(trainer.overflow_seen.item()) != 0:
            raise RuntimeError("pair capacity overflowed during training")
        p = evaluator.psnr(trainer.params)
        hist.append((done, wall, p))
        if log:
            log(f"step {done}: {wall:.2f} s, PSNR {p:.3f}")
        if target_psnr is not None and reached is None and p >= target_psnr:
            reached = (done, wall)
            break
    return hist, reached


def plain_schedule(train_frames, budget, seed=0):
    rng = np.random.default_rng(seed)
    return [int(f) for f in rng.choice(train_frames, budget)]


def group_schedule(n_groups, budget, seed=0):
    """Each group once per epoch, in a fresh seeded order every epoch."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < budget:
        out.extend(int(k) for k in rng.permutation(n_groups))
    return out[:budget]


def batched_lrs(lr_mult=1.0, decay=1.0):
    """Learning rates of the batched form: the single-view rates times
    lr_mult (a step sees `group` frames), every rate decayed exponentially by
    `decay` over the budget (the position rate keeps its own 100x decay)."""
    from .train import LR_DEFAULTS
    return {k: (v[0] * lr_mult, v[1] * lr_mult * (1.0 if k.startswith("mean") else decay))
            for k, v in LR_DEFAULTS.items()}


def batched_run(params0, views, images, train_frames, evaluator, budget, lr_mult=1.0, group=8,
                eval_every=25, target_psnr=None, seed=0, log=None, decay=1.0):
    """Batched training from params0; returns (history, reached, trainer)."""
    lrs = batched_lrs(lr_mult, decay)
    tr = GroupTrainer(params0.clone(), views, images, train_frames, group=group, budget=budget,
                      lrs=lrs, seed=seed)
    tr.size_pairs(margin=1.6)
    hist, reached = run(tr, group_schedule(len(tr.groups), budget, seed), evaluator, eval_every,
                        budget, target_psnr=target_psnr, log=log)
    return hist, reached, tr


# Batched-form settings chosen on validation scenes 950-951 (neither training
# scenes of the network nor test scenes) for the time to reach the plain
# form's PSNR, over frames per step 2-16, rate multipliers 2-16, decays
# 0.01-0.1 and budgets 600-2500: four frames per step, rates x6, all decayed
# to 0.03x over at most 1,500 steps (larger groups need more frame-iterations,
# x16 diverges, short budgets miss the target).
BATCHED_GROUP, BATCHED_LR_MULT, BATCHED_DECAY, BATCHED_BUDGET = 4, 6.0, 0.03, 1500
# Eight frames per step (the many-view launch of the batched configuration):
# rates x9 decayed to 0.01x, chosen on the same validation scenes from
# multipliers 6 / 9 / 12 and decays 0.03 / 0.01.
BATCHED8_LR_MULT, BATCHED8_DECAY = 9.0, 0.01


def time_to_psnr(sc, images, params0, pruned, model=None, plain_budget=5000,
                 budget=BATCHED_BUDGET, lr_mult=BATCHED_LR_MULT, decay=BATCHED_DECAY,
                 group=BATCHED_GROUP,
                 seed=0, log=None, classes=None):
    """The plain single-view form (heuristic init, `plain_budget` steps) fixes
    the reference PSNR on the held-out frames; the batched form from the
    heuristic and from the learned initialisation then trains until it is
    within 0.1 dB of it (or `budget` steps).  Wall times exclude evaluation
    and scene synthesis; the learned initialisation's own time (neighbours,
    features, network, rotor map; measured after one untimed call, so
    without the process's first kernel loads) is added to its run."""
    from . import learned_init as LI
    train_f, held_f = split_frames(sc.frames)
    ev = Evaluator(params0.shape[1], sc.cams, images, held_f)
    tr = Trainer(params0.clone(), sc.cams, images, budget=plain_budget)
    tr.size_pairs(train_f[::9], margin=2.0)
    hist_p, _ = run(tr, plain_schedule(train_f, plain_budget, seed), ev, plain_budget // 10,
                    plain_budget, log=log)
    ref = hist_p[-1][2]
    plain_s = hist_p[-1][1]
    del tr
    target = ref - 0.1
    out = dict(psnr_ref=round(ref, 3), plain_steps=plain_budget, plain_s=round(plain_s, 3),
               target_psnr=round(target, 3), batched=dict(group=group, lr_mult=lr_mult,
                                                          decay=decay, max_steps=budget))
    runs = {"heuristic": params0}
    if model is not None:
        # once untimed: the first launches of a process load the kernels'
        # code objects; the timed call is the per-scene cost
        LI.apply(params0.clone(), pruned, model, classes=classes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p_l = LI.apply(params0.clone(), pruned, model, classes=classes)
        torch.cuda.synchronize()
        out["learned_init_s"] = round(time.perf_counter() - t0, 4)
        runs["learned"] = p_l
    for name, p in runs.items():
        # held-out PSNR every 10 steps (~20 ms of training): the crossing is
        # located to that resolution; evaluation time is not counted
        hist, reached, _ = batched_run(p, sc.cams, images, train_f, ev, budget, lr_mult, group,
                                       eval_every=10, target_psnr=target, seed=seed, log=log,
                                       decay=decay)
        extra = out.get("learned_init_s", 0.0) if name == "learned" else 0.0
        out[name] = dict(
            psnr_init=round(ev.psnr(p), 3),
            reached=reached is not None,
            steps=(reached[0] if reached else None),
            seconds=(round(reached[1] + extra, 3) if reached else None),
            best_psnr=round(max(h[2] for h in hist), 3),
            speedup=(round(plain_s / (reached[1] + extra), 2) if reached else None),
            history=[(a, round(b, 3), round(c, 3)) for a, b, c in hist])
        torch.cuda.empty_cache()
    return out


def init_gain(sc, images, params0, pruned, model, budget=300, lr_mult=2.0, group=8, seed=0,
              decay=1.0, classes=None):
    """PSNR after a fixed batched budget from the heuristic and from the
    learned initialisation."""
    from . import learned_init as LI
    train_f, held_f = split_frames(sc.frames)
    ev = Evaluator(params0.shape[1], sc.cams, images, held_f)
    res = {}
    for name, p in (("heuristic", params0),
                    ("learned", LI.apply(params0.clone(), pruned, model, classes=classes))):
        hist, _, _ = batched_run(p, sc.cams, images, train_f, ev, budget, lr_mult, group,
                                 eval_every=budget // 3, seed=seed, decay=decay)
        res[name] = dict(psnr_init=round(ev.psnr(p), 3), psnr=[round(h[2], 3) for h in hist])
    return res
