"""TEST INFRASTRUCTURE: one process of the benchmark's CPU baseline -- the
oracle's training step (FP32-decided preprocess, FP64 compositing and chain
rule, numpy L1 + 0.2 (1 - SSIM) and Adam) run as it stands, on one host
core, repeatedly on one frame until a time budget is spent.  The benchmark
starts one such process per host core it may use and reports their summed
rate.

usage: python -m oracle.bench_worker DIR FRAME BUDGET_S
DIR holds params.npy (float32 [20, N]), views.npy ([F, 23]) and
targets.npy ([F, 3, H, W]); prints one JSON line {"steps", "seconds"}.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from oracle import adam as oadam  # noqa: E402
from oracle import losses as olosses  # noqa: E402

LRS = [1e-5] * 4 + [5e-3] * 4 + [1e-3] * 8 + [5e-2] + [2.5e-3] * 3


def main():
    d, frame, budget = sys.argv[1], int(sys.argv[2]), float(sys.argv[3])
    p = np.load(os.path.join(d, "params.npy")).astype(np.float64)
    views = np.load(os.path.join(d, "views.npy"))
    targets = np.load(os.path.join(d, "targets.npy"))
    view, target = views[frame % len(views)], targets[frame % len(targets)]
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    t0 = time.perf_counter()
    steps = 0
    while True:
        fwd = oracle.forward(p.astype(np.float32), view, "f32")
        _, g = olosses.scene_loss(fwd["image"][0], target)
        d_p, _ = oracle.backward(p.astype(np.float32), view, g[None], fwd=fwd)
        p, m, v = oadam.adam_step(p, d_p, m, v, steps + 1, LRS)
        steps += 1
        if time.perf_counter() - t0 >= budget:
            break
    print(json.dumps({"steps": steps, "seconds": time.perf_counter() - t0}), flush=True)


if __name__ == "__main__":
    main()
