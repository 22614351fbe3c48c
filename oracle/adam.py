"""TEST INFRASTRUCTURE: plain numpy Adam (Kingma & Ba 2015) with bias
correction and per-parameter-group learning rates.

The paper keeps the 3D Gaussian splatting optimiser settings except the
position learning rate, lowered to 1e-5, with the learning-rate schedule
stretched to the iteration budget (Sec. 4.1).  The schedule is read as the
exponential decay of 3D Gaussian splatting, lr(s) = lr0^(1-u) lr1^u with
u = s / budget (clamped to [0, 1]).
"""
from __future__ import annotations

import numpy as np


def lr_schedule(step, lr0, lr1, budget):
    u = min(max(step / max(budget, 1), 0.0), 1.0)
    return float(np.exp(np.log(lr0) * (1 - u) + np.log(lr1) * u))


def adam_step(param, grad, m, v, step, lr_per_row, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (step counts from 1).  lr_per_row: [rows] learning rate
    of each parameter row.  Returns updated (param, m, v) in FP64."""
    p = np.asarray(param, np.float64)
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    lr = np.asarray(lr_per_row, np.float64)[:, None]
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
