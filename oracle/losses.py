"""TEST INFRASTRUCTURE: plain numpy losses of the optimisation loop (FP64).

The method optimises a single photometric loss with the loss weights of
3D Gaussian splatting (Sec. 4.1, implementation details; Sec. B
"Discussion with previous work").  Readings:
  * L1 = mean |C - C*| over pixels and channels;
  * SSIM (Wang et al. 2004): 11x11 Gaussian window, sigma 1.5, C1 = 0.01^2,
    C2 = 0.03^2, zero-padded 'same' windows, mean over pixels and channels,
    computed here by direct 2D windowed sums (no separable filtering);
  * scene-scale loss = L1 + 0.2 (1 - SSIM);
  * PSNR = -10 log10(MSE) for images in [0, 1].
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2


def gaussian_window(size=11, sigma=1.5):
    x = np.arange(size) - size // 2
    g = np.exp(-(x ** 2) / (2 * sigma ** 2))
    g /= g.sum()
    return np.outer(g, g)


def _window_sum(img, win):
    """Zero-padded 'same' windowed sum: out[y, x] = sum_{u,v} win[u, v] img[y+u-r, x+v-r]."""
    H, W = img.shape
    r = win.shape[0] // 2
    pad = np.zeros((H + 2 * r, W + 2 * r))
    pad[r:r + H, r:r + W] = img
    out = np.zeros((H, W))
    for u in range(win.shape[0]):
        for v in range(win.shape[1]):
            out += win[u, v] * pad[u:u + H, v:v + W]
    return out


def l1(img, target):
    img = np.asarray(img, np.float64)
    d = img - np.asarray(target, np.float64)
    return np.abs(d).mean(), np.sign(d) / d.size


def ssim_map(img, target):
    """Per-pixel SSIM map [C, H, W]."""
    x = np.asarray(img, np.float64)
    y = np.asarray(target, np.float64)
    win = gaussian_window()
    out = np.zeros_like(x)
    for c in range(x.shape[0]):
        mx = _window_sum(x[c], win)
        my = _window_sum(y[c], win)
        sxx = _window_sum(x[c] * x[c], win) - mx * mx
        syy = _window_sum(y[c] * y[c], win) - my * my
        sxy = _window_sum(x[c] * y[c], win) - mx * my
        out[c] = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
    return out


def ssim(img, target, want_grad=True):
    """Mean SSIM of img [C, H, W] against target, and d mean-SSIM / d img."""
    x = np.asarray(img, np.float64)
    y = np.asarray(target, np.float64)
    win = gaussian_window()
    total = 0.0
    grad = np.zeros_like(x)
    n = x.size
    for c in range(x.shape[0]):
        mx = _window_sum(x[c], win)
        my = _window_sum(y[c], win)
        exx = _window_sum(x[c] * x[c], win)
        eyy = _window_sum(y[c] * y[c], win)
        exy = _window_sum(x[c] * y[c], win)
        sxx = exx - mx * mx
        syy = eyy - my * my
        sxy = exy - mx * my
        A1 = 2 * mx * my + C1
        A2 = 2 * sxy + C2
        B1 = mx * mx + my * my + C1
        B2 = sxx + syy + C2
        S = (A1 * A2) / (B1 * B2)
        total += S.sum()
        if want_grad:
            dmx = S * (2 * my / A1 - 2 * mx / B1 - 2 * my / A2 + 2 * mx / B2)
            dexx = -S / B2
            dexy = 2 * S / A2
            # adjoint of a symmetric zero-padded window sum is the same window sum
            grad[c] = (_window_sum(dmx, win) + 2 * x[c] * _window_sum(dexx, win)
                       + y[c] * _window_sum(dexy, win)) / n
    return total / n, grad


def scene_loss(img, target, w_ssim=0.2):
    """L1 + w (1 - SSIM) and its gradient."""
    lv, lg = l1(img, target)
    sv, sg = ssim(img, target)
    return lv + w_ssim * (1 - sv), lg - w_ssim * sg


def psnr(img, target):
    mse = np.mean((np.asarray(img, np.float64) - np.asarray(target, np.float64)) ** 2)
    return -10.0 * np.log10(mse)
