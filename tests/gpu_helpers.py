"""Shared helpers for the GPU parity tests (run the HIP path, compare with
the oracle, classify threshold-adjacent pixels)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

ALPHA_MIN = 1.0 / 255.0


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_01119_amd import gs4d
    gs4d.lib()


def gpu_forward(params_np, views, batch=256, capacity=None, count_blends=False):
    from paper_2510_01119_amd.rasterizer import Rasterizer
    p = torch.from_numpy(np.ascontiguousarray(params_np, np.float32)).cuda()
    r = Rasterizer(p.shape[1], views, pair_capacity=capacity, batch=batch, count_blends=count_blends)
    r.forward(p)
    torch.cuda.synchronize()
    return r, p


def to_np(r):
    P = int(r.n_pairs.item())
    out = dict(
        rec=r.rec.cpu().numpy(), rect=r.rect.cpu().numpy(), touched=r.touched.cpu().numpy(),
        keys=r.keys[:P].cpu().numpy().view(np.uint64), vals=r.vals[:P].cpu().numpy().view(np.uint32),
        ranges=r.ranges.cpu().numpy(), image=r.image.cpu().numpy(), T_final=r.T_final.cpu().numpy(),
        last=r.last.cpu().numpy(), n_pairs=P)
    if r.counters is not None:
        c = r.counters.cpu().numpy()
        out["n_eval"], out["n_blend"] = int(c[0]), int(c[1])
    return out


def near_threshold_pixels(rec64, views, vals, ranges, rtol=1e-5, return_tainted=False,
                          taint="pixel"):
    """Boolean [V, H, W]: pixels where some entry's FP64 alpha lies within
    the FP32 evaluation error of 1/255 or 0.99, its exponent within that
    error of 0, or the transmittance test within it of 1e-4.  Such pixels
    may legitimately differ between an FP32 and an FP64 render.

    The FP32 error of the exponent -(a dx^2 + c dy^2)/2 - b dx dy is bounded
    by a few units of roundoff times the sum of its terms' magnitudes S (the
    terms can cancel for thin splats, so S can be much larger than the
    exponent); exp turns that absolute error into the same relative error of
    alpha.  Transmittance after n blends carries about 2n roundoffs.  rtol
    covers the exp approximation and the rest.

    With return_tainted, also a boolean per Gaussian: its gradient may
    differ between the two renders.
      taint="pixel": every Gaussian that reaches alpha >= 1/255 (less the
        tolerance) at such a pixel before it stops.
      taint="entry": only the entries whose own decision is in doubt: an
        alpha or clamp decision next to its threshold taints that entry (a
        1/255 blend that flips changes the others' terms at that pixel by
        about 0.4%); a transmittance stop next to 1e-4 taints the stopping
        entry and the next two blends it would have allowed (their weights
        are ~1e-4); an exponent next to 0 (blend at full alpha or skip)
        taints every later entry at that pixel up to its stop and 64 blends
        past it."""
    u = 2.0 ** -24
    views = np.atleast_2d(views)
    V = views.shape[0]
    n = rec64.shape[1]
    W, H = int(views[0, 16]), int(views[0, 17])
    tx, ty = (W + 15) // 16, (H + 15) // 16
    flag = np.zeros((V, H, W), bool)
    tainted = np.zeros(n, bool)
    ys, xs = np.mgrid[0:16, 0:16]
    for v in range(V):
        for tile_y in range(ty):
            for tile_x in range(tx):
                tile = v * tx * ty + tile_y * tx + tile_x
                b, e = ranges[tile]
                if e <= b:
                    continue
                px = tile_x * 16 + xs + 0.5
                py = tile_y * 16 + ys + 0.5
                y0, x0 = tile_y * 16, tile_x * 16
                hh, ww = min(16, H - y0), min(16, W - x0)
                inside = np.zeros((16, 16), bool)
                inside[:hh, :ww] = True
                T = np.ones((16, 16))
                nb = np.zeros((16, 16))
                near = np.zeros((16, 16), bool)
                alive = np.ones((16, 16), bool)
                pending = np.zeros((16, 16), np.int64)   # entry mode: blends still tainted
                wide = np.zeros((16, 16), bool)          # entry mode: exponent next to 0
                alphas = []
                for k in range(b, e):
                    r = rec64[v, vals[k]]
                    dx, dy = px - r[0], py - r[1]
                    power = -0.5 * (r[2] * dx * dx + r[4] * dy * dy) - r[3] * dx * dy
                    S = 0.5 * (abs(r[2]) * dx * dx + abs(r[4]) * dy * dy) + abs(r[3] * dx * dy)
                    tol = rtol + 8.0 * u * S
                    at = r[5] * np.exp(np.minimum(power, 0.0))
                    a = np.minimum(0.99, at)
                    reach = a >= ALPHA_MIN * (1 - tol)
                    own = alive & ((np.abs(a - ALPHA_MIN) <= tol * ALPHA_MIN)
                                   | (np.abs(at - 0.99) <= tol * 0.99))
                    zero = alive & (np.abs(power) <= 8.0 * u * S + 1e-6)
                    near |= own | zero
                    ok = alive & (power <= 0) & (a >= ALPHA_MIN)
                    Tn = T * (1 - a)
                    stop_near = ok & (np.abs(Tn - 1e-4) <= (rtol + 4.0 * u * (nb + 1)) * 1e-4)
                    near |= stop_near
                    if taint == "entry" and return_tainted:
                        wide |= zero
                        hit = inside & (own | stop_near | (wide & reach) | ((pending > 0) & reach))
                        if hit.any():
                            tainted[vals[k]] = True
                        pending = np.where((pending > 0) & reach, pending - 1, pending)
                        pending = np.where(stop_near, 2, pending)
                    else:
                        alphas.append((a, tol, alive.copy()))
                    stop = ok & (Tn < 1e-4)
                    if taint == "entry" and return_tainted:
                        # an exponent next to 0 changes this pixel's transmittance by a
                        # factor up to 100: the other render stops up to ~64 blends later
                        pending = np.where(wide & stop, 64, pending)
                        wide &= ~stop
                    alive &= ~stop
                    blend = ok & ~stop
                    T = np.where(blend, Tn, T)
                    nb += blend
                    if not alive.any() and not (taint == "entry" and ((pending > 0) | wide).any()):
                        break
                near &= inside
                flag[v, y0:y0 + hh, x0:x0 + ww] = near[:hh, :ww]
                if return_tainted and taint == "pixel" and near.any():
                    for k, (a, tol, live) in zip(range(b, e), alphas):
                        if np.any(near & live & (a >= ALPHA_MIN * (1 - tol))):
                            tainted[vals[k]] = True
    if return_tainted:
        return flag, tainted
    return flag
