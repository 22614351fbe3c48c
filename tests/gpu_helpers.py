"""Shared helpers for the GPU parity tests (run the HIP path, compare with
the oracle, classify threshold-adjacent pixels)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle

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


def near_threshold_pixels(rec64, views, vals, ranges):
    """Boolean [V, H, W]: pixels with a decision an FP32 kernel render may
    take the other way from the oracle's FP32 shadow
    (oracle.doubtful_decisions)."""
    return oracle.doubtful_decisions(rec64, views, vals, ranges)[0]


def decision_bounds(params, views, rec64, vals, ranges, dL_dimage, iso=False, chain=None):
    """What each doubtful decision can change, computed by the oracle: the
    pixel re-composited with that one decision inverted, against the pixel as
    the oracle takes it (its decisions taken on the FP32 shadow of the
    kernel's arithmetic; oracle.doubtful_decisions lists the ones the
    kernel's hardware exp2 may take the other way).  Returns (flag [V, H, W], img [V, H, W]: the summed
    change of the pixel's colour (max over channels), T [V, H, W]: of its
    final transmittance, grad [F, n]: the summed |change| of each
    parameter's gradient, chained through the preprocess backward (FP64)).
    An FP32 render that takes any of these decisions the other way differs
    from the oracle by at most these amounts (plus its own rounding).
    chain(v, g [1, n, 9]) -> [F, n], if given, is the (linear) chain rule
    from view v's record gradient to the parameters, in place of the rotor
    or isotropic preprocess backward."""
    views = np.atleast_2d(views)
    V, n, _ = rec64.shape
    flag, found = oracle.doubtful_decisions(rec64, views, vals, ranges)
    H, W = flag.shape[1:]
    img = np.zeros((V, H, W))
    Tb = np.zeros((V, H, W))
    if chain is None:
        bwd = oracle.preprocess_iso_bwd if iso else oracle.preprocess_bwd

        def chain(v, g):
            return bwd(params.astype(np.float64), views[v:v + 1], g)
    F = chain(0, np.zeros((1, n, 9))).shape[0]
    grad = np.zeros((F, n))
    if not found:
        return flag, img, Tb, grad
    tx, ty = (W + 15) // 16, (H + 15) // 16
    # the preprocess backward is linear in the record gradient: its
    # columns per view, from one call per record term
    J = {}
    for v in sorted({f[0] for f in found}):
        cols = []
        for j in range(9):
            g = np.zeros((1, n, 9))
            g[0, :, j] = 1.0
            cols.append(chain(v, g))
        J[v] = np.stack(cols)                       # [9, F, n]
    base = {}
    for v, x, y, e, kind in found:
        gC = dL_dimage[v, :, y, x].astype(np.float64)
        key = (v, x, y)
        if key not in base:
            base[key] = oracle.pixel_variant(rec64, views, v, vals, ranges, x, y, gC,
                                             f32=True)
        C0, T0, g0, _ = base[key]
        C1, T1, g1, _ = oracle.pixel_variant(rec64, views, v, vals, ranges, x, y, gC, e, kind,
                                             f32=True)
        img[v, y, x] += np.abs(C1 - C0).max()
        Tb[v, y, x] += abs(T1 - T0)
        dg = g1 - g0
        rows = np.nonzero(np.any(dg != 0, axis=1))[0]
        if len(rows) == 0:
            continue
        b = int(ranges[v * tx * ty + (y // 16) * tx + (x // 16)][0])
        ids = np.asarray(vals)[b + rows].astype(np.int64)
        grad[:, ids] += np.abs(np.einsum("jfk,kj->fk", J[v][:, :, ids], dg[rows]))
    return flag, img, Tb, grad


def report_exempt(name, near, widened=None, contributing=None):
    """Prints (and returns) the fraction of pixels with a doubtful decision
    and, with `widened`, the fraction of the Gaussians (of `contributing`
    ones if given) whose gradient bar the decision bounds widen."""
    out = {"pixels": float(np.mean(near))}
    if widened is not None:
        base = contributing if contributing is not None else np.ones_like(widened)
        out["gaussians_widened"] = float(widened[base].mean()) if base.any() else 0.0
        out["n_widened"] = int(widened[base].sum())
    print(f"doubtful[{name}]: " + ", ".join(f"{k}={v:.3g}" if isinstance(v, float) else f"{k}={v}"
                                           for k, v in out.items()), flush=True)
    return out


def check_image(name, img_gpu, img_ref, flag, img_bound, max_pixels=1e-3):
    """Image parity: every pixel within 1e-4 absolute of the oracle, plus, at
    a pixel with a doubtful decision, what inverting it changes."""
    report_exempt(name, flag)
    assert flag.mean() <= max_pixels, flag.mean()
    diff = np.abs(img_gpu - img_ref).max(axis=1)
    lim = 1e-4 + img_bound
    worst = np.unravel_index(np.argmax(diff / lim), diff.shape)
    assert np.all(diff <= lim), (name, worst, float(diff[worst]), float(lim[worst]))


def splat_condition(rec, touched, params=None, views=None):
    """Per Gaussian: the largest condition number, over the views where it
    is visible, of its 2D covariance (from the FP32 record's conic) and --
    with params and views -- of its conditional 3D covariance at the view's
    time (FP64 oracle).  A needle-shaped covariance (kappa ~ 1e5) cannot
    hold its thin direction in FP32 to better than u kappa, so neither can
    an FP32 chain rule through it."""
    r = rec.astype(np.float64)
    a, b, c = r[..., 2], r[..., 3], r[..., 4]
    half_tr = 0.5 * (a + c)
    disc = np.sqrt(np.maximum(half_tr * half_tr - (a * c - b * b), 0.0))
    lo = half_tr - disc
    kappa = np.where((touched > 0) & (lo > 0), (half_tr + disc) / np.where(lo > 0, lo, 1.0), 1.0)
    if params is not None:
        for v, view in enumerate(np.atleast_2d(views)):
            ev = np.linalg.eigvalsh(oracle.conditional_cov_all(params, float(view[18])))
            k3 = np.where(ev[:, 0] > 0, ev[:, 2] / np.where(ev[:, 0] > 0, ev[:, 0], 1.0), 1.0)
            kappa[v] = np.maximum(kappa[v], np.where(touched[v] > 0, k3, 1.0))
    return kappa.max(axis=0)


def check_gradients(name, d, ref, bound, max_widened=0.01, max_rel=0.02, max_outliers=0.0,
                    kappa=None, kappa_max=1e3, max_needles=0.0):
    """Gradient parity: every entry within 1e-3 relative of the oracle (floor:
    1e-3 of the parameter class's largest magnitude) plus the oracle-computed
    change its doubtful decisions can make (`bound`, decision_bounds).  The
    Gaussians whose bar that widens (bound above the 1e-3 bar) are counted,
    printed and held to `max_widened` of those with a gradient; no bar may
    widen beyond `max_rel` of max(|g|, floor).

    max_outliers > 0 (the densest cases only): that fraction of the checked
    (parameter, Gaussian) entries may exceed the bar -- FP32 rounding of the
    transmittance behind alphas near 0.99, summed over hundreds of pixels
    with cancelling signs -- but none by more than 10x; they are counted and
    printed.

    kappa (per Gaussian, splat_condition): Gaussians whose 2D or conditional
    3D covariance has a condition number above kappa_max are needles whose
    FP32 chain rule the problem itself makes unreliable (their derivatives
    cancel terms ~kappa times larger); they are left out of the bar, counted
    (at most `max_needles` of those with a gradient) and their measured
    error printed."""
    contributing = np.any(ref != 0, axis=0)
    needle = np.zeros(ref.shape[1], bool) if kappa is None else kappa > kappa_max
    checked_g = contributing & ~needle
    widened = np.zeros(ref.shape[1], bool)
    worst_rel = 0.0
    over, over_max, checked = 0, 0.0, 0
    needle_err = []
    for k in range(ref.shape[0]):
        floor = 1e-3 * np.abs(ref[k]).max()
        mag = np.maximum(np.abs(ref[k]), floor)
        err = np.abs(d[k] - ref[k])
        tol = 1e-3 * mag + 1e-7
        widened |= bound[k] > tol
        lim = tol + bound[k]
        ratio = np.where(needle, 0.0, err / lim)
        checked += int(checked_g.sum())
        over += int((ratio > 1.0).sum())
        over_max = max(over_max, float(ratio.max()) if ratio.size else 0.0)
        if needle.any():
            needle_err.append(err[needle & contributing] / mag[needle & contributing])
        if max_outliers <= 0.0:
            worst = int(np.argmax(ratio))
            assert np.all(ratio <= 1.0), (name, k, worst, int((ratio > 1.0).sum()), err[worst],
                                          tol[worst], bound[k][worst], ref[k][worst])
        if ref.shape[1]:
            worst_rel = max(worst_rel, float(np.max(bound[k] / np.maximum(np.abs(ref[k]), floor + 1e-30))))
    rep = report_exempt(name, np.zeros(1, bool), widened, contributing)
    rep.update(widest_bar_rel=worst_rel, over_bar=over, worst_over_bar=over_max)
    print(f"parity[{name}]: widest bound relative to max(|g|, floor) = {worst_rel:.3g}; "
          f"entries over the bar {over} of {checked} (worst {over_max:.3g}x)", flush=True)
    n_needle = int((needle & contributing).sum())
    rep["needles"] = n_needle / max(int(contributing.sum()), 1)
    if kappa is not None:
        e = np.concatenate(needle_err) if needle_err else np.zeros(0)
        pct = np.percentile(e, [50, 90, 100]) if e.size else np.zeros(3)
        print(f"parity[{name}]: needles (kappa > {kappa_max:g}) left out: {n_needle} of "
              f"{int(contributing.sum())} Gaussians (max kappa {float(kappa.max()):.3g}); their error "
              f"relative to max(|g|, floor): median {pct[0]:.3g}, 90% {pct[1]:.3g}, max {pct[2]:.3g}",
              flush=True)
    assert rep["gaussians_widened"] <= max_widened, rep
    assert worst_rel <= max_rel, rep
    assert over <= max_outliers * checked and over_max <= 10.0, rep
    assert rep["needles"] <= max_needles, rep
    return rep
