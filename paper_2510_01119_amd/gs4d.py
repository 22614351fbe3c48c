"""Thin ctypes binding of libgs4d.so.

Every function here has the name of the C entry point it wraps and does
argument marshalling only: torch tensors become device pointers, numpy view
arrays become ``gs4d_view`` structs, and a non-zero status raises
``GS4DError`` with the library's message.  All arithmetic happens in the
HIP kernels.  There is no fallback: if the library is missing, loading
fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs4d.so")

N_FIELDS = 20
ISO_FIELDS = 13   # isotropic, motion-aware parameterisation (gs4d_preprocess_iso)
REC_FLOATS = 12
GRAD2D_FLOATS = 9
TILE = 16
MAX_VIEWS = 16
RENDER_GRAD2D_ZEROED = 1   # gs4d_render_opts.flags


class GS4DError(RuntimeError):
    pass


class gs4d_view(ctypes.Structure):
    _fields_ = [("Rt", ctypes.c_float * 12), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("t", ctypes.c_float), ("near_z", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("reserved", ctypes.c_int32)]


class gs4d_render_opts(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("n_workgroups", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("target", ctypes.c_void_p), ("l1_weight", ctypes.c_float),
                ("loss_per_view", ctypes.c_void_p), ("dL_dimage", ctypes.c_void_p),
                ("counters", ctypes.c_void_p), ("order", ctypes.c_void_p),
                ("queue", ctypes.c_void_p)]


class gs4d_sch(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("n_freq", ctypes.c_int32), ("period", ctypes.c_float),
                ("reserved", ctypes.c_int32)]


def make_sch(degree: int, n_freq: int, period: float) -> gs4d_sch:
    s = gs4d_sch()
    s.degree, s.n_freq, s.period, s.reserved = int(degree), int(n_freq), float(period), 0
    return s


class gs4d_adam_cfg(ctypes.Structure):
    _fields_ = [("lr0", ctypes.c_float * N_FIELDS), ("lr1", ctypes.c_float * N_FIELDS),
                ("budget", ctypes.c_int32), ("rows", ctypes.c_int32), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_f32 = ctypes.c_float
_sz = ctypes.c_size_t

_SIGS = {
    "gs4d_preprocess": (_i32, [_p, _i64, _p, _i32, _p, _p, _p, _p]),
    "gs4d_bin_sort_workspace_size": (_sz, [_i64, _i32, _i64]),
    "gs4d_bin_sort": (_i32, [_p, _p, _p, _i64, _p, _i32, _i64, _p, _p, _p, _p, _p, _p, _sz, _p]),
    "gs4d_bin_sort_noalloc": (_i32, [_p, _p, _p, _i64, _p, _i32, _i64, _p, _p, _p, _p, _p, _p]),
    "gs4d_render_fwd": (_i32, [_p, _i64, _p, _p, _p, _i32, _p, _p, _p, _p, _p]),
    "gs4d_render_bwd_workspace_size": (_sz, [_i64, _i32]),
    "gs4d_render_bwd": (_i32, [_p, _i64, _p, _p, _p, _p, _p, _i32, _p, _p, _p, _p, _p, _p, _p, _sz,
                               _p]),
    "gs4d_render_bwd_2d": (_i32, [_p, _i64, _p, _p, _p, _i32, _p, _p, _p, _p, _p, _p]),
    "gs4d_tile_order_workspace_size": (_sz, [_i64]),
    "gs4d_tile_order": (_i32, [_p, _i64, _p, _p, _i32, _p, _sz, _p]),
    "gs4d_preprocess_bwd": (_i32, [_p, _i64, _p, _i32, _p, _p, _p, _p]),
    "gs4d_preprocess_iso": (_i32, [_p, _i64, _p, _i32, _p, _p, _p, _p]),
    "gs4d_preprocess_iso_bwd": (_i32, [_p, _i64, _p, _i32, _p, _p, _p, _p]),
    "gs4d_sch_rows": (_i64, [_i32, _i32]),
    "gs4d_preprocess_sch": (_i32, [_p, _p, _i64, _p, _p, _i32, _p, _p, _p, _p]),
    "gs4d_preprocess_sch_bwd": (_i32, [_p, _p, _i64, _p, _p, _i32, _p, _p, _p, _p, _p]),
    "gs4d_sch_from_rgb": (_i32, [_p, _i64, _i64, _p, _p, _p]),
    "gs4d_otsu_workspace_size": (_sz, []),
    "gs4d_threshold_mask": (_i32, [_p, _i64, _p, _p, _p]),
    "gs4d_otsu_mask": (_i32, [_p, _i64, _p, _p, _p, _sz, _p]),
    "gs4d_set_bwd_variant": (_i32, [_i32]),
    "gs4d_set_bin_strategy": (_i32, [_i32]),
    "gs4d_grid_prune_workspace_size": (_sz, [_i64, _i32]),
    "gs4d_grid_prune": (_i32, [_p, _p, _i32, _p, _i64, _f32, _f32, _i32, _i64, _p, _p, _p, _p, _p,
                               _p, _p, _sz, _p]),
    "gs4d_backproject_workspace_size": (_sz, [_i64]),
    "gs4d_backproject": (_i32, [_p, _p, _p, _f32, _i64, _p, _p, _p, _p, _p, _p, _sz, _p]),
    "gs4d_heuristic_init": (_i32, [_p, _p, _p, _p, _p, _i64, _i64, _f32, _f32, _f32, _i32, _p, _p]),
    "gs4d_adam_step": (_i32, [_p, _p, _p, _p, _i64, _p, _p, _p]),
    "gs4d_loss_l1": (_i32, [_p, _p, _i64, _f32, _p, _p, _p]),
    "gs4d_ssim_workspace_size": (_sz, [_i32, _i32, _i32, _i32]),
    "gs4d_ssim": (_i32, [_p, _p, _i32, _i32, _i32, _i32, _f32, _p, _p, _p, _sz, _p]),
    "gs4d_photometric_loss_workspace_size": (_sz, [_i32, _i32, _i32, _i32]),
    "gs4d_photometric_loss": (_i32, [_p, _p, _i32, _i32, _i32, _i32, _f32, _f32, _p, _p, _p, _sz,
                                     _p]),
    "gs4d_sse": (_i32, [_p, _p, _i64, _p, _p]),
    "gs4d_knn8_workspace_size": (_sz, [_i64]),
    "gs4d_knn8": (_i32, [_p, _i64, _f32, _p, _p, _p, _p, _sz, _p]),
    "gs4d_init_features": (_i32, [_p, _p, _p, _p, _i64, _p, _p, _p, _p]),
    "gs4d_mlp_fwd": (_i32, [_p, _p, _i64, _p, _p]),
    "gs4d_mlp_bwd_workspace_size": (_sz, [_i64]),
    "gs4d_mlp_bwd": (_i32, [_p, _p, _i64, _p, _p, _p, _p, _p, _p, _p, _sz, _p]),
    "gs4d_mlp_adam": (_i32, [_p, _p, _p, _p, _p, _i64, _f32, _f32, _f32, _f32, _p, _p]),
    "gs4d_to_bf16": (_i32, [_p, _p, _i64, _p]),
    "gs4d_motion_init": (_i32, [_p, _p, _i64, _p]),
    "gs4d_motion_of": (_i32, [_p, _i64, _p, _p]),
    "gs4d_fill_f32": (_i32, [_p, _f32, _i64, _p]),
    "gs4d_fill_u32": (_i32, [_p, ctypes.c_uint32, _i64, _p]),
    "gs4d_status_string": (ctypes.c_char_p, [_i32]),
    "gs4d_last_error": (ctypes.c_char_p, []),
    "gs4d_version": (_i32, []),
}

EXPORTED = tuple(_SIGS)
_lib = None


def lib():
    """Load libgs4d.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GS4DError(f"libgs4d.so not found at {LIB_PATH}; run paper_2510_01119_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            if not hasattr(L, name):
                continue
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != 0:
        L = lib()
        raise GS4DError(f"{what}: {L.gs4d_status_string(status).decode()} "
                        f"({L.gs4d_last_error().decode()})")


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if t.numel() > 0 and not t.is_cuda:
            raise GS4DError("expected a device tensor")
        if not t.is_contiguous():
            raise GS4DError("expected a contiguous tensor")
        return ctypes.c_void_p(t.data_ptr()) if t.numel() > 0 else None
    return t


def _ptr_rows(t, rows):
    """Device pointer of `rows` rows of one common stride, each row
    contiguous (a [rows, k] slice of a wider buffer)."""
    if t.numel() > 0 and not t.is_cuda:
        raise GS4DError("expected a device tensor")
    if t.dim() != 2 or t.shape[0] != rows or t.stride(1) != 1:
        raise GS4DError(f"expected [{rows}, k] rows, each contiguous")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() > 0 else None


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_views(views) -> ctypes.Array:
    """numpy [V, 23] (see synth.make_view) -> ctypes array of gs4d_view."""
    v = np.atleast_2d(np.asarray(views, dtype=np.float64))
    arr = (gs4d_view * v.shape[0])()
    for i, row in enumerate(v):
        s = arr[i]
        for k in range(12):
            s.Rt[k] = float(np.float32(row[k]))
        s.fx, s.fy, s.cx, s.cy = (float(np.float32(x)) for x in row[12:16])
        s.width, s.height = int(row[16]), int(row[17])
        s.t = float(np.float32(row[18]))
        s.near_z = float(np.float32(row[19]))
        for k in range(3):
            s.bg[k] = float(np.float32(row[20 + k]))
        s.reserved = 0
    return arr


# ---------------------------------------------------------------- entry points
def gs4d_preprocess(params, views, rec, rect, touched, stream=None):
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    n = params.shape[1]
    _check(lib().gs4d_preprocess(_ptr(params), n, va, len(va), _ptr(rec), _ptr(rect),
                                 _ptr(touched), _stream(stream)), "gs4d_preprocess")


def gs4d_bin_sort_workspace_size(n, n_views, pair_capacity):
    return int(lib().gs4d_bin_sort_workspace_size(n, n_views, pair_capacity))


def gs4d_bin_sort(rec, rect, touched, n, views, pair_capacity, keys, vals, ranges, n_pairs,
                  overflow, ws, stream=None):
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    _check(lib().gs4d_bin_sort(_ptr(rec), _ptr(rect), _ptr(touched), n, va, len(va), pair_capacity,
                               _ptr(keys), _ptr(vals), _ptr(ranges), _ptr(n_pairs), _ptr(overflow),
                               _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)),
           "gs4d_bin_sort")


def gs4d_bin_sort_noalloc(rec, rect, touched, n, views, pair_capacity, keys, vals, ranges, n_pairs,
                          overflow, stream=None):
    """gs4d_bin_sort with the library's own scratch memory (no workspace)."""
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    _check(lib().gs4d_bin_sort_noalloc(_ptr(rec), _ptr(rect), _ptr(touched), n, va, len(va),
                                       pair_capacity, _ptr(keys), _ptr(vals), _ptr(ranges),
                                       _ptr(n_pairs), _ptr(overflow), _stream(stream)),
           "gs4d_bin_sort_noalloc")


def gs4d_render_fwd(rec, n, vals, ranges, views, image, T_final, last, opts=None, stream=None):
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    _check(lib().gs4d_render_fwd(_ptr(rec), n, _ptr(vals), _ptr(ranges), va, len(va),
                                 ctypes.byref(opts) if opts is not None else None, _ptr(image),
                                 _ptr(T_final), _ptr(last), _stream(stream)), "gs4d_render_fwd")


def gs4d_render_bwd_workspace_size(n, n_views):
    return int(lib().gs4d_render_bwd_workspace_size(n, n_views))


def gs4d_render_bwd(params, rec, touched, vals, ranges, views, dL_dimage, T_final, last, dparams,
                    grad2d=None, ws=None, opts=None, stream=None):
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    n = params.shape[1]
    _check(lib().gs4d_render_bwd(_ptr(params), n, _ptr(rec), _ptr(touched), _ptr(vals), _ptr(ranges),
                                 va, len(va), ctypes.byref(opts) if opts is not None else None,
                                 _ptr(dL_dimage), _ptr(T_final), _ptr(last), _ptr(dparams),
                                 _ptr(grad2d), _ptr(ws),
                                 0 if ws is None else ws.numel() * ws.element_size(),
                                 _stream(stream)), "gs4d_render_bwd")


def gs4d_render_bwd_2d(rec, n, vals, ranges, views, dL_dimage, T_final, last, grad2d, opts=None,
                       stream=None):
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    _check(lib().gs4d_render_bwd_2d(_ptr(rec), n, _ptr(vals), _ptr(ranges), va, len(va),
                                    ctypes.byref(opts) if opts is not None else None,
                                    _ptr(dL_dimage), _ptr(T_final), _ptr(last), _ptr(grad2d),
                                    _stream(stream)), "gs4d_render_bwd_2d")


def gs4d_preprocess_bwd(params, touched, grad2d, views, dparams, stream=None):
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    _check(lib().gs4d_preprocess_bwd(_ptr(params), params.shape[1], va, len(va), _ptr(touched),
                                     _ptr(grad2d), _ptr(dparams), _stream(stream)),
           "gs4d_preprocess_bwd")


def gs4d_preprocess_iso(params, views, rec, rect, touched, stream=None):
    """Preprocess of the isotropic, motion-aware parameters [13][n]."""
    assert params.shape[0] == ISO_FIELDS
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    _check(lib().gs4d_preprocess_iso(_ptr(params), params.shape[1], va, len(va), _ptr(rec),
                                     _ptr(rect), _ptr(touched), _stream(stream)),
           "gs4d_preprocess_iso")


def gs4d_preprocess_iso_bwd(params, touched, grad2d, views, dparams, stream=None):
    assert params.shape[0] == ISO_FIELDS
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    _check(lib().gs4d_preprocess_iso_bwd(_ptr(params), params.shape[1], va, len(va),
                                         _ptr(touched), _ptr(grad2d), _ptr(dparams),
                                         _stream(stream)),
           "gs4d_preprocess_iso_bwd")


def gs4d_sch_rows(degree, n_freq):
    return int(lib().gs4d_sch_rows(degree, n_freq))


def _sch_shape(coef, sch, n):
    rows = gs4d_sch_rows(sch.degree, sch.n_freq)
    if tuple(coef.shape) != (rows, n):
        raise GS4DError(f"SCH coefficients must be [{rows}, {n}], got {tuple(coef.shape)}")


def gs4d_preprocess_sch(params, coef, sch, views, rec, rect, touched, stream=None):
    """Preprocess with the SCH colour: rotor-form params [20][n] (rows 17-19
    ignored), coefficients [3 K][n]."""
    _sch_shape(coef, sch, params.shape[1])
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    _check(lib().gs4d_preprocess_sch(_ptr(params), _ptr(coef), params.shape[1], ctypes.byref(sch),
                                     va, len(va), _ptr(rec), _ptr(rect), _ptr(touched),
                                     _stream(stream)), "gs4d_preprocess_sch")


def gs4d_preprocess_sch_bwd(params, coef, sch, touched, grad2d, views, dparams, dcoef,
                            stream=None):
    _sch_shape(coef, sch, params.shape[1])
    _sch_shape(dcoef, sch, params.shape[1])
    va = views if isinstance(views, ctypes.Array) else make_views(views)
    _check(lib().gs4d_preprocess_sch_bwd(_ptr(params), _ptr(coef), params.shape[1],
                                         ctypes.byref(sch), va, len(va), _ptr(touched),
                                         _ptr(grad2d), _ptr(dparams), _ptr(dcoef),
                                         _stream(stream)), "gs4d_preprocess_sch_bwd")


def gs4d_sch_from_rgb(rgb, sch, coef, stream=None):
    """rgb: [3, n] view of a parameter block (row stride rgb.stride(0))."""
    n = rgb.shape[1]
    _sch_shape(coef, sch, n)
    _check(lib().gs4d_sch_from_rgb(_ptr_rows(rgb, 3), rgb.stride(0), n, ctypes.byref(sch), _ptr(coef),
                                   _stream(stream)), "gs4d_sch_from_rgb")


def gs4d_threshold_mask(prob, threshold, mask, stream=None):
    """mask = 1 where bin(prob) >= 256 * threshold (a device float written
    by gs4d_otsu_mask)."""
    assert mask.numel() == prob.numel() and mask.dtype == torch.uint8
    _check(lib().gs4d_threshold_mask(_ptr(prob), prob.numel(), _ptr(threshold), _ptr(mask),
                                     _stream(stream)), "gs4d_threshold_mask")


def gs4d_otsu_workspace_size():
    return int(lib().gs4d_otsu_workspace_size())


def gs4d_otsu_mask(prob, threshold, mask, ws, stream=None):
    """Otsu split of one motion-probability map (float32 device tensor):
    threshold (device float [1] or None), mask (uint8 like prob, or None)."""
    _check(lib().gs4d_otsu_mask(_ptr(prob), prob.numel(), _ptr(threshold), _ptr(mask), _ptr(ws),
                                ws.numel(), _stream(stream)), "gs4d_otsu_mask")


BIN_AUTO, BIN_PER_TILE, BIN_PRESORT, BIN_COUNT = 0, 1, 2, 3


def gs4d_set_bin_strategy(strategy):
    """Binning strategy of gs4d_bin_sort (process-wide): BIN_AUTO,
    BIN_PER_TILE, BIN_PRESORT or BIN_COUNT; the output is the same."""
    _check(lib().gs4d_set_bin_strategy(int(strategy)), "gs4d_set_bin_strategy")


def gs4d_tile_order_workspace_size(n_tiles):
    return int(lib().gs4d_tile_order_workspace_size(n_tiles))


def gs4d_tile_order(ranges, order, queues, ws, stream=None):
    nq = 0 if queues is None else queues.numel()
    _check(lib().gs4d_tile_order(_ptr(ranges), ranges.shape[0], _ptr(order), _ptr(queues), nq,
                                 _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)),
           "gs4d_tile_order")


def gs4d_set_bwd_variant(pixels_per_lane):
    _check(lib().gs4d_set_bwd_variant(int(pixels_per_lane)), "gs4d_set_bwd_variant")


def gs4d_grid_prune_workspace_size(m, k_attr):
    return int(lib().gs4d_grid_prune_workspace_size(m, k_attr))


def gs4d_grid_prune(xyz, attr, cls, voxel_static, voxel_dynamic, min_count, capacity, out_xyz,
                    out_attr, out_count, out_key, n_out, status, ws, stream=None):
    m = xyz.shape[1]
    k = 0 if attr is None else attr.shape[0]
    _check(lib().gs4d_grid_prune(_ptr(xyz), _ptr(attr), k, _ptr(cls), m, float(voxel_static),
                                 float(voxel_dynamic), int(min_count), int(capacity), _ptr(out_xyz),
                                 _ptr(out_attr), _ptr(out_count), _ptr(out_key), _ptr(n_out),
                                 _ptr(status), _ptr(ws), ws.numel() * ws.element_size(),
                                 _stream(stream)), "gs4d_grid_prune")


def gs4d_backproject_workspace_size(hw):
    return int(lib().gs4d_backproject_workspace_size(hw))


def gs4d_backproject(depth_acc, cover, view, min_cover, capacity, out_xyz, out_depth, out_pixel,
                     n_out, ws, depth_sum=None, stream=None):
    """view: a gs4d_view struct (make_views(...)[0]) or a numpy view row."""
    v = view if isinstance(view, gs4d_view) else make_views(np.atleast_2d(view))[0]
    _check(lib().gs4d_backproject(_ptr(depth_acc), _ptr(cover), ctypes.byref(v), float(min_cover),
                                  int(capacity), _ptr(out_xyz), _ptr(out_depth), _ptr(out_pixel),
                                  _ptr(n_out), _ptr(depth_sum), _ptr(ws), ws.numel() * ws.element_size(),
                                  _stream(stream)), "gs4d_backproject")


def gs4d_heuristic_init(xyz, rgb, t, depth, dynamic, k, voxel_static, voxel_dynamic, focal, frames,
                        params, stream=None):
    """xyz, rgb: [3, stride] row blocks (the first k columns used)."""
    stride = int(xyz.stride(0))
    if rgb.stride(0) != stride:
        raise GS4DError("gs4d_heuristic_init: xyz and rgb rows must share one stride")
    _check(lib().gs4d_heuristic_init(_ptr_rows(xyz, 3), _ptr_rows(rgb, 3), _ptr(t), _ptr(depth),
                                     _ptr(dynamic), int(k),
                                     stride, float(voxel_static), float(voxel_dynamic), float(focal),
                                     int(frames), _ptr(params), _stream(stream)),
           "gs4d_heuristic_init")


def gs4d_adam_step(params, grads, m, v, cfg, step, stream=None):
    _check(lib().gs4d_adam_step(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.shape[-1],
                                ctypes.byref(cfg), _ptr(step), _stream(stream)), "gs4d_adam_step")


def gs4d_loss_l1(img, target, weight, loss, dL_dimg=None, stream=None):
    _check(lib().gs4d_loss_l1(_ptr(img), _ptr(target), img.numel(), float(weight), _ptr(loss),
                              _ptr(dL_dimg), _stream(stream)), "gs4d_loss_l1")


def gs4d_ssim_workspace_size(b, c, h, w):
    return int(lib().gs4d_ssim_workspace_size(b, c, h, w))


def gs4d_ssim(img, target, weight, ssim_sum, dL_dimg, ws, stream=None):
    b, c, h, w = img.shape
    _check(lib().gs4d_ssim(_ptr(img), _ptr(target), b, c, h, w, float(weight), _ptr(ssim_sum),
                           _ptr(dL_dimg), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)),
           "gs4d_ssim")


def gs4d_photometric_loss_workspace_size(b, c, h, w):
    return int(lib().gs4d_photometric_loss_workspace_size(b, c, h, w))


def gs4d_photometric_loss(img, target, w_l1, w_ssim, loss, dL_dimg, ws, stream=None):
    b, c, h, w = img.shape
    _check(lib().gs4d_photometric_loss(_ptr(img), _ptr(target), b, c, h, w, float(w_l1),
                                       float(w_ssim), _ptr(loss), _ptr(dL_dimg), _ptr(ws),
                                       ws.numel() * ws.element_size(), _stream(stream)),
           "gs4d_photometric_loss")


def gs4d_sse(img, target, sse, stream=None):
    _check(lib().gs4d_sse(_ptr(img), _ptr(target), img.numel(), _ptr(sse), _stream(stream)),
           "gs4d_sse")


def _host_f32(values, count):
    arr = (ctypes.c_float * count)(*[float(v) for v in values])
    if len(values) != count:
        raise GS4DError(f"expected {count} host values")
    return arr


def gs4d_knn8_workspace_size(n):
    return int(lib().gs4d_knn8_workspace_size(n))


def gs4d_knn8(xyz, cell, nbr, d2, status, ws, stream=None):
    n = xyz.shape[1]
    _check(lib().gs4d_knn8(_ptr(xyz), n, float(cell), _ptr(nbr), _ptr(d2), _ptr(status), _ptr(ws),
                           ws.numel() * ws.element_size(), _stream(stream)), "gs4d_knn8")


def gs4d_init_features(xyz, attr, dyn, nbr, shift, scale, feat, stream=None):
    n = xyz.shape[1]
    _check(lib().gs4d_init_features(_ptr(xyz), _ptr(attr), _ptr(dyn), _ptr(nbr), n,
                                    _host_f32(shift, 16), _host_f32(scale, 16), _ptr(feat),
                                    _stream(stream)), "gs4d_init_features")


def gs4d_mlp_fwd(w_bf16, x, y, stream=None):
    _check(lib().gs4d_mlp_fwd(_ptr(w_bf16), _ptr(x), x.shape[1], _ptr(y), _stream(stream)),
           "gs4d_mlp_fwd")


def gs4d_mlp_bwd_workspace_size(n):
    return int(lib().gs4d_mlp_bwd_workspace_size(n))


def gs4d_mlp_bwd(w_bf16, x, grad, ws, dy=None, target=None, out_weight=None, dx=None, loss=None,
                 stream=None):
    ow = _host_f32(out_weight, 4) if out_weight is not None else None
    _check(lib().gs4d_mlp_bwd(_ptr(w_bf16), _ptr(x), x.shape[1], _ptr(dy), _ptr(target), ow,
                              _ptr(grad), _ptr(dx), _ptr(loss), _ptr(ws),
                              ws.numel() * ws.element_size(), _stream(stream)), "gs4d_mlp_bwd")


def gs4d_mlp_adam(master, grad, m, v, w_bf16, lr, beta1, beta2, eps, step, stream=None):
    _check(lib().gs4d_mlp_adam(_ptr(master), _ptr(grad), _ptr(m), _ptr(v), _ptr(w_bf16),
                               master.numel(), float(lr), float(beta1), float(beta2), float(eps),
                               _ptr(step), _stream(stream)), "gs4d_mlp_adam")


def gs4d_to_bf16(src, dst, stream=None):
    _check(lib().gs4d_to_bf16(_ptr(src), _ptr(dst), src.numel(), _stream(stream)), "gs4d_to_bf16")


def gs4d_motion_init(params, pred, stream=None):
    _check(lib().gs4d_motion_init(_ptr(params), _ptr(pred), params.shape[1], _stream(stream)),
           "gs4d_motion_init")


def gs4d_motion_of(params, out, stream=None):
    _check(lib().gs4d_motion_of(_ptr(params), params.shape[1], _ptr(out), _stream(stream)),
           "gs4d_motion_of")


def gs4d_fill_f32(dst, value, stream=None):
    _check(lib().gs4d_fill_f32(_ptr(dst), float(value), dst.numel(), _stream(stream)), "gs4d_fill_f32")


def gs4d_fill_u32(dst, value, stream=None):
    _check(lib().gs4d_fill_u32(_ptr(dst), int(value), dst.numel(), _stream(stream)), "gs4d_fill_u32")
