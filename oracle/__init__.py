"""TEST INFRASTRUCTURE: the CPU oracle (ctypes wrapper around liboracle4d.so
plus plain numpy routines).

Only ``tests/``, the smoke check and the benchmark's ``cpu_baseline`` leg may
import this package.  It shares no code with the HIP path.

Precision: integer-deciding quantities (cull, tile rectangles, sort-key depth
bits) are computed in FP32 with a fixed operation order; images,
transmittance and gradients in FP64.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle4d.so")
_lib = None

REC = 12
VIEW_LEN = 23

_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_f32 = ctypes.c_float
_f64 = ctypes.c_double

_SIGS = {
    "or_expf_public": (_f32, [_f32]),
    "or_logf_public": (_f32, [_f32]),
    "or_preprocess_f32": (None, [_p, _i64, _p, _i32, _p, _p, _p]),
    "or_preprocess_f64": (None, [_p, _i64, _p, _i32, _p, _p, _p]),
    "or_preprocess_iso_f32": (None, [_p, _i64, _p, _i32, _p, _p, _p]),
    "or_preprocess_iso_f64": (None, [_p, _i64, _p, _i32, _p, _p, _p]),
    "or_covariance_f64": (_i32, [_p, _i64, _i64, _p]),
    "or_conditional_f64": (_i32, [_p, _i64, _i64, _f64, _p, _p, _p]),
    "or_conditional_f32": (_i32, [_p, _i64, _i64, _f32, _p, _p, _p]),
    "or_conditional_cov_f64_all": (None, [_p, _i64, _f64, _p]),
    "or_conditional_mean_f64_all": (None, [_p, _i64, _f64, _p]),
    "or_bin_sort": (_i64, [_p, _p, _p, _i64, _i32, _i32, _i32, _i64, _p, _p, _p]),
    "or_floor_skip_f32": (_i32, [_p, _f64, _f64]),
    "or_doubtful_decisions": (_i64, [_p, _i64, _p, _i32, _p, _p, _p, _i64, _p]),
    "or_render_fwd": (None, [_p, _i64, _p, _i32, _p, _p, _p, _p, _p, _p, _p, _i32]),
    "or_trace_pixel": (_i64, [_p, _i64, _p, _i32, _p, _p, _i32, _i32, _p, _p, _i64, _p, _i32]),
    "or_render_brute": (None, [_p, _i64, _p, _i32, _p, _p, _p, _p, _i32]),
    "or_render_bwd": (None, [_p, _i64, _p, _i32, _p, _p, _p, _p, _i32]),
    "or_pixel_variant": (_i64, [_p, _i64, _p, _i32, _p, _p, _i32, _i32, _i64, _i32, _p, _p, _p, _p,
                                _i32]),
    "or_preprocess_bwd": (None, [_p, _i64, _p, _i32, _p, _p]),
    "or_preprocess_bwd_mu": (None, [_p, _i64, _p, _i32, _p, _p, _p]),
    "or_preprocess_iso_bwd": (None, [_p, _i64, _p, _i32, _p, _p]),
    "or_grid_prune": (_i64, [_p, _p, _i32, _p, _i64, _f32, _f32, _i32, _i64, _p, _p, _p, _p]),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build_oracle
            build_oracle.build()
        L = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _views(views):
    v = np.ascontiguousarray(np.atleast_2d(np.asarray(views, dtype=np.float64)))
    assert v.shape[1] == VIEW_LEN
    return v


def view_dims(views):
    v = _views(views)
    W, H = int(v[0, 16]), int(v[0, 17])
    return W, H, (W + 15) // 16, (H + 15) // 16


# ---------------------------------------------------------------- FP32 maths
def expf(x: float) -> float:
    return lib().or_expf_public(float(x))


def logf(x: float) -> float:
    return lib().or_logf_public(float(x))


# ---------------------------------------------------------------- preprocess
def preprocess_f32(params, views):
    P = np.ascontiguousarray(params, dtype=np.float32)
    v = _views(views)
    n = P.shape[1]
    V = v.shape[0]
    rec = np.zeros((V, n, REC), np.float32)
    rect = np.zeros((V, n, 4), np.int32)
    touched = np.zeros((V, n), np.int32)
    lib().or_preprocess_f32(_ptr(P), n, _ptr(v), V, _ptr(rec), _ptr(rect), _ptr(touched))
    return rec, rect, touched


def preprocess_f64(params, views):
    P = np.ascontiguousarray(params, dtype=np.float64)
    v = _views(views)
    n = P.shape[1]
    V = v.shape[0]
    rec = np.zeros((V, n, REC), np.float64)
    rect = np.zeros((V, n, 4), np.int32)
    touched = np.zeros((V, n), np.int32)
    lib().or_preprocess_f64(_ptr(P), n, _ptr(v), V, _ptr(rec), _ptr(rect), _ptr(touched))
    return rec, rect, touched


ISO_FIELDS = 13   # isotropic, motion-aware parameters per Gaussian


def preprocess_iso_f32(params, views):
    """Preprocess of the isotropic, motion-aware parameterisation ([13][n]:
    mean xyz t, log s, log s_t, velocity xyz, opacity logit, rgb) in the
    kernel's precision; same outputs as preprocess_f32."""
    P = np.ascontiguousarray(params, dtype=np.float32)
    assert P.shape[0] == ISO_FIELDS
    v = _views(views)
    n = P.shape[1]
    V = v.shape[0]
    rec = np.zeros((V, n, REC), np.float32)
    rect = np.zeros((V, n, 4), np.int32)
    touched = np.zeros((V, n), np.int32)
    lib().or_preprocess_iso_f32(_ptr(P), n, _ptr(v), V, _ptr(rec), _ptr(rect), _ptr(touched))
    return rec, rect, touched


def preprocess_iso_f64(params, views):
    P = np.ascontiguousarray(params, dtype=np.float64)
    assert P.shape[0] == ISO_FIELDS
    v = _views(views)
    n = P.shape[1]
    V = v.shape[0]
    rec = np.zeros((V, n, REC), np.float64)
    rect = np.zeros((V, n, 4), np.int32)
    touched = np.zeros((V, n), np.int32)
    lib().or_preprocess_iso_f64(_ptr(P), n, _ptr(v), V, _ptr(rec), _ptr(rect), _ptr(touched))
    return rec, rect, touched


def covariance(params, g):
    P = np.ascontiguousarray(params, dtype=np.float64)
    out = np.zeros(16)
    ok = lib().or_covariance_f64(_ptr(P), P.shape[1], g, _ptr(out))
    return out.reshape(4, 4) if ok else None


def conditional(params, g, t):
    P = np.ascontiguousarray(params, dtype=np.float64)
    mu = np.zeros(3)
    sc = np.zeros(9)
    ot = np.zeros(1)
    ok = lib().or_conditional_f64(_ptr(P), P.shape[1], g, float(t), _ptr(mu), _ptr(sc), _ptr(ot))
    return (mu, sc.reshape(3, 3), float(ot[0])) if ok else None


def conditional_cov_all(params, t):
    """FP64 conditional covariance of every Gaussian at time t: [n, 3, 3]
    (zeros where degenerate)."""
    P = np.ascontiguousarray(params, dtype=np.float64)
    out = np.zeros((P.shape[1], 9))
    lib().or_conditional_cov_f64_all(_ptr(P), P.shape[1], float(t), _ptr(out))
    return out.reshape(-1, 3, 3)


def conditional_mean_all(params, views):
    """FP64 conditional mean of every Gaussian at each view's time: [V, n, 3]
    (zeros where degenerate)."""
    P = np.ascontiguousarray(params, dtype=np.float64)
    v = _views(views)
    out = np.zeros((v.shape[0], P.shape[1], 3))
    for vi in range(v.shape[0]):
        lib().or_conditional_mean_f64_all(_ptr(P), P.shape[1], float(v[vi, 18]), _ptr(out[vi]))
    return out


def conditional_f32(params, g, t):
    """The FP32 instance's conditional (the kernel's precision and evaluation
    order): (mu [3], Sc [3, 3], o_t) as float32, or None."""
    P = np.ascontiguousarray(params, dtype=np.float32)
    mu = np.zeros(3, np.float32)
    sc = np.zeros(9, np.float32)
    ot = np.zeros(1, np.float32)
    ok = lib().or_conditional_f32(_ptr(P), P.shape[1], g, float(np.float32(t)), _ptr(mu), _ptr(sc),
                                  _ptr(ot))
    return (mu, sc.reshape(3, 3), float(ot[0])) if ok else None


def depth_bits(rec):
    """uint32 bit patterns of the FP32 depth of each record."""
    return np.ascontiguousarray(rec[..., 6].astype(np.float32)).view(np.uint32)


# ---------------------------------------------------------------- binning
def bin_sort(rect, touched, dbits, views, capacity=None):
    v = _views(views)
    V, n = touched.shape
    W, H, tx, ty = view_dims(v)
    total = int(touched.astype(np.int64).sum())
    cap = total if capacity is None else int(capacity)
    keys = np.zeros(max(cap, 1), np.uint64)
    vals = np.zeros(max(cap, 1), np.uint32)
    ranges = np.zeros((V * tx * ty, 2), np.int32)
    P = lib().or_bin_sort(_ptr(np.ascontiguousarray(rect, np.int32)),
                          _ptr(np.ascontiguousarray(touched, np.int32)),
                          _ptr(np.ascontiguousarray(dbits, np.uint32)), n, V, tx, ty, cap,
                          _ptr(keys), _ptr(vals), _ptr(ranges))
    if P < 0:
        return None
    return keys[:P], vals[:P], ranges


# ---------------------------------------------------------------- render
def render_fwd(rec64, views, vals, ranges, signature=False, *, f32):
    """Binned compositing in FP64.  f32: records from the FP32
    preprocess, whose alpha >= 1/255 decisions are taken in the kernel's
    precision (bit for bit as the kernel takes them); False for FP64
    records (self-checks, finite differences)."""
    v = _views(views)
    rec64 = np.ascontiguousarray(rec64, np.float64)
    V, n, _ = rec64.shape
    W, H, _, _ = view_dims(v)
    image = np.zeros((V, 3, H, W))
    T = np.zeros((V, H, W))
    last = np.zeros((V, H, W), np.int32)
    counts = np.zeros(2, np.int64)
    sig = np.zeros((V, H, W), np.uint64) if signature else None
    lib().or_render_fwd(_ptr(rec64), n, _ptr(v), V, _ptr(np.ascontiguousarray(vals, np.uint32)),
                        _ptr(np.ascontiguousarray(ranges, np.int32)), _ptr(image), _ptr(T),
                        _ptr(last), _ptr(counts), _ptr(sig), int(bool(f32)))
    out = dict(image=image, T_final=T, last=last, n_eval=int(counts[0]), n_blend=int(counts[1]))
    if signature:
        out["sig"] = sig
    return out


def trace_pixel(rec64, views, vi, vals, ranges, x, y, *, f32):
    v = _views(views)
    rec64 = np.ascontiguousarray(rec64, np.float64)
    V, n, _ = rec64.shape
    cap = max(len(vals), 1)
    a = np.zeros(cap)
    T = np.zeros(cap)
    Tf = np.zeros(1)
    nb = lib().or_trace_pixel(_ptr(rec64), n, _ptr(v), vi, _ptr(np.ascontiguousarray(vals, np.uint32)),
                              _ptr(np.ascontiguousarray(ranges, np.int32)), x, y, _ptr(a), _ptr(T),
                              cap, _ptr(Tf), int(bool(f32)))
    return a[:nb], T[:nb], float(Tf[0])


def floor_skip_f32(rec12, px, py):
    """The alpha >= 1/255 floor as decided in the kernel's precision: 1 to
    skip the entry (FP32 record rec12 at pixel centre (px, py))."""
    r = np.ascontiguousarray(rec12, np.float64)
    return int(lib().or_floor_skip_f32(_ptr(r), float(px), float(py)))


DECISION_KIND = {1: "alpha", 2: "clamp", 3: "stop"}


def doubtful_decisions(rec64, views, vals, ranges):
    """Decisions an FP32 kernel render may take the other way from the
    oracle's FP32 shadow: (flag [V, H, W] of their pixels, list of (view, x,
    y, entry position in the tile's list, kind))."""
    v = _views(views)
    rec64 = np.ascontiguousarray(rec64, np.float64)
    V, n, _ = rec64.shape
    W, H, _, _ = view_dims(v)
    flag = np.zeros((V, H, W), np.uint8)
    cap = 1 << 16
    while True:
        out = np.zeros((cap, 5), np.int32)
        k = lib().or_doubtful_decisions(_ptr(rec64), n, _ptr(v), V,
                                        _ptr(np.ascontiguousarray(vals, np.uint32)),
                                        _ptr(np.ascontiguousarray(ranges, np.int32)), _ptr(out), cap,
                                        _ptr(flag))
        if k <= cap:
            break
        cap = int(k)
        flag[:] = 0
    found = [(int(a), int(b), int(c), int(d), DECISION_KIND[int(e)]) for a, b, c, d, e in out[:k]]
    return flag.astype(bool), found


PIXEL_FORCE = {"alpha": 1, "clamp": 2, "stop": 3}


def pixel_variant(rec64, views, vi, vals, ranges, x, y, gC, force_entry=-1, force="alpha", *,
                  f32):
    """One pixel composited with (optionally) one discrete decision inverted:
    entry `force_entry` of its tile's list takes the other side of its
    alpha >= 1/255 test ("alpha"), its 0.99 clamp ("clamp") or its
    transmittance stop ("stop").  Returns (colour [3] with background,
    T_final, d/d(record) [m, 9] per entry of the tile's list for the upstream
    colour gradient gC [3], number of blends)."""
    v = _views(views)
    rec64 = np.ascontiguousarray(rec64, np.float64)
    V, n, _ = rec64.shape
    W, H, tx, ty = view_dims(v)
    tile = vi * tx * ty + (y // 16) * tx + (x // 16)
    b, e = (int(q) for q in np.asarray(ranges)[tile])
    m = max(e - b, 0)
    grec = np.zeros((max(m, 1), 9))
    C = np.zeros(3)
    T = np.zeros(1)
    gc = np.ascontiguousarray(gC, np.float64)
    nb = lib().or_pixel_variant(_ptr(rec64), n, _ptr(v), vi, _ptr(np.ascontiguousarray(vals, np.uint32)),
                                _ptr(np.ascontiguousarray(ranges, np.int32)), int(x), int(y),
                                int(force_entry), PIXEL_FORCE[force] if force_entry >= 0 else 0,
                                _ptr(gc), _ptr(C), _ptr(T), _ptr(grec), int(bool(f32)))
    return C, float(T[0]), grec[:m], int(nb)


def render_brute(rec64, views, touched, dbits, *, f32):
    v = _views(views)
    rec64 = np.ascontiguousarray(rec64, np.float64)
    V, n, _ = rec64.shape
    W, H, _, _ = view_dims(v)
    image = np.zeros((V, 3, H, W))
    T = np.zeros((V, H, W))
    lib().or_render_brute(_ptr(rec64), n, _ptr(v), V, _ptr(np.ascontiguousarray(touched, np.int32)),
                          _ptr(np.ascontiguousarray(dbits, np.uint32)), _ptr(image), _ptr(T),
                          int(bool(f32)))
    return image, T


def render_bwd(rec64, views, vals, ranges, dL_dimage, *, f32):
    v = _views(views)
    rec64 = np.ascontiguousarray(rec64, np.float64)
    V, n, _ = rec64.shape
    g = np.zeros((V, n, 9))
    lib().or_render_bwd(_ptr(rec64), n, _ptr(v), V, _ptr(np.ascontiguousarray(vals, np.uint32)),
                        _ptr(np.ascontiguousarray(ranges, np.int32)),
                        _ptr(np.ascontiguousarray(dL_dimage, np.float64)), _ptr(g),
                        int(bool(f32)))
    return g


def preprocess_bwd(params, views, grad_rec, grad_mu3=None):
    """Chain rule (FP64) from grad_rec [V, n, 9] = d(mean2D, conic, o_t, rgb)
    to d params [20, n]; grad_mu3 [V, n, 3] (optional) is a further gradient
    with respect to the conditional mean at each view's time."""
    P = np.ascontiguousarray(params, dtype=np.float64)
    v = _views(views)
    n = P.shape[1]
    d = np.zeros((20, n))
    if grad_mu3 is None:
        lib().or_preprocess_bwd(_ptr(P), n, _ptr(v), v.shape[0],
                                _ptr(np.ascontiguousarray(grad_rec, np.float64)), _ptr(d))
    else:
        lib().or_preprocess_bwd_mu(_ptr(P), n, _ptr(v), v.shape[0],
                                   _ptr(np.ascontiguousarray(grad_rec, np.float64)),
                                   _ptr(np.ascontiguousarray(grad_mu3, np.float64)), _ptr(d))
    return d


def preprocess_iso_bwd(params, views, grad_rec):
    """Chain rule of the isotropic, motion-aware preprocess (FP64): grad_rec
    [V, n, 9] = d(mean2D, conic, o_t, rgb) -> d params [13, n]."""
    P = np.ascontiguousarray(params, dtype=np.float64)
    assert P.shape[0] == ISO_FIELDS
    v = _views(views)
    n = P.shape[1]
    d = np.zeros((ISO_FIELDS, n))
    lib().or_preprocess_iso_bwd(_ptr(P), n, _ptr(v), v.shape[0],
                                _ptr(np.ascontiguousarray(grad_rec, np.float64)), _ptr(d))
    return d


# ---------------------------------------------------------------- pipelines
def forward(params, views, precision="f32"):
    """Full forward.  precision="f32": the kernel-precision preprocess (whose
    integers the GPU must match bit for bit) promoted to FP64 for compositing,
    the alpha >= 1/255 decisions taken in the kernel's precision.
    precision="f64": everything in FP64 (self-checks, finite differences)."""
    if precision == "f32":
        rec, rect, touched = preprocess_f32(params, views)
    else:
        rec, rect, touched = preprocess_f64(params, views)
    dbits = depth_bits(rec)
    keys, vals, ranges = bin_sort(rect, touched, dbits, views)
    rec64 = rec.astype(np.float64)
    out = render_fwd(rec64, views, vals, ranges, f32=precision == "f32")
    out.update(rec=rec, rect=rect, touched=touched, keys=keys, vals=vals, ranges=ranges,
               dbits=dbits, f32=precision == "f32")
    return out


def backward(params, views, dL_dimage, fwd=None, precision="f32"):
    """dL/dparams [20, N] for an upstream image gradient (FP64 chain rule)."""
    if fwd is None:
        fwd = forward(params, views, precision)
    grec = render_bwd(fwd["rec"].astype(np.float64), views, fwd["vals"], fwd["ranges"], dL_dimage,
                      f32=fwd["f32"])
    return preprocess_bwd(params, views, grec), grec


# ---------------------------------------------------------------- prune
def grid_prune(xyz, attr, cls, voxel_static, voxel_dynamic=None, min_count=1, capacity=None):
    xyz = np.ascontiguousarray(xyz, np.float32)
    m = xyz.shape[1]
    attr = np.ascontiguousarray(attr if attr is not None else np.zeros((0, m)), np.float32)
    k = attr.shape[0]
    cl = np.ascontiguousarray(cls, np.uint8) if cls is not None else None
    cap = m if capacity is None else capacity
    vd = voxel_static if voxel_dynamic is None else voxel_dynamic
    ox = np.zeros((3, max(cap, 1)), np.float32)
    oa = np.zeros((max(k, 1), max(cap, 1)), np.float32)
    oc = np.zeros(max(cap, 1), np.int32)
    ok = np.zeros(max(cap, 1), np.uint64)
    nout = lib().or_grid_prune(_ptr(xyz), _ptr(attr), k, _ptr(cl), m, float(voxel_static), float(vd),
                               int(min_count), cap, _ptr(ox), _ptr(oa), _ptr(oc), _ptr(ok))
    if nout < 0:
        return None
    return dict(xyz=ox[:, :nout], attr=oa[:k, :nout], count=oc[:nout], key=ok[:nout])
