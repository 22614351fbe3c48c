/*
 * TEST INFRASTRUCTURE: the CPU oracle for the 4D Gaussian-splatting hot path.
 *
 * This file is a plain, slow, deliberately unoptimised C implementation of
 * what the GPU path computes.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or helper with the HIP library.
 *
 * Precision policy
 *   - Every quantity that decides an integer (cull, tile rectangle, the depth
 *     bits of a sort key) is computed in FP32, the kernel's precision, with a
 *     fixed operation order and project-written exp/ln (pre_tmpl.inc, FP32
 *     instance).
 *   - Images, transmittance and gradients are computed in FP64.
 *   - An FP64 instance of the same preprocess serves the self-checks and the
 *     gradient chain rule.
 *
 * Paper passages followed (arXiv 2510.01119):
 *   Sec. 3.3 "Motion Modeling", Eq. "4dgs": the conditional mean and
 *     covariance of a 4D Gaussian at time t.
 *   Sec. 3.3 "Motion-Aware Gaussian": o_t = o N(t; mu_4, Sigma_44) and the
 *     cull of Gaussians whose o_t falls below a threshold.
 *   Sec. 3.1 "4D Gaussian Splatting": the Gaussian G(p) = a exp(-1/2 d^T S^-1 d)
 *     and the splatting renderer it inherits (projection, tiles, depth-sorted
 *     alpha compositing) from 3D/4D Gaussian splatting.
 *   Sec. 3.2 "Grid Pruning": voxel assignment by integer division with S_v,
 *     centroid and attribute averaging, low-support voxels discarded.
 *
 * The readings taken where the paper is silent are stated next to each step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_REC 12
#define OR_VIEW 23   /* Rt[12] fx fy cx cy W H t near bg[3] */

/* ------------------------------------------------------------------------- *
 * Project-written FP32 exp and ln.  Both are textbook methods:
 *   exp: Cody-Waite reduction x = k ln2 + r with a two-part ln2, then the
 *        degree-7 Taylor polynomial of e^r in Horner form, then 2^k scaling.
 *   ln : x = m 2^e with m in [1/sqrt2, sqrt2), ln m = 2 atanh(u),
 *        u = (m-1)/(m+1), atanh series to u^9.
 * They exist so that the FP32 preprocess has a single, reproducible
 * definition; accuracy is a few ulp.
 * ------------------------------------------------------------------------- */
static float or_expf(float x)
{
    if (x != x) return x;
    if (x < -87.0f) return 0.0f;
    if (x > 88.0f) return INFINITY;
    const float k = rintf(x * 1.44269504088896341f);
    float r = x - k * 0.693145751953125f;
    r = r - k * 1.428606765330187e-06f;
    float p = 1.0f / 5040.0f;
    p = fmaf(p, r, 1.0f / 720.0f);
    p = fmaf(p, r, 1.0f / 120.0f);
    p = fmaf(p, r, 1.0f / 24.0f);
    p = fmaf(p, r, 1.0f / 6.0f);
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    return ldexpf(p, (int)k);
}

static float or_logf(float x)
{
    if (x != x) return x;
    if (x < 0.0f) return NAN;
    if (x == 0.0f) return -INFINITY;
    if (x == INFINITY) return x;
    int e;
    float m = frexpf(x, &e);
    if (m < 0.70710678118654752f) { m = m * 2.0f; e = e - 1; }
    const float u = (m - 1.0f) / (m + 1.0f);
    const float u2 = u * u;
    float s = 1.0f / 9.0f;
    s = fmaf(s, u2, 1.0f / 7.0f);
    s = fmaf(s, u2, 1.0f / 5.0f);
    s = fmaf(s, u2, 1.0f / 3.0f);
    s = fmaf(s, u2, 1.0f);
    return fmaf((float)e, 0.693147180559945309f, (2.0f * u) * s);
}

float or_expf_public(float x) { return or_expf(x); }
float or_logf_public(float x) { return or_logf(x); }

/* ---- FP32 instance ---- */
#define REAL float
#define PROJECTED_SLICE 1
#define FN(x) x##_f32
#define EXPR(x) or_expf(x)
#define LOGR(x) or_logf(x)
#define SQRTR(x) sqrtf(x)
#define CEILR(x) ceilf(x)
#define FLOORR(x) floorf(x)
#define FMAXR(a, b) fmaxf(a, b)
#define FMINR(a, b) fminf(a, b)
#include "pre_tmpl.inc"
#undef REAL
#undef PROJECTED_SLICE
#undef FN
#undef EXPR
#undef LOGR
#undef SQRTR
#undef CEILR
#undef FLOORR
#undef FMAXR
#undef FMINR

/* ---- FP64 instance ---- */
#define REAL double
#define PROJECTED_SLICE 0
#define FN(x) x##_f64
#define EXPR(x) exp(x)
#define LOGR(x) log(x)
#define SQRTR(x) sqrt(x)
#define CEILR(x) ceil(x)
#define FLOORR(x) floor(x)
#define FMAXR(a, b) fmax(a, b)
#define FMINR(a, b) fmin(a, b)
#include "pre_tmpl.inc"
#undef REAL
#undef PROJECTED_SLICE
#undef FN
#undef EXPR
#undef LOGR
#undef SQRTR
#undef CEILR
#undef FLOORR
#undef FMAXR
#undef FMINR

/* params: [20][n] planes; views: [n_views][OR_VIEW]; outputs per (view, g) */
void or_preprocess_f32(const float *params, int64_t n, const double *views, int32_t n_views,
                       float *rec, int32_t *rect, int32_t *touched)
{
    for (int32_t vi = 0; vi < n_views; ++vi)
        for (int64_t g = 0; g < n; ++g) {
            const int64_t o = (int64_t)vi * n + g;
            preprocess_one_f32(params, n, g, views + (int64_t)vi * OR_VIEW, rec + o * OR_REC,
                               rect + o * 4, touched + o);
        }
}

void or_preprocess_f64(const double *params, int64_t n, const double *views, int32_t n_views,
                       double *rec, int32_t *rect, int32_t *touched)
{
    for (int32_t vi = 0; vi < n_views; ++vi)
        for (int64_t g = 0; g < n; ++g) {
            const int64_t o = (int64_t)vi * n + g;
            preprocess_one_f64(params, n, g, views + (int64_t)vi * OR_VIEW, rec + o * OR_REC,
                               rect + o * 4, touched + o);
        }
}

/* Isotropic, motion-aware parameterisation: params [13][n] planes. */
void or_preprocess_iso_f32(const float *params, int64_t n, const double *views, int32_t n_views,
                           float *rec, int32_t *rect, int32_t *touched)
{
    for (int32_t vi = 0; vi < n_views; ++vi)
        for (int64_t g = 0; g < n; ++g) {
            const int64_t o = (int64_t)vi * n + g;
            preprocess_iso_one_f32(params, n, g, views + (int64_t)vi * OR_VIEW, rec + o * OR_REC,
                                   rect + o * 4, touched + o);
        }
}

void or_preprocess_iso_f64(const double *params, int64_t n, const double *views, int32_t n_views,
                           double *rec, int32_t *rect, int32_t *touched)
{
    for (int32_t vi = 0; vi < n_views; ++vi)
        for (int64_t g = 0; g < n; ++g) {
            const int64_t o = (int64_t)vi * n + g;
            preprocess_iso_one_f64(params, n, g, views + (int64_t)vi * OR_VIEW, rec + o * OR_REC,
                                   rect + o * 4, touched + o);
        }
}

/* Self-check helpers (FP64): Sigma (row-major 4x4) of Gaussian g, and its
 * conditional at time t: mu[3], Sc (row-major 3x3), o_t.  Return 0 if
 * degenerate. */
int or_covariance_f64(const double *params, int64_t n, int64_t g, double *sigma16)
{
    double v[20], Sg[4][4], M[4][4], s[4], o;
    for (int k = 0; k < 20; ++k) v[k] = params[(int64_t)k * n + g];
    if (!covariance_f64(v, Sg, M, s, &o)) return 0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) sigma16[4 * i + j] = Sg[i][j];
    return 1;
}

int or_conditional_f64(const double *params, int64_t n, int64_t g, double t, double *mu3,
                       double *sc9, double *ot)
{
    double v[20], Sg[4][4], M[4][4], s[4], o, mu[3], Sc[3][3];
    for (int k = 0; k < 20; ++k) v[k] = params[(int64_t)k * n + g];
    if (!covariance_f64(v, Sg, M, s, &o)) return 0;
    if (!conditional_f64(v, Sg, M, o, t, mu, Sc, ot)) return 0;
    for (int i = 0; i < 3; ++i) {
        mu3[i] = mu[i];
        for (int j = 0; j < 3; ++j) sc9[3 * i + j] = Sc[i][j];
    }
    return 1;
}

/* The FP64 conditional covariance of every Gaussian at time t: sc9 [n][9]
 * (row-major 3x3; zeros where degenerate). */
void or_conditional_cov_f64_all(const double *params, int64_t n, double t, double *sc9)
{
    for (int64_t g = 0; g < n; ++g) {
        double v[20], Sg[4][4], M[4][4], s[4], o, mu[3], Sc[3][3], ot;
        for (int k = 0; k < 20; ++k) v[k] = params[(int64_t)k * n + g];
        int ok = covariance_f64(v, Sg, M, s, &o) && conditional_f64(v, Sg, M, o, t, mu, Sc, &ot);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) sc9[9 * g + 3 * i + j] = ok ? Sc[i][j] : 0.0;
    }
}

/* The FP64 conditional mean of every Gaussian at time t: mu3 [n][3] (zeros
 * where degenerate). */
void or_conditional_mean_f64_all(const double *params, int64_t n, double t, double *mu3)
{
    for (int64_t g = 0; g < n; ++g) {
        double v[20], Sg[4][4], M[4][4], s[4], o, mu[3], Sc[3][3], ot;
        for (int k = 0; k < 20; ++k) v[k] = params[(int64_t)k * n + g];
        int ok = covariance_f64(v, Sg, M, s, &o) && conditional_f64(v, Sg, M, o, t, mu, Sc, &ot);
        for (int i = 0; i < 3; ++i) mu3[3 * g + i] = ok ? mu[i] : 0.0;
    }
}

/* The FP32 instance's conditional (the kernel's precision and evaluation
 * order): mu[3], Sc (row-major 3x3), o_t of Gaussian g at time t.  Returns
 * 0 if degenerate. */
int or_conditional_f32(const float *params, int64_t n, int64_t g, float t, float *mu3,
                       float *sc9, float *ot)
{
    float v[20], Sg[4][4], M[4][4], s[4], o, mu[3], Sc[3][3];
    for (int k = 0; k < 20; ++k) v[k] = params[(int64_t)k * n + g];
    if (!covariance_f32(v, Sg, M, s, &o)) return 0;
    if (!conditional_f32(v, Sg, M, o, t, mu, Sc, ot)) return 0;
    for (int i = 0; i < 3; ++i) {
        mu3[i] = mu[i];
        for (int j = 0; j < 3; ++j) sc9[3 * i + j] = Sc[i][j];
    }
    return 1;
}

/* ------------------------------------------------------------------------- *
 * Tile binning.  A view of W x H pixels has ceil(W/16) x ceil(H/16) tiles;
 * global tile id = view * tiles_per_view + ty * tiles_x + tx.  A pair's key
 * is (global tile id << 32) | bits(float depth); depth is positive, so the
 * bit pattern orders like the value.  Pairs are sorted ascending by
 * (key, Gaussian id), which is a total order.
 * ------------------------------------------------------------------------- */
static int cmp_pair(const void *pa, const void *pb)
{
    const uint64_t *a = (const uint64_t *)pa, *b = (const uint64_t *)pb;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    return 0;
}

/* depth_bits: [n_views][n] uint32 bit patterns of the FP32 depth.
 * Returns the number of pairs, or -1 if it exceeds capacity. */
int64_t or_bin_sort(const int32_t *rect, const int32_t *touched, const uint32_t *depth_bits,
                    int64_t n, int32_t n_views, int32_t tiles_x, int32_t tiles_y, int64_t capacity,
                    uint64_t *keys, uint32_t *vals, int32_t *ranges)
{
    const int64_t tpv = (int64_t)tiles_x * tiles_y;
    int64_t total = 0;
    for (int64_t i = 0; i < (int64_t)n_views * n; ++i) total += touched[i];
    for (int64_t tile = 0; tile < tpv * n_views; ++tile) { ranges[2 * tile] = 0; ranges[2 * tile + 1] = 0; }
    if (total > capacity) return -1;
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)(total > 0 ? total : 1));
    int64_t p = 0;
    for (int32_t vi = 0; vi < n_views; ++vi)
        for (int64_t g = 0; g < n; ++g) {
            const int64_t o = (int64_t)vi * n + g;
            if (touched[o] == 0) continue;
            const int32_t *rc = rect + 4 * o;
            for (int32_t ty = rc[1]; ty < rc[3]; ++ty)
                for (int32_t tx = rc[0]; tx < rc[2]; ++tx) {
                    const uint64_t tile = (uint64_t)(vi * tpv + (int64_t)ty * tiles_x + tx);
                    tmp[2 * p] = (tile << 32) | depth_bits[o];
                    tmp[2 * p + 1] = (uint64_t)g;
                    ++p;
                }
        }
    qsort(tmp, (size_t)total, sizeof(uint64_t) * 2, cmp_pair);
    for (int64_t i = 0; i < total; ++i) {
        keys[i] = tmp[2 * i];
        vals[i] = (uint32_t)tmp[2 * i + 1];
    }
    free(tmp);
    /* ranges: [first, last + 1) per tile; (0, 0) for an empty tile */
    for (int64_t i = 0; i < total; ++i) {
        const int64_t tile = (int64_t)(keys[i] >> 32);
        if (i == 0 || (int64_t)(keys[i - 1] >> 32) != tile) ranges[2 * tile] = (int32_t)i;
        if (i == total - 1 || (int64_t)(keys[i + 1] >> 32) != tile) ranges[2 * tile + 1] = (int32_t)(i + 1);
    }
    return total;
}

/* ------------------------------------------------------------------------- *
 * Per-pixel compositing (FP64).  Pixel centres sit at (x + 1/2, y + 1/2).
 * For each entry, front to back:
 *   power = min(0, -1/2 (a dx^2 + c dy^2) - b dx dy)
 *   alpha = min(0.99, o_t exp(power)); skip if alpha < 1/255
 *   T' = T (1 - alpha); stop (without blending) if T' < 1e-4
 *   C += rgb alpha T; T = T'
 * Output C + T bg.  These per-pixel constants are those of the 3D Gaussian
 * splatting renderer the paper builds on.  The conic of a visible record is
 * positive definite (its determinant is positive and its diagonal carries
 * the 0.3 px^2 dilation), so the exponent is <= 0 in exact arithmetic; the
 * min() only absorbs rounding, so alpha never exceeds o_t and the pixel
 * value stays continuous where the exponent passes 0.  The derivative is
 * that of the exponent itself (the min is the identity on the exact values).
 * ------------------------------------------------------------------------- */
typedef struct {
    double alpha, atil, ex, T;
    int clamped;
    int64_t entry;
} or_blend;

/* Compositing decisions taken in the kernel's precision.
 *
 * Blending an entry, clamping its alpha and stopping a pixel are integer
 * decisions that FP32 and FP64 evaluations can take differently near a
 * threshold.  With f32 decisions the oracle takes them on an FP32 shadow of
 * the kernel's per-entry arithmetic, in the kernel's fixed order:
 *   dx = (x + 1/2) - mx, dy likewise,
 *   qx = fma(a, dx, b dy), qy = fma(c, dy, b dx),
 *   arg = min(0, fma(dx, qx, dy qy) * (-(1/2) log2 e))   (the exponent in log2 units),
 *   skip iff arg < lo, lo = ln(255 o_t) * (-log2 e) with the project-defined
 *     logarithm (in exact arithmetic the same as alpha < 1/255),
 *   at = o_t 2^arg, alpha = min(0.99, at),
 *   clamped iff at > 0.99, stop iff T (1 - alpha) < 1e-4 (T in FP32),
 * with 2^x correctly rounded where the kernel uses the hardware exp2 (within
 * an ulp).  Colour, transmittance and gradients stay FP64.  The floor is
 * then the same bit for bit; clamp and stop can differ only where the
 * shadow lies within the hardware exp2's ulps of the threshold (see
 * or_doubtful_decisions). */
static const float NEG_HALF_LOG2E_F32 = -0.72134752044448170368f;   /* -(1/2) log2 e */
static const float NEG_LOG2E_F32 = -1.44269504088896340736f;        /* -log2 e */

typedef struct {
    float arg, lo, at;
} or_shadow;

static void shadow_entry(const double *r, double px, double py, or_shadow *sh)
{
    const float mx = (float)r[0], my = (float)r[1];
    const float a = (float)r[2], b = (float)r[3], c = (float)r[4], ot = (float)r[5];
    const float dx = (float)px - mx, dy = (float)py - my;
    const float qx = fmaf(a, dx, b * dy);
    const float qy = fmaf(c, dy, b * dx);
    sh->arg = fminf(fmaf(dx, qx, dy * qy) * NEG_HALF_LOG2E_F32, 0.0f);
    sh->lo = or_logf(255.0f * ot) * NEG_LOG2E_F32;
    const float ex = (float)exp2((double)sh->arg);
    sh->at = ot * ex;
}

static int floor_skip_f32(const double *r, double px, double py)
{
    or_shadow sh;
    shadow_entry(r, px, py, &sh);
    return sh.arg < sh.lo;
}

int32_t or_floor_skip_f32(const double *rec12, double px, double py)
{
    return floor_skip_f32(rec12, px, py);
}

/* Composites the pixel over the ordered Gaussian list ids[0..m).  Records are
 * FP64 [*][12] at rec_view.  Fills up to max_b blends.  Returns count.
 * force_e >= 0 inverts one discrete decision of entry force_e (for error
 * bounds: what the pixel would be had a rounding taken that decision the
 * other way): force_kind 1 the alpha >= 1/255 test, 2 the 0.99 clamp, 3 the
 * T' < 1e-4 stop.  f32: take the decisions in the kernel's precision (the
 * FP32 shadow above; records from the FP32 preprocess), else in FP64. */
static int64_t composite_pixel_ex(const double *rec_view, const uint32_t *ids, int64_t m, double px,
                                  double py, double *C, double *Tout, int64_t *last, or_blend *bl,
                                  int64_t max_b, int64_t *n_eval, int64_t force_e, int force_kind,
                                  int f32)
{
    double T = 1.0;
    float T32 = 1.0f;
    int64_t nb = 0;
    C[0] = C[1] = C[2] = 0.0;
    *last = -1;
    for (int64_t e = 0; e < m; ++e) {
        const double *r = rec_view + (int64_t)ids[e] * OR_REC;
        const double dx = px - r[0], dy = py - r[1];
        const double power = fmin(-0.5 * (r[2] * dx * dx + r[4] * dy * dy) - r[3] * dx * dy, 0.0);
        ++*n_eval;
        const double ex = exp(power);
        const double atil = r[5] * ex;
        or_shadow sh = { 0.0f, 0.0f, 0.0f };
        if (f32) shadow_entry(r, px, py, &sh);
        int clamped = f32 ? sh.at > 0.99f : atil > 0.99;
        if (e == force_e && force_kind == 2) clamped = !clamped;
        const double alpha = clamped ? 0.99 : atil;
        int skip = f32 ? sh.arg < sh.lo : alpha < 1.0 / 255.0;
        if (e == force_e && force_kind == 1) skip = !skip;
        if (skip) continue;
        const double Tn = T * (1.0 - alpha);
        const float Tn32 = T32 * (1.0f - (clamped ? 0.99f : sh.at));
        int stop = f32 ? Tn32 < 1e-4f : Tn < 1e-4;
        if (e == force_e && force_kind == 3) stop = !stop;
        if (stop) break;
        for (int ch = 0; ch < 3; ++ch) C[ch] += r[8 + ch] * alpha * T;
        if (bl && nb < max_b) {
            bl[nb].alpha = alpha; bl[nb].atil = atil; bl[nb].ex = ex; bl[nb].T = T;
            bl[nb].clamped = clamped; bl[nb].entry = e;
        }
        ++nb;
        T = Tn;
        T32 = Tn32;
        *last = e;
    }
    *Tout = T;
    return nb;
}

static int64_t composite_pixel(const double *rec_view, const uint32_t *ids, int64_t m, double px,
                               double py, double *C, double *Tout, int64_t *last, or_blend *bl,
                               int64_t max_b, int64_t *n_eval, int f32)
{
    return composite_pixel_ex(rec_view, ids, m, px, py, C, Tout, last, bl, max_b, n_eval, -1, 0,
                              f32);
}

/* The decisions an FP32 kernel render may take the other way from the FP32
 * shadow (for parity bounds).  The shadow matches the kernel bit for bit
 * except its correctly rounded 2^x against the hardware's (within 1 ulp of
 * exact), so at = o_t 2^x may differ by a few ulp: EPS_AT = 2^-21 of it.
 * A clamp is doubtful when at lies within that of 0.99.  1 - alpha then
 * differs by at most EPS_AT alpha / (1 - alpha) relative (0 when both
 * clamp), and the FP32 transmittance by the sum of those over the blends
 * so far: a stop is doubtful when T (1 - alpha) lies within that of 1e-4.
 * (The 1/255 floor is the same bit for bit.)  For every pixel with a tile
 * list, each doubtful decision is written to out [cap][5] as (view, x, y,
 * entry position in the tile's list, kind: 2 clamp, 3 stop), and
 * flag [n_views][H][W] (zeroed first) marks its pixel.  Returns the number
 * found (entries past cap are counted, not written). */
int64_t or_doubtful_decisions(const double *rec, int64_t n, const double *views, int32_t n_views,
                              const uint32_t *vals, const int32_t *ranges, int32_t *out, int64_t cap,
                              uint8_t *flag)
{
    const float EPS_AT = 1.0f / 2097152.0f;
    int64_t found = 0;
    for (int32_t vi = 0; vi < n_views; ++vi) {
        const double *vw = views + (int64_t)vi * OR_VIEW;
        const int W = (int)vw[16], H = (int)vw[17];
        const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
        const int64_t tpv = (int64_t)tiles_x * tiles_y;
        const double *rv = rec + (int64_t)vi * n * OR_REC;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                const int64_t tile = vi * tpv + (int64_t)(y >> 4) * tiles_x + (x >> 4);
                const int32_t b = ranges[2 * tile], e = ranges[2 * tile + 1];
                const double px = x + 0.5, py = y + 0.5;
                float T32 = 1.0f, epsT = 0.0f;
                for (int32_t k = b; k < e; ++k) {
                    const double *r = rv + (int64_t)vals[k] * OR_REC;
                    or_shadow sh;
                    shadow_entry(r, px, py, &sh);
                    if (sh.arg < sh.lo) continue;
                    const int clamped = sh.at > 0.99f;
                    int kind = 0;
                    if (fabsf(sh.at - 0.99f) <= 0.99f * EPS_AT) kind = 2;
                    const float a = clamped ? 0.99f : sh.at;
                    const float e_one = clamped && kind == 0 ? 0.0f : EPS_AT * a / (1.0f - a);
                    const float Tn = T32 * (1.0f - a);
                    for (int pass = 0; pass < 2; ++pass) {
                        if (pass == 1) kind = fabsf(Tn - 1e-4f) <= Tn * (epsT + e_one) ? 3 : 0;
                        if (!kind) continue;
                        if (found < cap) {
                            int32_t *o = out + 5 * found;
                            o[0] = vi; o[1] = x; o[2] = y; o[3] = k - b; o[4] = kind;
                        }
                        ++found;
                        flag[((int64_t)vi * H + y) * W + x] = 1;
                    }
                    if (Tn < 1e-4f) break;
                    T32 = Tn;
                    epsT += e_one;
                }
            }
    }
    return found;
}

/* Back-to-front gradient of one pixel's colour (see or_render_bwd) for its
 * nb blends bl[]: adds d/d(mx, my, a, b, c, o_t, r, g, b) of each blended
 * entry to dst + 9 * key, key = the entry's Gaussian id (by_entry = 0) or
 * its position in the list (by_entry = 1). */
static void pixel_backward(const double *rv, const uint32_t *ids, const or_blend *bl, int64_t nb,
                           double px, double py, const double gC[3], const double bg[3],
                           double *dst, int by_entry)
{
    double Bk[3] = { bg[0], bg[1], bg[2] };
    for (int64_t k = nb - 1; k >= 0; --k) {
        const uint32_t g = ids[bl[k].entry];
        const double *r = rv + (int64_t)g * OR_REC;
        double *gg = dst + 9 * (by_entry ? bl[k].entry : (int64_t)g);
        const double a = bl[k].alpha, Ti = bl[k].T;
        double dalpha = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
            gg[6 + ch] += a * Ti * gC[ch];
            dalpha += gC[ch] * Ti * (r[8 + ch] - Bk[ch]);
            Bk[ch] = a * r[8 + ch] + (1.0 - a) * Bk[ch];
        }
        if (bl[k].clamped) continue;
        const double dx = px - r[0], dy = py - r[1];
        const double dpow = dalpha * bl[k].atil;
        gg[5] += dalpha * bl[k].ex;
        gg[2] += dpow * (-0.5 * dx * dx);
        gg[3] += dpow * (-dx * dy);
        gg[4] += dpow * (-0.5 * dy * dy);
        gg[0] += dpow * (r[2] * dx + r[3] * dy);
        gg[1] += dpow * (r[4] * dy + r[3] * dx);
    }
}

/* One pixel (x, y) of view vi with one decision inverted (force_e, force_kind
 * as in composite_pixel_ex; force_e < 0: none): its colour C[3] (background
 * included), T_final, and the d/d(record) of each entry of the pixel's tile
 * list for the upstream colour gradient gC[3], written to grec_entry
 * [m][9] (m = the tile's list length; overwritten).  Returns the number of
 * blends. */
int64_t or_pixel_variant(const double *rec, int64_t n, const double *views, int32_t vi,
                         const uint32_t *vals, const int32_t *ranges, int32_t x, int32_t y,
                         int64_t force_e, int32_t force_kind, const double *gC, double *C_out,
                         double *T_out, double *grec_entry, int32_t f32)
{
    const double *vw = views + (int64_t)vi * OR_VIEW;
    const int W = (int)vw[16], H = (int)vw[17];
    const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
    const int64_t tile = vi * (int64_t)tiles_x * tiles_y + (int64_t)(y >> 4) * tiles_x + (x >> 4);
    const int32_t b = ranges[2 * tile], e = ranges[2 * tile + 1];
    const int64_t m = e - b;
    const double *rv = rec + (int64_t)vi * n * OR_REC;
    or_blend *bl = (or_blend *)malloc(sizeof(or_blend) * (size_t)(m > 0 ? m : 1));
    double C[3], T;
    int64_t lst, dummy = 0;
    const double px = x + 0.5, py = y + 0.5;
    const int64_t nb = composite_pixel_ex(rv, vals + b, m, px, py, C, &T, &lst, bl, m, &dummy,
                                          force_e, force_kind, f32);
    for (int ch = 0; ch < 3; ++ch) C_out[ch] = C[ch] + T * vw[20 + ch];
    *T_out = T;
    memset(grec_entry, 0, sizeof(double) * 9 * (size_t)(m > 0 ? m : 1));
    pixel_backward(rv, vals + b, bl, nb, px, py, gC, vw + 20, grec_entry, 1);
    free(bl);
    return nb;
}

/* Binned render.  rec: FP64 [n_views][n][12].  image [V][3][H][W], T_final
 * and last [V][H][W]; last is the global pair index of the last blended
 * entry (-1 if none).  counts[0] += evaluated entries, counts[1] += blends. */
void or_render_fwd(const double *rec, int64_t n, const double *views, int32_t n_views,
                   const uint32_t *vals, const int32_t *ranges, double *image, double *T_final,
                   int32_t *last, int64_t *counts, uint64_t *sig, int32_t f32)
{
    for (int32_t vi = 0; vi < n_views; ++vi) {
        const double *vw = views + (int64_t)vi * OR_VIEW;
        const int W = (int)vw[16], H = (int)vw[17];
        const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
        const int64_t tpv = (int64_t)tiles_x * tiles_y;
        const double *rv = rec + (int64_t)vi * n * OR_REC;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                const int64_t tile = vi * tpv + (int64_t)(y >> 4) * tiles_x + (x >> 4);
                const int32_t b = ranges[2 * tile], e = ranges[2 * tile + 1];
                double C[3], T;
                int64_t lst;
                const int64_t m = e - b;
                or_blend *bl = sig ? (or_blend *)malloc(sizeof(or_blend) * (size_t)(m > 0 ? m : 1)) : NULL;
                const int64_t nb = composite_pixel(rv, vals + b, m, x + 0.5, y + 0.5, C, &T,
                                                   &lst, bl, m, &counts[0], f32);
                counts[1] += nb;
                const int64_t pix = (int64_t)y * W + x;
                const int64_t HW = (int64_t)H * W;
                if (sig) {
                    /* decision signature: which entries blended, which clamped */
                    uint64_t hsh = 1469598103934665603ULL;
                    for (int64_t k = 0; k < nb; ++k) {
                        hsh = (hsh ^ (uint64_t)(bl[k].entry * 2 + bl[k].clamped)) * 1099511628211ULL;
                    }
                    sig[(int64_t)vi * HW + pix] = hsh;
                    free(bl);
                }
                for (int ch = 0; ch < 3; ++ch)
                    image[((int64_t)vi * 3 + ch) * HW + pix] = C[ch] + T * vw[20 + ch];
                T_final[(int64_t)vi * HW + pix] = T;
                last[(int64_t)vi * HW + pix] = lst < 0 ? -1 : (int32_t)(b + lst);
            }
    }
}

/* Trace of one pixel's compositing: for each blend, its alpha and the
 * transmittance in front of it.  Returns the number of blends (<= max_b
 * are written) and the final transmittance in *T_final. */
int64_t or_trace_pixel(const double *rec, int64_t n, const double *views, int32_t vi,
                       const uint32_t *vals, const int32_t *ranges, int32_t x, int32_t y,
                       double *alpha_out, double *T_out, int64_t max_b, double *T_final, int32_t f32)
{
    const double *vw = views + (int64_t)vi * OR_VIEW;
    const int W = (int)vw[16], H = (int)vw[17];
    const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
    const int64_t tile = vi * (int64_t)tiles_x * tiles_y + (int64_t)(y >> 4) * tiles_x + (x >> 4);
    const int32_t b = ranges[2 * tile], e = ranges[2 * tile + 1];
    const int64_t m = e - b;
    or_blend *bl = (or_blend *)malloc(sizeof(or_blend) * (size_t)(m > 0 ? m : 1));
    double C[3];
    int64_t lst, dummy = 0;
    const int64_t nb = composite_pixel(rec + (int64_t)vi * n * OR_REC, vals + b, m, x + 0.5, y + 0.5,
                                       C, T_final, &lst, bl, m, &dummy, f32);
    for (int64_t k = 0; k < nb && k < max_b; ++k) { alpha_out[k] = bl[k].alpha; T_out[k] = bl[k].T; }
    free(bl);
    return nb;
}

/* Brute-force render: every pixel composites ALL visible Gaussians of its
 * view in ascending (FP32 depth bits, id) order, ignoring tiles. */
static const uint32_t *g_sort_bits;
static int cmp_depth_id(const void *pa, const void *pb)
{
    const uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    if (g_sort_bits[a] != g_sort_bits[b]) return g_sort_bits[a] < g_sort_bits[b] ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

void or_render_brute(const double *rec, int64_t n, const double *views, int32_t n_views,
                     const int32_t *touched, const uint32_t *depth_bits, double *image,
                     double *T_final, int32_t f32)
{
    uint32_t *ids = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t vi = 0; vi < n_views; ++vi) {
        const double *vw = views + (int64_t)vi * OR_VIEW;
        const int W = (int)vw[16], H = (int)vw[17];
        int64_t m = 0;
        for (int64_t g = 0; g < n; ++g)
            if (touched[(int64_t)vi * n + g] > 0) ids[m++] = (uint32_t)g;
        g_sort_bits = depth_bits + (int64_t)vi * n;
        qsort(ids, (size_t)m, sizeof(uint32_t), cmp_depth_id);
        const double *rv = rec + (int64_t)vi * n * OR_REC;
        const int64_t HW = (int64_t)H * W;
        int64_t dummy = 0;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double C[3], T;
                int64_t lst;
                composite_pixel(rv, ids, m, x + 0.5, y + 0.5, C, &T, &lst, NULL, 0, &dummy, f32);
                const int64_t pix = (int64_t)y * W + x;
                for (int ch = 0; ch < 3; ++ch)
                    image[((int64_t)vi * 3 + ch) * HW + pix] = C[ch] + T * vw[20 + ch];
                T_final[(int64_t)vi * HW + pix] = T;
            }
    }
    free(ids);
}

/* ------------------------------------------------------------------------- *
 * Render backward (FP64).  For each pixel the forward is recomputed, keeping
 * every blend's alpha and its transmittance in front of it (stored here, not
 * recovered), then walked back to front:
 *   dC/drgb_i = alpha_i T_i;  dC/dalpha_i = T_i (rgb_i - B_i),
 *   B_last = bg,  B_{i-1} = alpha_i rgb_i + (1 - alpha_i) B_i.
 * Through alpha = min(0.99, o_t e^power): zero when clamped to 0.99;
 * otherwise (the exponent's min with 0 passes its derivative through)
 *   dalpha/do_t = e^power, dalpha/dpower = alpha~,
 *   dpower/d(a, b, c) = (-dx^2/2, -dx dy, -dy^2/2),
 *   dpower/dmean = (a dx + b dy, c dy + b dx).
 * grad_rec: [n_views][n][9] = d/d(mx, my, a, b, c, o_t, r, g, b).
 * ------------------------------------------------------------------------- */
void or_render_bwd(const double *rec, int64_t n, const double *views, int32_t n_views,
                   const uint32_t *vals, const int32_t *ranges, const double *dL_dimage,
                   double *grad_rec, int32_t f32)
{
    memset(grad_rec, 0, sizeof(double) * 9 * (size_t)n * (size_t)n_views);
    for (int32_t vi = 0; vi < n_views; ++vi) {
        const double *vw = views + (int64_t)vi * OR_VIEW;
        const int W = (int)vw[16], H = (int)vw[17];
        const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
        const int64_t tpv = (int64_t)tiles_x * tiles_y;
        const int64_t HW = (int64_t)H * W;
        const double *rv = rec + (int64_t)vi * n * OR_REC;
        double *gv = grad_rec + (int64_t)vi * n * 9;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                const int64_t tile = vi * tpv + (int64_t)(y >> 4) * tiles_x + (x >> 4);
                const int32_t b = ranges[2 * tile], e = ranges[2 * tile + 1];
                const int64_t m = e - b;
                or_blend *bl = (or_blend *)malloc(sizeof(or_blend) * (size_t)(m > 0 ? m : 1));
                double C[3], T;
                int64_t lst, dummy = 0;
                const double px = x + 0.5, py = y + 0.5;
                const int64_t nb = composite_pixel(rv, vals + b, m, px, py, C, &T, &lst, bl, m, &dummy,
                                                   f32);
                const int64_t pix = (int64_t)y * W + x;
                double gC[3];
                for (int ch = 0; ch < 3; ++ch) gC[ch] = dL_dimage[((int64_t)vi * 3 + ch) * HW + pix];
                pixel_backward(rv, vals + b, bl, nb, px, py, gC, vw + 20, gv, 0);
                free(bl);
            }
    }
}

/* Backward of the projection (FP64) for one record: d(mean2D, conic) in
 * G[0..4] -> d(conditional mean) Gmu and d(conditional covariance) GSc,
 * through Sigma2D = T Sc T^T + 0.3 I, T = J W, the guard-banded Jacobian and
 * the camera point (no gradient through a clamped coordinate). */
static void proj_bwd_f64(const double *vw, const double mu[3], double Sc[3][3], const double *G,
                         double Gmu[3], double GSc[3][3])
{
    int i, j, k;
    double Wm[3][3];
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) Wm[i][j] = vw[4 * i + j];
    const double fx = vw[12], fy = vw[13];
    const int Wd = (int)vw[16], Hd = (int)vw[17];
    double xc[3];
    for (i = 0; i < 3; ++i) xc[i] = Wm[i][0] * mu[0] + Wm[i][1] * mu[1] + Wm[i][2] * mu[2] + vw[4 * i + 3];
    const double z = xc[2];
    const double limx = 1.3 * (0.5 * Wd / fx), limy = 1.3 * (0.5 * Hd / fy);
    const double ux0 = xc[0] / z, uy0 = xc[1] / z;
    const int clx = (ux0 < -limx) || (ux0 > limx), cly = (uy0 < -limy) || (uy0 > limy);
    const double ux = fmin(fmax(ux0, -limx), limx), uy = fmin(fmax(uy0, -limy), limy);
    double J[2][3] = { { fx / z, 0.0, -fx * ux / z }, { 0.0, fy / z, -fy * uy / z } };
    double T[2][3];
    for (i = 0; i < 2; ++i)
        for (j = 0; j < 3; ++j) {
            T[i][j] = 0.0;
            for (k = 0; k < 3; ++k) T[i][j] += J[i][k] * Wm[k][j];
        }
    double S2[2][2];
    for (i = 0; i < 2; ++i)
        for (j = 0; j < 2; ++j) {
            double acc = 0.0;
            for (k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += T[i][k] * Sc[k][l] * T[j][l];
            S2[i][j] = acc + (i == j ? 0.3 : 0.0);
        }
    const double det = S2[0][0] * S2[1][1] - S2[0][1] * S2[0][1];
    double Qc[2][2] = { { S2[1][1] / det, -S2[0][1] / det }, { -S2[0][1] / det, S2[0][0] / det } };

    /* ---- backward ---- */
    /* conic -> Sigma2D : dL/dS2 = -Q Gq Q, Gq symmetric */
    double Gq[2][2] = { { G[2], 0.5 * G[3] }, { 0.5 * G[3], G[4] } };
    double tmp[2][2], GS2[2][2];
    for (i = 0; i < 2; ++i)
        for (j = 0; j < 2; ++j) tmp[i][j] = Gq[i][0] * Qc[0][j] + Gq[i][1] * Qc[1][j];
    for (i = 0; i < 2; ++i)
        for (j = 0; j < 2; ++j) GS2[i][j] = -(Qc[i][0] * tmp[0][j] + Qc[i][1] * tmp[1][j]);
    /* Sigma2D = T Sc T^T : dL/dSc = T^T GS2 T ; dL/dT = 2 GS2 T Sc */
    double GT[2][3];
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l) acc += T[k][i] * GS2[k][l] * T[l][j];
            GSc[i][j] = acc;
        }
    for (i = 0; i < 2; ++i)
        for (j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (k = 0; k < 2; ++k)
                for (int l = 0; l < 3; ++l) acc += GS2[i][k] * T[k][l] * Sc[l][j];
            GT[i][j] = 2.0 * acc;
        }
    /* T = J W : dL/dJ = GT W^T */
    double GJ[2][3];
    for (i = 0; i < 2; ++i)
        for (j = 0; j < 3; ++j) {
            GJ[i][j] = 0.0;
            for (k = 0; k < 3; ++k) GJ[i][j] += GT[i][k] * Wm[j][k];
        }
    /* J entries -> camera-space point */
    double gx = 0.0, gy = 0.0, gz = 0.0;
    gz += GJ[0][0] * (-fx / (z * z)) + GJ[1][1] * (-fy / (z * z));
    /* J02 = -fx ux / z with ux = x/z unless clamped */
    if (clx) gz += GJ[0][2] * (fx * ux / (z * z));
    else { gx += GJ[0][2] * (-fx / (z * z)); gz += GJ[0][2] * (2.0 * fx * xc[0] / (z * z * z)); }
    if (cly) gz += GJ[1][2] * (fy * uy / (z * z));
    else { gy += GJ[1][2] * (-fy / (z * z)); gz += GJ[1][2] * (2.0 * fy * xc[1] / (z * z * z)); }
    /* mean2D = (fx x/z + cx, fy y/z + cy) */
    gx += G[0] * fx / z;
    gy += G[1] * fy / z;
    gz += -G[0] * fx * xc[0] / (z * z) - G[1] * fy * xc[1] / (z * z);
    /* camera -> conditional mean */
    for (j = 0; j < 3; ++j) Gmu[j] = Wm[0][j] * gx + Wm[1][j] * gy + Wm[2][j] * gz;
}

/* ------------------------------------------------------------------------- *
 * Preprocess backward (FP64): chain rule from d(mean2D, conic, o_t, rgb) per
 * (view, Gaussian) to the 20 raw parameters, summed over views.
 * grad_mu3 (may be NULL): [n_views][n][3], a further gradient of the loss
 * with respect to the conditional mean at the view's time (a colour that
 * depends on the viewing direction puts one there); it joins the
 * projection's before the conditional's chain rule.
 * dparams: [20][n], overwritten.
 * ------------------------------------------------------------------------- */
void or_preprocess_bwd_mu(const double *params, int64_t n, const double *views, int32_t n_views,
                          const double *grad_rec, const double *grad_mu3, double *dparams)
{
    memset(dparams, 0, sizeof(double) * 20 * (size_t)n);
    for (int32_t vi = 0; vi < n_views; ++vi) {
        const double *vw = views + (int64_t)vi * OR_VIEW;
        for (int64_t g = 0; g < n; ++g) {
            double rec[OR_REC];
            int32_t rect[4], touched;
            if (!preprocess_one_f64(params, n, g, vw, rec, rect, &touched)) continue;
            const double *G = grad_rec + ((int64_t)vi * n + g) * 9;
            double v[20];
            int i, j, k;
            for (k = 0; k < 20; ++k) v[k] = params[(int64_t)k * n + g];
            const double t = vw[18];

            /* ---- recompute forward intermediates ---- */
            double s[4];
            for (k = 0; k < 4; ++k) s[k] = exp(v[4 + k]);
            const double o = 1.0 / (1.0 + exp(-v[16]));
            const double nl = sqrt(v[8] * v[8] + v[9] * v[9] + v[10] * v[10] + v[11] * v[11]);
            const double nr = sqrt(v[12] * v[12] + v[13] * v[13] + v[14] * v[14] + v[15] * v[15]);
            double ql[4], qr[4];
            for (k = 0; k < 4; ++k) { ql[k] = v[8 + k] / nl; qr[k] = v[12 + k] / nr; }
            double A[4][4] = { { ql[0], -ql[1], -ql[2], -ql[3] }, { ql[1], ql[0], -ql[3], ql[2] },
                               { ql[2], ql[3], ql[0], -ql[1] }, { ql[3], -ql[2], ql[1], ql[0] } };
            double B[4][4] = { { qr[0], -qr[1], -qr[2], -qr[3] }, { qr[1], qr[0], qr[3], -qr[2] },
                               { qr[2], -qr[3], qr[0], qr[1] }, { qr[3], qr[2], -qr[1], qr[0] } };
            double Q[4][4];
            for (i = 0; i < 4; ++i)
                for (j = 0; j < 4; ++j) {
                    Q[i][j] = 0.0;
                    for (k = 0; k < 4; ++k) Q[i][j] += A[i][k] * B[k][j];
                }
            static const int perm[4] = { 1, 2, 3, 0 };
            double R[4][4], M[4][4], Sg[4][4];
            for (i = 0; i < 4; ++i)
                for (j = 0; j < 4; ++j) { R[i][j] = Q[perm[i]][perm[j]]; M[i][j] = R[i][j] * s[j]; }
            for (i = 0; i < 4; ++i)
                for (j = 0; j < 4; ++j) {
                    Sg[i][j] = 0.0;
                    for (k = 0; k < 4; ++k) Sg[i][j] += M[i][k] * M[j][k];
                }
            const double c = Sg[3][3], dt = t - v[3];
            double a3[3], mu[3], Sc[3][3];
            for (i = 0; i < 3; ++i) { a3[i] = Sg[i][3]; mu[i] = v[i] + a3[i] * dt / c; }
            for (i = 0; i < 3; ++i)
                for (j = 0; j < 3; ++j) Sc[i][j] = Sg[i][j] - a3[i] * a3[j] / c;
            const double ef = exp(-0.5 * dt * dt / c);
            const double ot = o * ef;
            double Gmu[3], GSc[3][3];
            proj_bwd_f64(vw, mu, Sc, G, Gmu, GSc);
            if (grad_mu3)
                for (i = 0; i < 3; ++i) Gmu[i] += grad_mu3[((int64_t)vi * n + g) * 3 + i];
            /* conditional -> Sigma blocks, mean, opacity */
            const double go = G[5];
            double Gmua = Gmu[0] * a3[0] + Gmu[1] * a3[1] + Gmu[2] * a3[2];
            double aGa = 0.0, Ga[3];
            for (i = 0; i < 3; ++i) {
                Ga[i] = 0.0;
                for (j = 0; j < 3; ++j) { aGa += a3[i] * GSc[i][j] * a3[j]; Ga[i] += GSc[i][j] * a3[j]; }
            }
            double dmu[4];
            for (i = 0; i < 3; ++i) dmu[i] = Gmu[i];
            dmu[3] = -Gmua / c + go * ot * dt / c;
            double Gda[3];
            for (i = 0; i < 3; ++i) Gda[i] = Gmu[i] * dt / c - 2.0 * Ga[i] / c;
            const double Gdc = -Gmua * dt / (c * c) + aGa / (c * c) + go * ot * dt * dt / (2.0 * c * c);
            const double Gdo = go * ef;
            /* symmetric 4x4 gradient of Sigma */
            double G4[4][4];
            for (i = 0; i < 3; ++i)
                for (j = 0; j < 3; ++j) G4[i][j] = GSc[i][j];
            for (i = 0; i < 3; ++i) { G4[i][3] = 0.5 * Gda[i]; G4[3][i] = 0.5 * Gda[i]; }
            G4[3][3] = Gdc;
            /* Sigma = M M^T : dL/dM = 2 G4 M */
            double GM[4][4];
            for (i = 0; i < 4; ++i)
                for (j = 0; j < 4; ++j) {
                    GM[i][j] = 0.0;
                    for (k = 0; k < 4; ++k) GM[i][j] += 2.0 * G4[i][k] * M[k][j];
                }
            double GR[4][4], Gs[4] = { 0, 0, 0, 0 };
            for (i = 0; i < 4; ++i)
                for (j = 0; j < 4; ++j) { GR[i][j] = GM[i][j] * s[j]; Gs[j] += GM[i][j] * R[i][j]; }
            /* R = Pi Q Pi^T : dL/dQ[perm i][perm j] = GR[i][j] */
            double GQ[4][4];
            for (i = 0; i < 4; ++i)
                for (j = 0; j < 4; ++j) GQ[perm[i]][perm[j]] = GR[i][j];
            /* Q = A B : dL/dA = GQ B^T, dL/dB = A^T GQ */
            double GA[4][4], GB[4][4];
            for (i = 0; i < 4; ++i)
                for (j = 0; j < 4; ++j) {
                    GA[i][j] = 0.0; GB[i][j] = 0.0;
                    for (k = 0; k < 4; ++k) { GA[i][j] += GQ[i][k] * B[j][k]; GB[i][j] += A[k][i] * GQ[k][j]; }
                }
            /* matrix entries -> unit quaternion components */
            double gql[4], gqr[4];
            gql[0] = GA[0][0] + GA[1][1] + GA[2][2] + GA[3][3];
            gql[1] = -GA[0][1] + GA[1][0] - GA[2][3] + GA[3][2];
            gql[2] = -GA[0][2] + GA[1][3] + GA[2][0] - GA[3][1];
            gql[3] = -GA[0][3] - GA[1][2] + GA[2][1] + GA[3][0];
            gqr[0] = GB[0][0] + GB[1][1] + GB[2][2] + GB[3][3];
            gqr[1] = -GB[0][1] + GB[1][0] + GB[2][3] - GB[3][2];
            gqr[2] = -GB[0][2] - GB[1][3] + GB[2][0] + GB[3][1];
            gqr[3] = -GB[0][3] + GB[1][2] - GB[2][1] + GB[3][0];
            /* normalisation: dL/dq = (g - qhat (qhat . g)) / |q| */
            double dl = 0.0, dr = 0.0;
            for (k = 0; k < 4; ++k) { dl += ql[k] * gql[k]; dr += qr[k] * gqr[k]; }
            double *dp = dparams;
            for (k = 0; k < 4; ++k) {
                dp[(int64_t)k * n + g] += dmu[k];
                dp[(int64_t)(4 + k) * n + g] += Gs[k] * s[k];
                dp[(int64_t)(8 + k) * n + g] += (gql[k] - ql[k] * dl) / nl;
                dp[(int64_t)(12 + k) * n + g] += (gqr[k] - qr[k] * dr) / nr;
            }
            dp[(int64_t)16 * n + g] += Gdo * o * (1.0 - o);
            for (k = 0; k < 3; ++k) dp[(int64_t)(17 + k) * n + g] += G[6 + k];
        }
    }
}

void or_preprocess_bwd(const double *params, int64_t n, const double *views, int32_t n_views,
                       const double *grad_rec, double *dparams)
{
    or_preprocess_bwd_mu(params, n, views, n_views, grad_rec, NULL, dparams);
}

/* ------------------------------------------------------------------------- *
 * Preprocess backward of the isotropic, motion-aware form (FP64), summed
 * over views; dparams [13][n] overwritten.  With dt = t - mu_t and
 * c = s_t^2:
 *   mu_c = mu + v dt    -> d mu += Gmu, d v += Gmu dt, d mu_t -= v . Gmu;
 *   Sc = s^2 I          -> d log s = 2 s^2 trace(GSc);
 *   o_t = o exp(-dt^2 / (2c)) -> d mu_t += go o_t dt / c,
 *                          d log s_t = go o_t dt^2 / c,
 *                          d logit = go exp(-dt^2 / (2c)) o (1 - o).
 * ------------------------------------------------------------------------- */
void or_preprocess_iso_bwd(const double *params, int64_t n, const double *views, int32_t n_views,
                           const double *grad_rec, double *dparams)
{
    memset(dparams, 0, sizeof(double) * 13 * (size_t)n);
    for (int32_t vi = 0; vi < n_views; ++vi) {
        const double *vw = views + (int64_t)vi * OR_VIEW;
        for (int64_t g = 0; g < n; ++g) {
            double rec[OR_REC];
            int32_t rect[4], touched;
            if (!preprocess_iso_one_f64(params, n, g, vw, rec, rect, &touched)) continue;
            const double *G = grad_rec + ((int64_t)vi * n + g) * 9;
            double v[13], d[13];
            int i, k;
            for (k = 0; k < 13; ++k) { v[k] = params[(int64_t)k * n + g]; d[k] = 0.0; }
            const double t = vw[18];
            const double s = exp(v[4]), st = exp(v[5]);
            const double o = 1.0 / (1.0 + exp(-v[9]));
            const double c = st * st, dt = t - v[3];
            double mu[3], Sc[3][3] = { { s * s, 0.0, 0.0 }, { 0.0, s * s, 0.0 }, { 0.0, 0.0, s * s } };
            for (i = 0; i < 3; ++i) mu[i] = v[i] + v[6 + i] * dt;
            const double ef = exp(-0.5 * dt * dt / c), ot = o * ef;
            double Gmu[3], GSc[3][3];
            proj_bwd_f64(vw, mu, Sc, G, Gmu, GSc);
            const double go = G[5];
            double vG = 0.0;
            for (i = 0; i < 3; ++i) {
                d[i] += Gmu[i];
                d[6 + i] += Gmu[i] * dt;
                vG += v[6 + i] * Gmu[i];
            }
            d[3] += -vG + go * ot * dt / c;
            d[4] += 2.0 * s * s * (GSc[0][0] + GSc[1][1] + GSc[2][2]);
            d[5] += go * ot * dt * dt / c;
            d[9] += go * ef * o * (1.0 - o);
            for (k = 0; k < 3; ++k) d[10 + k] += G[6 + k];
            for (k = 0; k < 13; ++k) dparams[(int64_t)k * n + g] += d[k];
        }
    }
}

/* ------------------------------------------------------------------------- *
 * Grid pruning (Sec. 3.2).  Each point is assigned to a voxel by integer
 * division with the voxel edge -- read as floor(x / S_v), so that the cells
 * on either side of 0 stay distinct -- per motion class (the static and
 * dynamic edge lengths of the Lite/Full presets, Sec. 4.1).  Points of the
 * same (class, voxel) are replaced by their centroid and the mean of their
 * attributes; voxels with fewer than min_count points are discarded.  A
 * class whose edge length is <= 0 is not pruned: each of its points is its
 * own cell, in input order.
 *
 * key (uint64): bit 63 = class, bit 62 = unpruned flag,
 *   pruned:   three 20-bit fields (ix + 2^19) << 40 | (iy + 2^19) << 20 | (iz + 2^19),
 *             so a voxel index must lie in [-2^19, 2^19);
 *   unpruned: low 62 bits = point index.
 * Output is ascending by key.  Sums are accumulated in FP64.
 * xyz [3][m], attr [k][m], cls [m] (NULL -> all class 0)
 * Returns the number of output cells, or -1 for a voxel index out of range,
 * -2 for output over capacity.
 * ------------------------------------------------------------------------- */
typedef struct { uint64_t key; int64_t idx; } or_kv;
static int cmp_kv(const void *pa, const void *pb)
{
    const or_kv *a = (const or_kv *)pa, *b = (const or_kv *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

int64_t or_grid_prune(const float *xyz, const float *attr, int32_t k_attr, const uint8_t *cls,
                      int64_t m, float voxel_static, float voxel_dynamic, int32_t min_count,
                      int64_t capacity, float *out_xyz, float *out_attr, int32_t *out_count,
                      uint64_t *out_key)
{
    or_kv *kv = (or_kv *)malloc(sizeof(or_kv) * (size_t)(m > 0 ? m : 1));
    for (int64_t i = 0; i < m; ++i) {
        const int c = cls ? (cls[i] ? 1 : 0) : 0;
        const float vs = c ? voxel_dynamic : voxel_static;
        uint64_t key = (uint64_t)c << 63;
        if (!(vs > 0.0f)) {
            key |= (1ULL << 62) | (uint64_t)i;
        } else {
            int64_t q[3];
            for (int a = 0; a < 3; ++a) {
                const double f = floor((double)(xyz[(int64_t)a * m + i] / vs));
                if (!(f >= -524288.0 && f <= 524287.0)) { free(kv); return -1; }
                q[a] = (int64_t)f + 524288;
            }
            key |= ((uint64_t)q[0] << 40) | ((uint64_t)q[1] << 20) | (uint64_t)q[2];
        }
        kv[i].key = key;
        kv[i].idx = i;
    }
    qsort(kv, (size_t)m, sizeof(or_kv), cmp_kv);
    int64_t nout = 0;
    double *acc = (double *)malloc(sizeof(double) * (size_t)(3 + k_attr));
    for (int64_t s = 0; s < m;) {
        int64_t e = s;
        while (e < m && kv[e].key == kv[s].key) ++e;
        const int64_t cnt = e - s;
        if (cnt >= min_count) {
            if (nout >= capacity) { free(acc); free(kv); return -2; }
            for (int a = 0; a < 3 + k_attr; ++a) acc[a] = 0.0;
            for (int64_t i = s; i < e; ++i) {
                const int64_t p = kv[i].idx;
                for (int a = 0; a < 3; ++a) acc[a] += (double)xyz[(int64_t)a * m + p];
                for (int a = 0; a < k_attr; ++a) acc[3 + a] += (double)attr[(int64_t)a * m + p];
            }
            for (int a = 0; a < 3; ++a) out_xyz[(int64_t)a * capacity + nout] = (float)(acc[a] / (double)cnt);
            for (int a = 0; a < k_attr; ++a)
                out_attr[(int64_t)a * capacity + nout] = (float)(acc[3 + a] / (double)cnt);
            out_count[nout] = (int32_t)cnt;
            out_key[nout] = kv[s].key;
            ++nout;
        }
        s = e;
    }
    free(acc);
    free(kv);
    return nout;
}
