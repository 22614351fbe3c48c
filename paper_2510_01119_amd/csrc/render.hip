// Per-tile alpha compositing, forward and backward (the Gaussian-splatting
// renderer of Sec. 3.1; the backward of Table B-1 "Backward").
//
// A workgroup renders one 16x16 tile at a time: one workgroup per tile, or
// persistent workgroups walking the (view, tile) work list (from a shared
// counter, or a fixed share of it).  Its four wave64 each own a pixel block
// of the tile (8x8 at one pixel per lane; the backward's 2- and 4-pixel-per-
// lane variants use 8x16 and 16x16 with 128 and 64 threads).  The tile's
// sorted Gaussians are staged through LDS in batches; each wave walks the
// entries whose alpha >= 1/255 ellipse meets its block, with broadcast LDS
// reads.  Early termination: a pixel stops when its transmittance would fall
// below 1e-4; the workgroup leaves the tile as soon as no pixel is active.
//
// Backward: each pixel replays its entries back to front from the last
// blended one, recovering T_i = T_{i+1} / (1 - alpha_i) from T_final (no
// per-entry state is stored by the forward).  Each entry's nine gradient
// terms are summed over the wave with cross-lane reductions (skipped when
// no lane of the wave touched the entry), then over the four waves through
// LDS, and land in HBM with one atomic per (tile, Gaussian, term).
#include "common.hpp"

namespace gs4d {

namespace {

constexpr int RT_THREADS = 256;
constexpr int RT_WAVES = 4;
constexpr float ALPHA_MAX = 0.99f;
constexpr float T_EPS = 1e-4f;
// backward stages 128 Gaussians per round (per-wave partial sums: 18 KB of LDS)
constexpr int BWD_BATCH = 128;

struct TileInfo {
    int v, tx, ty;
};

__device__ __forceinline__ TileInfo tile_info(int64_t tile, const ViewPack &vp) {
    TileInfo ti;
    ti.v = (int)(tile / vp.tiles_per_view);
    const int lt = (int)(tile - (int64_t)ti.v * vp.tiles_per_view);
    ti.ty = lt / vp.tiles_x;
    ti.tx = lt - ti.ty * vp.tiles_x;
    return ti;
}

// The exponent of a Gaussian at pixel offset d = (dx, dy), in log2 units so
// that it feeds the hardware exp2 directly:
//   arg = min(0, -(1/2) log2(e) (dx qx + dy qy)),  (qx, qy) = Q d,
// Q = [[a, b], [b, c]] the conic; alpha~ = o_t 2^arg.  The conic of a visible
// record is positive definite (positive determinant, 0.3 px^2 dilation on
// the diagonal), so the quadratic form is >= 0 in exact arithmetic; the min
// with 0 only absorbs rounding (alpha never exceeds o_t, and the pixel stays
// continuous where the form passes 0).  Its derivative is the form's own.
// (qx, qy) are returned: the exponent's gradient with respect to the mean
// is -(1/2) of d/dd of the form, i.e. +Q d in natural units.  The forward
// and the backward evaluate this same instruction sequence.
constexpr float NEG_HALF_LOG2E = -0.72134752044448170368f;   // -(1/2) log2 e
constexpr float NEG_LOG2E = -1.44269504088896340736f;        // -log2 e
constexpr float LN2 = 0.69314718055994530942f;

__device__ __forceinline__ float gauss_arg(float4 a, float cc, float dx, float dy, float &qx,
                                           float &qy) {
    qx = fmaf(a.z, dx, a.w * dy);
    qy = fmaf(cc, dy, a.w * dx);
    return fminf(fmaf(dx, qx, dy * qy) * NEG_HALF_LOG2E, 0.0f);
}

// The alpha >= 1/255 floor as a bound on the exponent: o_t 2^arg >= 1/255
// iff arg >= lo = -log2(255 o_t) = -ln(255 o_t) log2 e.  Both operands are
// FP32 values with a fixed evaluation order (gauss_arg; the project-defined
// logarithm), so the decision to skip an entry is reproducible bit for bit.
__device__ __forceinline__ float alpha_floor(float o_t) {
    return fixed_log(255.0f * o_t) * NEG_LOG2E;
}

// Each wave owns a block of pixels of the tile.  For a staged batch, every
// wave marks (one ballot per 64 entries) the entries whose alpha >= 1/255
// ellipse meets its block (footprint box test, then the exact minimum of
// the quadratic form over the block); for the others alpha < 1/255 at every
// pixel of the block, so they are skipped without evaluating them -- the
// result is the same as evaluating them.
// Pixel block of one wave inside its 16x16 tile: BW columns by BH rows.
// PPL (pixels per lane) 1 and 2 use 8-wide blocks (8x8, 8x16): squarer
// blocks meet fewer footprints than 16-wide strips of the same area.  Lane l
// covers column l mod BW and rows l div BW + k * RPS, k < PPL.
template <int PPL>
struct WaveBlock {
    static constexpr int BW = PPL == 4 ? 16 : 8;
    static constexpr int RPS = 64 / BW;
    static constexpr int BH = RPS * PPL;
    static constexpr int CB = GS4D_TILE / BW;
};

template <int BATCH>
__device__ __forceinline__ void strip_masks(const float4 *sA, const float4 *sB, const float4 *sC,
                                            int cnt, float x0, float x1, float y0, float y1,
                                            int lane, uint64_t (&m)[BATCH / 64]) {
#pragma unroll
    for (int k = 0; k < BATCH / 64; ++k) {
        const int j = k * 64 + lane;
        bool hit = false;
        if (j < cnt) {
            const float4 a = sA[j];
            const float4 c = sC[j];   // b, lo, hx, hy
            hit = (a.x + c.z >= x0) && (a.x - c.z <= x1) && (a.y + c.w >= y0) && (a.y - c.w <= y1);
            if (hit) {
                // Refine: the alpha >= 1/255 ellipse q(d) = a dx^2 + 2 b dx dy + c dy^2
                // <= tau must meet the block's rectangle of pixel centres.  q is convex, so
                // its minimum over the rectangle is 0 (centre inside) or on an edge,
                // where it is the clamped 1D minimum.  Each candidate is lowered by
                // a bound on its FP32 rounding (its terms can cancel), and tau
                // carries the footprint's padding, so no entry that reaches
                // alpha >= 1/255 at a pixel of the block is dropped.
                // tau = 2 ln(255 o_t) = -2 lo ln 2, padded like the footprint
                // (relative and absolute 2^-10) plus 2^-12
                const float ca = a.z, cb = a.w, cc = sB[j].x;
                const float tau =
                    fmaf(-2.0f * LN2 * c.y, 1.0f + 1.25f / 1024.0f, 1.25f / 1024.0f);
                const float X0 = x0 - a.x, X1 = x1 - a.x, Y0 = y0 - a.y, Y1 = y1 - a.y;
                const bool inside = X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f;
                const float ia = __builtin_amdgcn_rcpf(ca), ic = __builtin_amdgcn_rcpf(cc);
                float qmin = __builtin_inff();
                auto edge = [&](float X, float Y) {
                    const float t1 = ca * X * X, t2 = 2.0f * cb * X * Y, t3 = cc * Y * Y;
                    const float q = t1 + t2 + t3;
                    qmin = fminf(qmin, q - 1e-5f * (t1 + fabsf(t2) + t3));
                };
                edge(X0, fminf(fmaxf(-cb * X0 * ic, Y0), Y1));
                edge(X1, fminf(fmaxf(-cb * X1 * ic, Y0), Y1));
                edge(fminf(fmaxf(-cb * Y0 * ia, X0), X1), Y0);
                edge(fminf(fmaxf(-cb * Y1 * ia, X0), X1), Y1);
                hit = inside || qmin <= tau;
            }
        }
        m[k] = __ballot(hit);
    }
}

template <int BATCH>
__device__ __forceinline__ void stage_batch(const float4 *__restrict__ recv,
                                            const uint32_t *__restrict__ vals, int start, int cnt,
                                            float4 *sA, float4 *sB, float4 *sC, uint32_t *sG) {
    const int t = threadIdx.x;
    if (t < cnt) {
        const uint32_t g = vals[start + t];
        const float4 r0 = recv[3 * (int64_t)g + 0];
        const float4 r1 = recv[3 * (int64_t)g + 1];
        const float4 r2 = recv[3 * (int64_t)g + 2];
        sA[t] = r0;                                       // mx my ca cb
        sB[t] = make_float4(r1.x, r1.y, r2.x, r2.y);      // cc o_t r g
        // b, lo, hx, hy.  lo = -log2(255 o_t): alpha = o_t 2^arg >= 1/255 iff
        // arg >= lo, the form in which the floor is decided (FP32, the
        // project-defined logarithm, so the decision is reproducible bit for bit)
        sC[t] = make_float4(r2.z, alpha_floor(r1.y), r1.w, r2.w);
        if (sG) sG[t] = g;
    }
}

// Static schedule of a persistent launch (mode 2): round r hands the
// workgroups the work-list positions base .. base + gridDim - 1, base =
// r * gridDim, workgroup i taking the i-th of them in even rounds and the
// (gridDim - 1 - i)-th in odd ones, so over a largest-first list each
// workgroup's long and short tiles alternate.  No counter is touched.
__device__ __forceinline__ int64_t static_position(int64_t r, int64_t base) {
    return base + ((r & 1) ? (int64_t)gridDim.x - 1 - blockIdx.x : (int64_t)blockIdx.x);
}

// COUNT: count evaluated and blended (pixel, entry) pairs into o.counters
// (a separate instantiation, so the plain forward carries no counting).
template <int BATCH, bool COUNT>
__device__ __forceinline__ void render_tile_fwd(int64_t tile, const float4 *__restrict__ rec,
                                                int64_t n, const uint32_t *__restrict__ vals,
                                                const int2 *__restrict__ ranges,
                                                const ViewPack &vp, const gs4d_render_opts &o,
                                                float *__restrict__ image,
                                                float *__restrict__ T_final,
                                                int32_t *__restrict__ last_out, float4 *sA,
                                                float4 *sB, float4 *sC) {
    using B = WaveBlock<1>;
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const TileInfo ti = tile_info(tile, vp);
    const int bx = ti.tx * GS4D_TILE + (w % B::CB) * B::BW;
    const int by = ti.ty * GS4D_TILE + (w / B::CB) * B::BH;
    const int px = bx + lane % B::BW;
    const int py = by + lane / B::BW;
    const int W = vp.width, H = vp.height;
    const bool inside = px < W && py < H;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    // this wave's block, as pixel-centre extents
    const float sx0 = (float)bx + 0.5f, sx1 = sx0 + (float)(B::BW - 1);
    const float sy0 = (float)by + 0.5f, sy1 = sy0 + (float)(B::BH - 1);
    const int2 rg = ranges[tile];
    const float4 *recv = rec + (int64_t)ti.v * n * 3;

    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    int32_t last = -1;
    uint32_t n_eval = 0, n_blend = 0, n_eval_last = 0;
    bool done = !inside;

    for (int start = rg.x; start < rg.y; start += BATCH) {
        const int cnt = min(BATCH, rg.y - start);
        __syncthreads();
        stage_batch<BATCH>(recv, vals, start, cnt, sA, sB, sC, nullptr);
        const int active = __syncthreads_count(!done);
        if (active == 0) break;
        if (__ballot(!done) == 0) continue;
        uint64_t m[BATCH / 64];
        strip_masks<BATCH>(sA, sB, sC, cnt, sx0, sx1, sy0, sy1, lane, m);
        // Branch-free per entry: every decision is a select, so the only
        // control flow is the wave-uniform walk over the mask bits; two
        // entries per step keep two sets of LDS reads in flight.
        auto blend_one = [&](int j, float4 a, float4 b, float2 c) {
            const bool live = !done;
            const float dx = fx - a.x, dy = fy - a.y;
            float qx, qy;
            const float arg = gauss_arg(a, b.x, dx, dy, qx, qy);
            const float at = b.y * __builtin_amdgcn_exp2f(arg);
            const float alpha = fminf(ALPHA_MAX, at);
            const bool ok = live && !(arg < c.y);   // alpha >= 1/255
            const float cb_ = c.x;
            const float Tn = T * (1.0f - alpha);
            const bool stop = ok && (Tn < T_EPS);
            const bool blend = ok && !stop;
            const float wgt = blend ? alpha * T : 0.0f;
            C0 = fmaf(b.z, wgt, C0);
            C1 = fmaf(b.w, wgt, C1);
            C2 = fmaf(cb_, wgt, C2);
            T = blend ? Tn : T;
            last = blend ? start + j : last;
            done = done || stop;
            if (COUNT) {
                n_eval += live ? 1u : 0u;
                n_blend += blend ? 1u : 0u;
                n_eval_last = blend ? n_eval : n_eval_last;
            }
        };
#pragma unroll
        for (int k = 0; k < BATCH / 64; ++k) {
            uint64_t mask = m[k];
            while (mask) {
                if (__ballot(!done) == 0) break;
                const int j0 = k * 64 + __builtin_ctzll(mask);
                mask &= mask - 1;
                const bool two = mask != 0;
                const int j1 = two ? k * 64 + __builtin_ctzll(mask) : j0;
                if (two) mask &= mask - 1;
                const float4 a0 = sA[j0], b0 = sB[j0];
                const float2 c0 = make_float2(sC[j0].x, sC[j0].y);
                const float4 a1 = sA[j1], b1 = sB[j1];
                const float2 c1 = make_float2(sC[j1].x, sC[j1].y);
                blend_one(j0, a0, b0, c0);
                if (two) blend_one(j1, a1, b1, c1);
            }
        }
    }

    const gs4d_view &V = vp.v[ti.v];
    const int64_t HW = (int64_t)H * W;
    float lsum = 0.0f;
    if (inside) {
        const int64_t pix = (int64_t)py * W + px;
        float out[3] = {C0 + T * V.bg[0], C1 + T * V.bg[1], C2 + T * V.bg[2]};
        float *img = image + (int64_t)ti.v * 3 * HW + pix;
        img[0] = out[0];
        img[HW] = out[1];
        img[2 * HW] = out[2];
        if (T_final) {   // null in forward-only rendering (no state for a backward)
            T_final[(int64_t)ti.v * HW + pix] = T;
            last_out[(int64_t)ti.v * HW + pix] = last;
        }
        if (o.target) {
            const float *tg = o.target + (int64_t)ti.v * 3 * HW + pix;
            const float scale = o.l1_weight / (float)(3 * HW);
            for (int c = 0; c < 3; ++c) {
                const float d = out[c] - tg[c * HW];
                lsum += fabsf(d);
                if (o.dL_dimage)
                    o.dL_dimage[(int64_t)ti.v * 3 * HW + pix + c * HW] =
                        d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
            }
        }
    }
    if (o.target && o.loss_per_view) {
        const float s = wave_sum(lsum);
        if (lane == 0 && s != 0.0f)
            atomicAdd(&o.loss_per_view[ti.v], s * (o.l1_weight / (float)(3 * HW)));
    }
    if (COUNT) {
        const uint32_t e = wave_sum_u32(n_eval);
        const uint32_t bl = wave_sum_u32(n_blend);
        const uint32_t el = wave_sum_u32(n_eval_last);
        if (lane == 0) {
            atomicAdd((unsigned long long *)&o.counters[0], (unsigned long long)e);
            atomicAdd((unsigned long long *)&o.counters[1], (unsigned long long)bl);
            atomicAdd((unsigned long long *)&o.counters[2], (unsigned long long)el);
        }
    }
}

template <int BATCH, bool COUNT>
__global__ void __launch_bounds__(RT_THREADS)
render_fwd_kernel(const float4 *__restrict__ rec, int64_t n, const uint32_t *__restrict__ vals,
                  const int2 *__restrict__ ranges, ViewPack vp, gs4d_render_opts o,
                  float *__restrict__ image, float *__restrict__ T_final,
                  int32_t *__restrict__ last) {
    __shared__ float4 sA[BATCH];
    __shared__ float4 sB[BATCH];
    __shared__ float4 sC[BATCH];
    const int64_t n_tiles = (int64_t)vp.tiles_per_view * vp.n_views;
    if (!o.persistent) {
        render_tile_fwd<BATCH, COUNT>(blockIdx.x, rec, n, vals, ranges, vp, o, image, T_final,
                                      last, sA, sB, sC);
        return;
    }
    if (o.persistent == 2) {
        for (int64_t r = 0, base = 0; base < n_tiles; ++r, base += gridDim.x) {
            const int64_t k = static_position(r, base);
            if (k < n_tiles) {
                const int64_t tile = o.order ? o.order[k] : k;
                render_tile_fwd<BATCH, COUNT>(tile, rec, n, vals, ranges, vp, o, image, T_final,
                                              last, sA, sB, sC);
            }
            __syncthreads();
        }
        return;
    }
    // Work list position k: a workgroup's first is its own index, the later
    // ones come from the counter offset by the grid size, so the launch does
    // not start with every workgroup hitting one counter (same-address
    // atomics serialise).
    __shared__ int next;
    for (int k = blockIdx.x; k < n_tiles;) {
        const int64_t tile = o.order ? o.order[k] : k;
        render_tile_fwd<BATCH, COUNT>(tile, rec, n, vals, ranges, vp, o, image, T_final, last, sA,
                                      sB, sC);
        __syncthreads();
        if (threadIdx.x == 0) next = (int)gridDim.x + atomicAdd(o.queue, 1);
        __syncthreads();
        k = next;
    }
}

// ---------------------------------------------------------------- backward
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float x) {
    // bound_ctrl: a source lane outside the row reads 0, so `x + dpp_f(x)`
    // folds into one v_add_f32_dpp with no zero-initialised temporary
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, true));
}

// Exchange of two registers between wave halves / 16-lane rows (gfx950):
// swap32 gives x = [x lanes 0-31, y lanes 0-31], y = [x lanes 32-63,
// y lanes 32-63]; swap16 gives x = [x row 0, y row 0, x row 2, y row 2],
// y = [x row 1, y row 1, x row 3, y row 3].  x + y afterwards sums two
// terms at once, each over half of the lanes.
__device__ __forceinline__ void swap32(float &x, float &y) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                    false);
    x = __uint_as_float(r[0]);
    y = __uint_as_float(r[1]);
}

__device__ __forceinline__ void swap16(float &x, float &y) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                    false);
    x = __uint_as_float(r[0]);
    y = __uint_as_float(r[1]);
}

// Reduce-scatter of the nine gradient terms of one entry over the wave.
// Terms 0-7 are paired across the halves (4 swaps + adds), then across rows
// (2 swaps + adds), leaving two registers whose 16-lane row sums are wave
// totals: lane 15 of row r holds in x[m] the total of term 4m + t(r),
// t = (0, 2, 1, 3).  Row sums: after row_shr 1/2/4 (bound_ctrl: lanes
// shifted in read 0) lane 15 of a row holds the sum of lanes 8..15 and lane
// 7 that of lanes 0..7, so x += row_ror:8(x) completes it -- one fused DPP
// add per register with every lane active (register operands only; the
// s_nop covers the two wait states a DPP read needs after a VALU write).
// Term 8 is summed on its own (row_shr 1/2/4/8, then row_bcast:15 into rows
// 1 and 3 and row_bcast:31 into rows 2 and 3): its total ends in lane 63,
// returned in x[2].
__device__ __forceinline__ void wave_scatter9(const float (&d)[9], float (&x)[3]) {
    float a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float p = d[2 * k], q = d[2 * k + 1];
        swap32(p, q);
        a[k] = p + q;
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        float p = a[2 * m], q = a[2 * m + 1];
        swap16(p, q);
        x[m] = p + q;
    }
    float e = d[8];
    x[0] += dpp_f<0x111, 0xF>(x[0]);
    x[1] += dpp_f<0x111, 0xF>(x[1]);
    e += dpp_f<0x111, 0xF>(e);
    x[0] += dpp_f<0x112, 0xF>(x[0]);
    x[1] += dpp_f<0x112, 0xF>(x[1]);
    e += dpp_f<0x112, 0xF>(e);
    x[0] += dpp_f<0x114, 0xF>(x[0]);
    x[1] += dpp_f<0x114, 0xF>(x[1]);
    e += dpp_f<0x114, 0xF>(e);
    e += dpp_f<0x118, 0xF>(e);   // row_shr:8 -> lane 15 of each row: the row's sum
    // rows outside a DPP row_mask are not written, so the broadcasts add
    // into rows 1 and 3, then 2 and 3 only
    asm volatile(
        "s_nop 1\n"
        "v_add_f32_dpp %0, %0, %0 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %1, %1, %1 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %2, %2, %2 row_bcast:15 row_mask:0xa bank_mask:0xf\n"
        "s_nop 1\n"
        "v_add_f32_dpp %2, %2, %2 row_bcast:31 row_mask:0xc bank_mask:0xf\n"
        : "+v"(x[0]), "+v"(x[1]), "+v"(e));
    x[2] = e;
}

// PPL = pixels per lane.  The workgroup has 256 / PPL threads; wave w owns
// the block given by WaveBlock<PPL> (8x8 for PPL 1, 8x16 for PPL 2, 16x16
// for PPL 4).  Each lane folds its PPL pixels' terms for an entry before the
// cross-lane reduction.
//
// Reduction of the nine gradient terms of one entry over one wave: a
// reduce-scatter in registers (wave_scatter9) leaves the wave totals in the
// four row-leader lanes, which store them into LDS slots
// part[wave][entry][term].  After the batch, each entry's slots are summed
// over the waves and added to HBM with one atomic per term.  A wave skips every entry its block test
// rejects and every entry no lane of it actually blends; the per-wave,
// per-row "written" masks record which slots hold data.
template <int BATCH, int PPL>
struct BwdShared {
    float4 sA[BATCH];
    float4 sB[BATCH];
    float4 sC[BATCH];
    uint32_t sG[BATCH];
    // [wave][entry * 9 + term]
    float part[RT_THREADS / PPL / 64][BATCH * 9];
    uint64_t written[RT_THREADS / PPL / 64][BATCH / 64];
    int smax;
};

template <int BATCH, int PPL>
__device__ __forceinline__ void render_tile_bwd(int64_t tile, const float4 *__restrict__ rec,
                                                int64_t n, const uint32_t *__restrict__ vals,
                                                const int2 *__restrict__ ranges, const ViewPack &vp,
                                                const float *__restrict__ dL_dimage,
                                                const float *__restrict__ T_final,
                                                const int32_t *__restrict__ last,
                                                float *__restrict__ grad2d,
                                                BwdShared<BATCH, PPL> &sh) {
    constexpr int NK = BATCH / 64;
    constexpr int NT = RT_THREADS / PPL;
    constexpr int NW = NT / 64;
    float4 *sA = sh.sA;
    float4 *sB = sh.sB;
    float4 *sC = sh.sC;
    uint32_t *sG = sh.sG;
    auto &part = sh.part;
    auto &written = sh.written;
    int &smax = sh.smax;

    using B = WaveBlock<PPL>;
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const TileInfo ti = tile_info(tile, vp);
    const int W = vp.width, H = vp.height;
    const int64_t HW = (int64_t)H * W;
    const int bx = ti.tx * GS4D_TILE + (w % B::CB) * B::BW;
    const int by = ti.ty * GS4D_TILE + (w / B::CB) * B::BH;
    const int px = bx + lane % B::BW;
    const int row0 = by + lane / B::BW;
    const float fx = (float)px + 0.5f;
    const float sx0 = (float)bx + 0.5f, sx1 = sx0 + (float)(B::BW - 1);
    const float sy0 = (float)by + 0.5f, sy1 = sy0 + (float)(B::BH - 1);
    const int2 rg = ranges[tile];
    const gs4d_view &V = vp.v[ti.v];

    int my_last[PPL];
    // gB: the upstream colour gradient dotted with the colour behind the
    // current entry (g . B, linear in B, so one scalar replaces B's three
    // channels in dC/dalpha = T (g . c - g . B) and in B's update)
    float T[PPL], g0[PPL], g1[PPL], g2[PPL], gB[PPL], fy[PPL];
    int lane_last = -1;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int py = row0 + B::RPS * k;
        fy[k] = (float)py + 0.5f;
        my_last[k] = -1;
        T[k] = 1.0f;
        g0[k] = g1[k] = g2[k] = 0.0f;
        if (px < W && py < H) {
            const int64_t pix = (int64_t)py * W + px;
            my_last[k] = last[(int64_t)ti.v * HW + pix];
            T[k] = T_final[(int64_t)ti.v * HW + pix];
            const float *d = dL_dimage + (int64_t)ti.v * 3 * HW + pix;
            g0[k] = d[0];
            g1[k] = d[HW];
            g2[k] = d[2 * HW];
        }
        gB[k] = fmaf(g2[k], V.bg[2], fmaf(g1[k], V.bg[1], g0[k] * V.bg[0]));
        lane_last = max(lane_last, my_last[k]);
    }
    if (t == 0) smax = -1;
    __syncthreads();
    if (lane_last >= 0) atomicMax(&smax, lane_last);
    // the wave's own furthest entry
    int wave_last = lane_last;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) wave_last = max(wave_last, __shfl_xor(wave_last, off, 64));
    __syncthreads();
    const int max_last = smax;
    if (max_last < rg.x) return;
    const float4 *recv = rec + (int64_t)ti.v * n * 3;
    float *gview = grad2d + (int64_t)ti.v * n * 9;
    const int drow = lane >> 4;
    const bool row_leader = (lane & 15) == 15;
    // first term whose wave total this row's leader holds (see wave_scatter9)
    const int trow = ((drow & 1) << 1) | (drow >> 1);
    // this wave's partial slots as an LDS pointer, so per-entry offsets are
    // 32-bit adds
    __attribute__((address_space(3))) float *wpart =
        (__attribute__((address_space(3))) float *)&part[w][0];

    for (int end = max_last + 1; end > rg.x; end -= BATCH) {
        const int start = max(rg.x, end - BATCH);
        const int cnt = end - start;
        __syncthreads();
        for (int i = t; i < cnt; i += NT) {
            const uint32_t g = vals[start + i];
            const float4 r0 = recv[3 * (int64_t)g + 0];
            const float4 r1 = recv[3 * (int64_t)g + 1];
            const float4 r2 = recv[3 * (int64_t)g + 2];
            sA[i] = r0;
            sB[i] = make_float4(r1.x, r1.y, r2.x, r2.y);
            sC[i] = make_float4(r2.z, alpha_floor(r1.y), r1.w, r2.w);   // as in stage_batch
            sG[i] = g;
        }
        __syncthreads();
        // entries beyond this wave's last blended one are skipped too
        const int wcnt = min(cnt, wave_last - start + 1);
        uint64_t m[NK], wr[NK];
        strip_masks<BATCH>(sA, sB, sC, wcnt, sx0, sx1, sy0, sy1, lane, m);
#pragma unroll
        for (int k = 0; k < NK; ++k) wr[k] = 0;
        // Branch-free per entry (selects only), entries taken back to front
        // two at a time so their LDS reads overlap.
        auto grad_one = [&](int j, float4 a, float4 b, float2 c) {
            const int idx = start + j;
            const float cbl = c.x;
            // the nine per-entry terms, summed over this lane's pixels (the
            // first pixel assigns, so no add of zero is issued):
            //   0, 1: dpow dx, dpow dy          (mean: Q times their sums)
            //   2, 3, 4: dpow dx^2, dx dy, dy^2 (conic, factors at the atomic)
            //   5: dpow                         (opacity: sum / o_t)
            //   6, 7, 8: alpha T g              (colour)
            // with dpow = dL/dalpha * alpha~, the gradient with respect to the
            // exponent in natural units
            float d[9];
            bool any = false;
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                const float dx = fx - a.x, dy = fy[k] - a.y;
                float qx, qy;
                const float arg = gauss_arg(a, b.x, dx, dy, qx, qy);
                const float ex = __builtin_amdgcn_exp2f(arg);
                const float at = b.y * ex;
                const bool ok = (idx <= my_last[k]) && !(arg < c.y);   // alpha >= 1/255
                any = any || ok;
                // alpha of a blended entry, 0 otherwise (then it changes nothing below)
                const float alpha = ok ? fminf(ALPHA_MAX, at) : 0.0f;
                // transmittance in front of this entry
                const float Tk = T[k] * __builtin_amdgcn_rcpf(1.0f - alpha);
                T[k] = ok ? Tk : T[k];
                const float wgt = alpha * Tk;
                // dC/dalpha . g = T (g . c - g . B); then B <- B + alpha (c - B)
                const float gc = fmaf(g2[k], cbl, fmaf(g1[k], b.w, g0[k] * b.z));
                const float diff = gc - gB[k];
                gB[k] = fmaf(alpha, diff, gB[k]);
                // no gradient through the 0.99 clamp
                const float dalpha = (ok && at <= ALPHA_MAX) ? Tk * diff : 0.0f;
                const float dpow = dalpha * at;
                const float pdx = dpow * dx, pdy = dpow * dy;
                if (k == 0) {
                    d[0] = pdx;
                    d[1] = pdy;
                    d[2] = pdx * dx;
                    d[3] = pdx * dy;
                    d[4] = pdy * dy;
                    d[5] = dpow;
                    d[6] = wgt * g0[k];
                    d[7] = wgt * g1[k];
                    d[8] = wgt * g2[k];
                } else {
                    d[0] += pdx;
                    d[1] += pdy;
                    d[2] = fmaf(pdx, dx, d[2]);
                    d[3] = fmaf(pdx, dy, d[3]);
                    d[4] = fmaf(pdy, dy, d[4]);
                    d[5] += dpow;
                    d[6] = fmaf(wgt, g0[k], d[6]);
                    d[7] = fmaf(wgt, g1[k], d[7]);
                    d[8] = fmaf(wgt, g2[k], d[8]);
                }
            }
            if (__ballot(any) == 0) return;   // no lane of this wave blends the entry
            wr[j >> 6] |= 1ull << (j & 63);
            float x[3];
            wave_scatter9(d, x);
            if (row_leader) {
                const int o = j * 9 + trow;
                wpart[o] = x[0];
                wpart[o + 4] = x[1];
                if (drow == 3) wpart[o + 5] = x[2];   // lane 63: term 8 (t(3) = 3)
            }
        };
#pragma unroll
        for (int kk = NK - 1; kk >= 0; --kk) {
            uint64_t mask = m[kk];
            while (mask) {
                const int bit0 = 63 - __builtin_clzll(mask);
                mask &= ~(1ull << bit0);
                const bool two = mask != 0;
                const int bit1 = two ? 63 - __builtin_clzll(mask) : bit0;
                if (two) mask &= ~(1ull << bit1);
                const int j0 = kk * 64 + bit0, j1 = kk * 64 + bit1;
                const float4 a0 = sA[j0], b0 = sB[j0];
                const float2 c0 = make_float2(sC[j0].x, sC[j0].y);
                const float4 a1 = sA[j1], b1 = sB[j1];
                const float2 c1 = make_float2(sC[j1].x, sC[j1].y);
                grad_one(j0, a0, b0, c0);
                if (two) grad_one(j1, a1, b1, c1);
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < NK; ++k) written[w][k] = wr[k];
        }
        __syncthreads();
        // one thread per (entry, term): sum the written slots, one atomic.
        // Terms 0 and 1 hold the moments S = sum dpow d; the mean's gradient
        // is Q S (d exponent / d mean = Q d), so their threads sum both.
        for (int i = t; i < cnt * 9; i += NT) {
            const int e = i / 9, q = i - 9 * e;
            const uint64_t bit = 1ull << (e & 63);
            const int i0 = (q < 2) ? i - q : i;
            float sum = 0.0f, sum1 = 0.0f;
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                if (written[ww][e >> 6] & bit) {
                    sum += part[ww][i0];
                    if (q < 2) sum1 += part[ww][i0 + 1];
                }
            }
            float g;
            if (q < 2) {
                // (a, b) = sA.zw, c = sB.x
                const float4 a = sA[e];
                g = (q == 0) ? fmaf(a.z, sum, a.w * sum1) : fmaf(a.w, sum, sB[e].x * sum1);
            } else if (q == 5) {
                g = sum / sB[e].y;   // d alpha~ / d o_t = alpha~ / o_t
            } else {
                // the conic terms' factors: d exponent / d(a, b, c) = (-dx^2/2, -dx dy, -dy^2/2)
                const float fac = (q == 2 || q == 4) ? -0.5f : (q == 3 ? -1.0f : 1.0f);
                g = sum * fac;
            }
            if (g != 0.0f) atomicAdd(gview + (int64_t)sG[e] * 9 + q, g);
        }
    }
}

template <int BATCH, int PPL>
__global__ void __launch_bounds__(RT_THREADS / PPL)
render_bwd_kernel(const float4 *__restrict__ rec, int64_t n, const uint32_t *__restrict__ vals,
                  const int2 *__restrict__ ranges, ViewPack vp,
                  const float *__restrict__ dL_dimage, const float *__restrict__ T_final,
                  const int32_t *__restrict__ last, float *__restrict__ grad2d, int persistent,
                  const int32_t *__restrict__ order, int32_t *__restrict__ queue) {
    __shared__ BwdShared<BATCH, PPL> sh;
    if (!persistent) {
        render_tile_bwd<BATCH, PPL>(blockIdx.x, rec, n, vals, ranges, vp, dL_dimage, T_final, last,
                                    grad2d, sh);
        return;
    }
    const int64_t n_tiles = (int64_t)vp.tiles_per_view * vp.n_views;
    if (persistent == 2) {
        for (int64_t r = 0, base = 0; base < n_tiles; ++r, base += gridDim.x) {
            const int64_t k = static_position(r, base);
            if (k < n_tiles) {
                const int64_t tile = order ? order[k] : k;
                render_tile_bwd<BATCH, PPL>(tile, rec, n, vals, ranges, vp, dL_dimage, T_final,
                                            last, grad2d, sh);
            }
            __syncthreads();
        }
        return;
    }
    // persistent: take tiles from the (largest-first) work list until it is
    // empty, the first one by workgroup index (as in the forward)
    __shared__ int next;
    for (int k = blockIdx.x; k < n_tiles;) {
        const int64_t tile = order ? order[k] : k;
        render_tile_bwd<BATCH, PPL>(tile, rec, n, vals, ranges, vp, dL_dimage, T_final, last,
                                    grad2d, sh);
        __syncthreads();
        if (threadIdx.x == 0) next = (int)gridDim.x + atomicAdd(queue, 1);
        __syncthreads();
        k = next;
    }
}

// Workgroups of a persistent launch: the caller's count, else 4 per CU.
unsigned persistent_grid(int32_t n_workgroups) {
    if (n_workgroups > 0) return (unsigned)n_workgroups;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    return (unsigned)(4 * cus);
}

int check_render_args(const float *rec, int64_t n, const uint32_t *vals, const int32_t *ranges) {
    GS4D_REQUIRE(n >= 0 && n <= (int64_t)0x7fffffff, "render: n out of range");
    GS4D_REQUIRE(ranges != nullptr, "render: null ranges");
    GS4D_REQUIRE(n == 0 || rec != nullptr, "render: null rec");
    (void)vals;
    return GS4D_OK;
}

}  // namespace
}  // namespace gs4d

using namespace gs4d;

extern "C" int gs4d_render_fwd(const float *rec, int64_t n, const uint32_t *vals,
                               const int32_t *ranges, const gs4d_view *views, int32_t n_views,
                               const gs4d_render_opts *opts, float *image, float *T_final,
                               int32_t *last, void *stream) {
    ViewPack vp;
    GS4D_TRY(make_view_pack(views, n_views, &vp));
    GS4D_TRY(check_render_args(rec, n, vals, ranges));
    GS4D_REQUIRE(image, "gs4d_render_fwd: null image");
    GS4D_REQUIRE((T_final == nullptr) == (last == nullptr),
                 "gs4d_render_fwd: T_final and last must both be given or both be null");
    gs4d_render_opts o{};
    if (opts) o = *opts;
    if (o.batch == 0) o.batch = 256;
    GS4D_REQUIRE(o.batch == 64 || o.batch == 128 || o.batch == 256,
                 "gs4d_render_fwd: batch must be 64, 128 or 256");
    GS4D_REQUIRE(!(o.loss_per_view || o.dL_dimage) || o.target,
                 "gs4d_render_fwd: loss outputs need a target");
    GS4D_REQUIRE(o.persistent >= 0 && o.persistent <= 2, "gs4d_render_fwd: persistent must be 0, 1 or 2");
    GS4D_REQUIRE(o.persistent != 1 || o.queue, "gs4d_render_fwd: persistent mode 1 needs a queue counter");
    const int64_t n_tiles = (int64_t)vp.tiles_per_view * n_views;
    hipStream_t st = as_stream(stream);
    unsigned grid = (unsigned)n_tiles;
    if (o.persistent) {
        grid = persistent_grid(o.n_workgroups);
    }
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const int2 *rg = reinterpret_cast<const int2 *>(ranges);
    const bool count = o.counters != nullptr;
    switch (o.batch) {
        case 64:
            if (count)
                render_fwd_kernel<64, true><<<grid, RT_THREADS, 0, st>>>(r4, n, vals, rg, vp, o, image, T_final, last);
            else
                render_fwd_kernel<64, false><<<grid, RT_THREADS, 0, st>>>(r4, n, vals, rg, vp, o, image, T_final, last);
            break;
        case 128:
            if (count)
                render_fwd_kernel<128, true><<<grid, RT_THREADS, 0, st>>>(r4, n, vals, rg, vp, o, image, T_final, last);
            else
                render_fwd_kernel<128, false><<<grid, RT_THREADS, 0, st>>>(r4, n, vals, rg, vp, o, image, T_final, last);
            break;
        default:
            if (count)
                render_fwd_kernel<256, true><<<grid, RT_THREADS, 0, st>>>(r4, n, vals, rg, vp, o, image, T_final, last);
            else
                render_fwd_kernel<256, false><<<grid, RT_THREADS, 0, st>>>(r4, n, vals, rg, vp, o, image, T_final, last);
            break;
    }
    GS4D_LAUNCH_CHECK("gs4d_render_fwd");
    return GS4D_OK;
}

extern "C" size_t gs4d_render_bwd_workspace_size(int64_t n, int32_t n_views) {
    return (size_t)(n > 0 ? n : 1) * (size_t)(n_views > 0 ? n_views : 1) * 9 * sizeof(float) + 256;
}

namespace gs4d {
namespace {
int g_bwd_ppl = 1;   // pixels per lane of the backward (1, 2 or 4)
}
}  // namespace gs4d

extern "C" int gs4d_set_bwd_variant(int32_t pixels_per_lane) {
    GS4D_REQUIRE(pixels_per_lane == 1 || pixels_per_lane == 2 || pixels_per_lane == 4,
                 "gs4d_set_bwd_variant: pixels_per_lane must be 1, 2 or 4");
    g_bwd_ppl = pixels_per_lane;
    return GS4D_OK;
}

extern "C" int gs4d_render_bwd_2d(const float *rec, int64_t n, const uint32_t *vals,
                                  const int32_t *ranges, const gs4d_view *views, int32_t n_views,
                                  const gs4d_render_opts *opts, const float *dL_dimage,
                                  const float *T_final, const int32_t *last, float *grad2d,
                                  void *stream) {
    ViewPack vp;
    GS4D_TRY(make_view_pack(views, n_views, &vp));
    GS4D_TRY(check_render_args(rec, n, vals, ranges));
    GS4D_REQUIRE(dL_dimage && T_final && last, "gs4d_render_bwd_2d: null input");
    GS4D_REQUIRE(n == 0 || grad2d, "gs4d_render_bwd_2d: null grad2d");
    gs4d_render_opts o{};
    if (opts) o = *opts;
    GS4D_REQUIRE(o.persistent >= 0 && o.persistent <= 2, "gs4d_render_bwd_2d: persistent must be 0, 1 or 2");
    GS4D_REQUIRE(o.persistent != 1 || o.queue, "gs4d_render_bwd_2d: persistent mode 1 needs a queue counter");
    GS4D_REQUIRE((o.flags & ~GS4D_RENDER_GRAD2D_ZEROED) == 0, "gs4d_render_bwd_2d: unknown flags");
    if (n == 0) return GS4D_OK;
    hipStream_t st = as_stream(stream);
    if (!(o.flags & GS4D_RENDER_GRAD2D_ZEROED))
        GS4D_TRY(launch_fill<float>(grad2d, 0.0f, n * n_views * 9, st));
    const int64_t n_tiles = (int64_t)vp.tiles_per_view * n_views;
    unsigned grid = (unsigned)n_tiles;
    if (o.persistent) {
        grid = persistent_grid(o.n_workgroups);
    }
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const int2 *rg = reinterpret_cast<const int2 *>(ranges);
    const int ps = o.persistent;
    switch (g_bwd_ppl) {
        case 1:
            render_bwd_kernel<BWD_BATCH, 1><<<grid, RT_THREADS, 0, st>>>(
                r4, n, vals, rg, vp, dL_dimage, T_final, last, grad2d, ps, o.order, o.queue);
            break;
        case 4:
            render_bwd_kernel<BWD_BATCH, 4><<<grid, RT_THREADS / 4, 0, st>>>(
                r4, n, vals, rg, vp, dL_dimage, T_final, last, grad2d, ps, o.order, o.queue);
            break;
        default:
            render_bwd_kernel<BWD_BATCH, 2><<<grid, RT_THREADS / 2, 0, st>>>(
                r4, n, vals, rg, vp, dL_dimage, T_final, last, grad2d, ps, o.order, o.queue);
            break;
    }
    GS4D_LAUNCH_CHECK("gs4d_render_bwd_2d");
    return GS4D_OK;
}

extern "C" int gs4d_render_bwd(const float *params, int64_t n, const float *rec,
                               const int32_t *touched, const uint32_t *vals,
                               const int32_t *ranges, const gs4d_view *views, int32_t n_views,
                               const gs4d_render_opts *opts, const float *dL_dimage,
                               const float *T_final, const int32_t *last, float *dparams,
                               float *grad2d, void *ws, size_t ws_bytes, void *stream) {
    GS4D_REQUIRE(n >= 0, "gs4d_render_bwd: n < 0");
    GS4D_REQUIRE(n == 0 || (params && touched && dparams), "gs4d_render_bwd: null pointer");
    float *g2d = grad2d;
    if (!g2d) {
        GS4D_REQUIRE(ws && ws_bytes >= gs4d_render_bwd_workspace_size(n, n_views),
                     "gs4d_render_bwd: workspace too small");
        g2d = static_cast<float *>(ws);
    }
    GS4D_TRY(gs4d_render_bwd_2d(rec, n, vals, ranges, views, n_views, opts, dL_dimage, T_final, last,
                                g2d, stream));
    return gs4d_preprocess_bwd(params, n, views, n_views, touched, g2d, dparams, stream);
}

// ---------------------------------------------------------------- tile order
namespace gs4d {
namespace {
// Work order of the persistent launches in one workgroup: tiles by
// decreasing size class (empty tiles, class 0, last), by index within a
// class -- a stable counting sort.  A pair count n >= 1 has class
// 1 + 8 floor(log2 n) + its three bits below the leading one, i.e. eight
// classes per octave (lengths within 12.5% share a class).  Each of the 16
// waves owns a contiguous run of tiles: it counts its classes, one block
// scan turns the counts into each (wave, class) start (classes largest
// first, waves in index order inside a class), and each wave then places its
// tiles 64 at a time, ranking a lane among the lanes of the same class with
// ballots.  Also zeroes the work counters.
constexpr int ORDER_CLASSES = 257;
constexpr int ORDER_THREADS = 1024;
constexpr int ORDER_WAVES = ORDER_THREADS / 64;

__device__ __forceinline__ int tile_class(const int2 r) {
    const uint32_t len = (uint32_t)(r.y - r.x);
    if (len == 0) return 0;
    const int e = 31 - __builtin_clz(len);
    const uint32_t m = e >= 3 ? (len >> (e - 3)) & 7u : (len << (3 - e)) & 7u;
    return 1 + 8 * e + (int)m;
}

__global__ void __launch_bounds__(ORDER_THREADS)
tile_order_kernel(const int2 *__restrict__ ranges, int64_t n_tiles, int32_t *__restrict__ order,
                  int32_t *__restrict__ queues, int n_queues) {
    __shared__ uint32_t cnt[ORDER_WAVES][ORDER_CLASSES];
    __shared__ uint32_t wsum[ORDER_WAVES];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    for (int i = t; i < ORDER_WAVES * ORDER_CLASSES; i += ORDER_THREADS) (&cnt[0][0])[i] = 0;
    if (t < n_queues) queues[t] = 0;
    __syncthreads();
    // this wave's tiles [lo, hi), a whole number of 64-tile steps
    const int64_t chunk = ((n_tiles + ORDER_WAVES - 1) / ORDER_WAVES + 63) / 64 * 64;
    const int64_t lo = (int64_t)w * chunk;
    const int64_t hi = lo + chunk < n_tiles ? lo + chunk : n_tiles;
    for (int64_t i = lo + l; i < hi; i += 64) atomicAdd(&cnt[w][tile_class(ranges[i])], 1u);
    __syncthreads();
    // thread p < ORDER_CLASSES handles class ORDER_CLASSES - 1 - p (placement
    // order): prefix over the waves, then a block scan of the class totals
    const int c = ORDER_CLASSES - 1 - t;
    uint32_t tot = 0;
    if (t < ORDER_CLASSES) {
        for (int k = 0; k < ORDER_WAVES; ++k) {
            const uint32_t x = cnt[k][c];
            cnt[k][c] = tot;
            tot += x;
        }
    }
    uint32_t incl = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (l >= off) incl += y;
    }
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    if (t < ORDER_CLASSES) {
        uint32_t start = incl - tot;
        for (int k = 0; k < w; ++k) start += wsum[k];
        for (int k = 0; k < ORDER_WAVES; ++k) cnt[k][c] += start;
    }
    __syncthreads();
    const uint64_t lt_mask = (l == 0) ? 0ull : (~0ull >> (64 - l));
    for (int64_t c0 = lo; c0 < hi; c0 += 64) {
        const int64_t i = c0 + l;
        const bool valid = i < hi;
        const int cls = valid ? tile_class(ranges[i]) : 0;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 9; ++bit) {
            const uint64_t m = __ballot((cls >> bit) & 1);
            peers &= ((cls >> bit) & 1) ? m : ~m;
        }
        const uint32_t before = __popcll(peers & lt_mask);
        if (valid) order[cnt[w][cls] + before] = (int32_t)i;
        // all lanes have read the start before the class leader advances it
        __builtin_amdgcn_wave_barrier();
        if (valid && before == 0) cnt[w][cls] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
}
}  // namespace
}  // namespace gs4d

extern "C" size_t gs4d_tile_order_workspace_size(int64_t n_tiles) {
    (void)n_tiles;
    return 256;   // the order is computed in LDS; kept for a stable interface
}

extern "C" int gs4d_tile_order(const int32_t *ranges, int64_t n_tiles, int32_t *order,
                               int32_t *queues, int32_t n_queues, void *ws, size_t ws_bytes,
                               void *stream) {
    (void)ws;
    (void)ws_bytes;
    GS4D_REQUIRE(n_tiles > 0 && n_tiles < ((int64_t)1 << 31), "gs4d_tile_order: n_tiles out of range");
    GS4D_REQUIRE(ranges && order, "gs4d_tile_order: null pointer");
    GS4D_REQUIRE(n_queues >= 0 && n_queues <= 64 && (n_queues == 0 || queues),
                 "gs4d_tile_order: bad queues (at most 64)");
    hipStream_t st = as_stream(stream);
    tile_order_kernel<<<1, ORDER_THREADS, 0, st>>>(reinterpret_cast<const int2 *>(ranges), n_tiles, order,
                                          queues, n_queues);
    GS4D_LAUNCH_CHECK("gs4d_tile_order");
    return GS4D_OK;
}
