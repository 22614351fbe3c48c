// Per-tile alpha compositing, forward and backward (the Gaussian-splatting
// renderer of Sec. 3.1; the backward of Table B-1 "Backward").
//
// One workgroup = one 16x16 tile = 256 threads = 4 wave64, one pixel per
// thread.  The tile's sorted Gaussians are staged through LDS in batches of
// up to 256 records; every thread then walks the batch with broadcast LDS
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

int launch_preprocess_bwd(const float *params, int64_t n, const ViewPack &vp,
                          const int32_t *touched, const float *grad2d, float *dparams,
                          hipStream_t st);

namespace {

constexpr int RT_THREADS = 256;
constexpr int RT_WAVES = 4;
constexpr float ALPHA_MIN = 1.0f / 255.0f;
constexpr float ALPHA_MAX = 0.99f;
constexpr float T_EPS = 1e-4f;

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

// The exact same instruction sequence decides skip / blend in the forward
// and the backward.
__device__ __forceinline__ float gauss_power(float4 a, float cc, float dx, float dy) {
    const float t1 = a.z * dx;   // conic.a dx
    const float t2 = cc * dy;    // conic.c dy
    const float q = fmaf(t1, dx, t2 * dy);
    return fmaf(-0.5f, q, -(a.w * dx) * dy);
}

template <int BATCH>
__device__ __forceinline__ void render_tile_fwd(int64_t tile, const float4 *__restrict__ rec,
                                                int64_t n, const uint32_t *__restrict__ vals,
                                                const int2 *__restrict__ ranges,
                                                const ViewPack &vp, const gs4d_render_opts &o,
                                                float *__restrict__ image,
                                                float *__restrict__ T_final,
                                                int32_t *__restrict__ last_out, float4 *sA,
                                                float4 *sB, float *sC) {
    const int t = threadIdx.x;
    const TileInfo ti = tile_info(tile, vp);
    const int px = ti.tx * GS4D_TILE + (t & 15);
    const int py = ti.ty * GS4D_TILE + (t >> 4);
    const int W = vp.width, H = vp.height;
    const bool inside = px < W && py < H;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const int2 rg = ranges[tile];
    const float4 *recv = rec + (int64_t)ti.v * n * 3;

    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    int32_t last = -1;
    uint32_t n_eval = 0, n_blend = 0;
    bool done = !inside;

    for (int start = rg.x; start < rg.y; start += BATCH) {
        const int cnt = min(BATCH, rg.y - start);
        __syncthreads();
        if (t < cnt) {
            const uint32_t g = vals[start + t];
            const float4 r0 = recv[3 * (int64_t)g + 0];
            const float4 r1 = recv[3 * (int64_t)g + 1];
            const float4 r2 = recv[3 * (int64_t)g + 2];
            sA[t] = r0;                                       // mx my ca cb
            sB[t] = make_float4(r1.x, r1.y, r2.x, r2.y);      // cc o_t r g
            sC[t] = r2.z;                                     // b
        }
        const int active = __syncthreads_count(!done);
        if (active == 0) break;
        if (!done) {
            for (int j = 0; j < cnt; ++j) {
                const float4 a = sA[j];
                const float4 b = sB[j];
                const float dx = fx - a.x, dy = fy - a.y;
                const float power = gauss_power(a, b.x, dx, dy);
                ++n_eval;
                if (power > 0.0f) continue;
                const float at = b.y * __expf(power);
                const float alpha = fminf(ALPHA_MAX, at);
                if (alpha < ALPHA_MIN) continue;
                const float Tn = T * (1.0f - alpha);
                if (Tn < T_EPS) {
                    done = true;
                    break;
                }
                const float w = alpha * T;
                C0 = fmaf(b.z, w, C0);
                C1 = fmaf(b.w, w, C1);
                C2 = fmaf(sC[j], w, C2);
                T = Tn;
                last = start + j;
                ++n_blend;
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
        T_final[(int64_t)ti.v * HW + pix] = T;
        last_out[(int64_t)ti.v * HW + pix] = last;
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
        if ((t & 63) == 0 && s != 0.0f)
            atomicAdd(&o.loss_per_view[ti.v], s * (o.l1_weight / (float)(3 * HW)));
    }
    if (o.counters) {
        const uint32_t e = wave_sum_u32(n_eval);
        const uint32_t bl = wave_sum_u32(n_blend);
        if ((t & 63) == 0) {
            atomicAdd((unsigned long long *)&o.counters[0], (unsigned long long)e);
            atomicAdd((unsigned long long *)&o.counters[1], (unsigned long long)bl);
        }
    }
}

template <int BATCH>
__global__ void __launch_bounds__(RT_THREADS)
render_fwd_kernel(const float4 *__restrict__ rec, int64_t n, const uint32_t *__restrict__ vals,
                  const int2 *__restrict__ ranges, ViewPack vp, gs4d_render_opts o,
                  float *__restrict__ image, float *__restrict__ T_final,
                  int32_t *__restrict__ last) {
    __shared__ float4 sA[BATCH];
    __shared__ float4 sB[BATCH];
    __shared__ float sC[BATCH];
    const int64_t n_tiles = (int64_t)vp.tiles_per_view * vp.n_views;
    if (!o.persistent) {
        render_tile_fwd<BATCH>(blockIdx.x, rec, n, vals, ranges, vp, o, image, T_final, last, sA,
                               sB, sC);
        return;
    }
    __shared__ int next;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) next = atomicAdd(o.queue, 1);
        __syncthreads();
        const int k = next;
        if (k >= n_tiles) break;
        const int64_t tile = o.order ? o.order[k] : k;
        render_tile_fwd<BATCH>(tile, rec, n, vals, ranges, vp, o, image, T_final, last, sA, sB,
                               sC);
    }
}

// ---------------------------------------------------------------- backward
template <int BATCH>
__global__ void __launch_bounds__(RT_THREADS)
render_bwd_kernel(const float4 *__restrict__ rec, int64_t n, const uint32_t *__restrict__ vals,
                  const int2 *__restrict__ ranges, ViewPack vp,
                  const float *__restrict__ dL_dimage, const float *__restrict__ T_final,
                  const int32_t *__restrict__ last, float *__restrict__ grad2d) {
    __shared__ float4 sA[BATCH];
    __shared__ float4 sB[BATCH];
    __shared__ float sC[BATCH];
    __shared__ uint32_t sG[BATCH];
    __shared__ float part[RT_WAVES][BATCH][9];
    __shared__ int smax;

    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int64_t tile = blockIdx.x;
    const TileInfo ti = tile_info(tile, vp);
    const int px = ti.tx * GS4D_TILE + (t & 15);
    const int py = ti.ty * GS4D_TILE + (t >> 4);
    const int W = vp.width, H = vp.height;
    const bool inside = px < W && py < H;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const int2 rg = ranges[tile];
    const int64_t HW = (int64_t)H * W;
    const int64_t pix = (int64_t)py * W + px;
    const gs4d_view &V = vp.v[ti.v];

    int my_last = -1;
    float T = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
    if (inside) {
        my_last = last[(int64_t)ti.v * HW + pix];
        T = T_final[(int64_t)ti.v * HW + pix];
        const float *d = dL_dimage + (int64_t)ti.v * 3 * HW + pix;
        g0 = d[0];
        g1 = d[HW];
        g2 = d[2 * HW];
    }
    float B0 = V.bg[0], B1 = V.bg[1], B2 = V.bg[2];
    if (t == 0) smax = -1;
    __syncthreads();
    if (my_last >= 0) atomicMax(&smax, my_last);
    __syncthreads();
    const int max_last = smax;
    if (max_last < rg.x) return;
    const float4 *recv = rec + (int64_t)ti.v * n * 3;
    float *gview = grad2d + (int64_t)ti.v * n * 9;

    for (int end = max_last + 1; end > rg.x; end -= BATCH) {
        const int start = max(rg.x, end - BATCH);
        const int cnt = end - start;
        __syncthreads();
        if (t < cnt) {
            const uint32_t g = vals[start + t];
            const float4 r0 = recv[3 * (int64_t)g + 0];
            const float4 r1 = recv[3 * (int64_t)g + 1];
            const float4 r2 = recv[3 * (int64_t)g + 2];
            sA[t] = r0;
            sB[t] = make_float4(r1.x, r1.y, r2.x, r2.y);
            sC[t] = r2.z;
            sG[t] = g;
        }
        for (int i = t; i < RT_WAVES * BATCH * 9; i += RT_THREADS) (&part[0][0][0])[i] = 0.0f;
        __syncthreads();
        for (int j = cnt - 1; j >= 0; --j) {
            const int idx = start + j;
            float d[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) d[k] = 0.0f;
            bool contrib = false;
            if (idx <= my_last) {
                const float4 a = sA[j];
                const float4 b = sB[j];
                const float cbl = sC[j];
                const float dx = fx - a.x, dy = fy - a.y;
                const float power = gauss_power(a, b.x, dx, dy);
                if (power <= 0.0f) {
                    const float ex = __expf(power);
                    const float at = b.y * ex;
                    const float alpha = fminf(ALPHA_MAX, at);
                    if (alpha >= ALPHA_MIN) {
                        contrib = true;
                        T = T / (1.0f - alpha);         // transmittance in front of entry
                        const float wgt = alpha * T;
                        d[6] = wgt * g0;
                        d[7] = wgt * g1;
                        d[8] = wgt * g2;
                        const float dalpha = T * (g0 * (b.z - B0) + g1 * (b.w - B1) + g2 * (cbl - B2));
                        B0 = alpha * b.z + (1.0f - alpha) * B0;
                        B1 = alpha * b.w + (1.0f - alpha) * B1;
                        B2 = alpha * cbl + (1.0f - alpha) * B2;
                        if (at <= ALPHA_MAX) {
                            const float dpow = dalpha * at;
                            d[5] = dalpha * ex;
                            d[2] = -0.5f * dpow * dx * dx;
                            d[3] = -dpow * dx * dy;
                            d[4] = -0.5f * dpow * dy * dy;
                            d[0] = dpow * (a.z * dx + a.w * dy);
                            d[1] = dpow * (b.x * dy + a.w * dx);
                        }
                    }
                }
            }
            if (__ballot(contrib)) {
#pragma unroll
                for (int k = 0; k < 9; ++k) d[k] = wave_sum(d[k]);
                if (l == 0) {
#pragma unroll
                    for (int k = 0; k < 9; ++k) part[w][j][k] = d[k];
                }
            }
        }
        __syncthreads();
        if (t < cnt) {
            float s[9];
            bool any = false;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                s[k] = part[0][t][k] + part[1][t][k] + part[2][t][k] + part[3][t][k];
                any |= s[k] != 0.0f;
            }
            if (any) {
                float *dst = gview + (int64_t)sG[t] * 9;
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    if (s[k] != 0.0f) atomicAdd(dst + k, s[k]);
            }
        }
    }
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
    GS4D_REQUIRE(image && T_final && last, "gs4d_render_fwd: null output");
    gs4d_render_opts o{};
    if (opts) o = *opts;
    if (o.batch == 0) o.batch = 256;
    GS4D_REQUIRE(o.batch == 64 || o.batch == 128 || o.batch == 256,
                 "gs4d_render_fwd: batch must be 64, 128 or 256");
    GS4D_REQUIRE(!(o.loss_per_view || o.dL_dimage) || o.target,
                 "gs4d_render_fwd: loss outputs need a target");
    GS4D_REQUIRE(!o.persistent || o.queue, "gs4d_render_fwd: persistent mode needs a queue counter");
    const int64_t n_tiles = (int64_t)vp.tiles_per_view * n_views;
    hipStream_t st = as_stream(stream);
    unsigned grid = (unsigned)n_tiles;
    if (o.persistent) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = (unsigned)(o.n_workgroups > 0 ? o.n_workgroups : 4 * cus);
    }
    const float4 *r4 = reinterpret_cast<const float4 *>(rec);
    const int2 *rg = reinterpret_cast<const int2 *>(ranges);
    switch (o.batch) {
        case 64:
            render_fwd_kernel<64><<<grid, RT_THREADS, 0, st>>>(r4, n, vals, rg, vp, o, image, T_final, last);
            break;
        case 128:
            render_fwd_kernel<128><<<grid, RT_THREADS, 0, st>>>(r4, n, vals, rg, vp, o, image, T_final, last);
            break;
        default:
            render_fwd_kernel<256><<<grid, RT_THREADS, 0, st>>>(r4, n, vals, rg, vp, o, image, T_final, last);
            break;
    }
    GS4D_LAUNCH_CHECK("gs4d_render_fwd");
    return GS4D_OK;
}

extern "C" size_t gs4d_render_bwd_workspace_size(int64_t n, int32_t n_views) {
    return (size_t)(n > 0 ? n : 1) * (size_t)(n_views > 0 ? n_views : 1) * 9 * sizeof(float) + 256;
}

extern "C" int gs4d_render_bwd(const float *params, int64_t n, const float *rec,
                               const int32_t *touched, const uint32_t *vals,
                               const int32_t *ranges, const gs4d_view *views, int32_t n_views,
                               const float *dL_dimage, const float *T_final, const int32_t *last,
                               float *dparams, float *grad2d, void *ws, size_t ws_bytes,
                               void *stream) {
    ViewPack vp;
    GS4D_TRY(make_view_pack(views, n_views, &vp));
    GS4D_TRY(check_render_args(rec, n, vals, ranges));
    GS4D_REQUIRE(dL_dimage && T_final && last, "gs4d_render_bwd: null input");
    GS4D_REQUIRE(n == 0 || (params && touched && dparams), "gs4d_render_bwd: null pointer");
    float *g2d = grad2d;
    if (!g2d) {
        GS4D_REQUIRE(ws && ws_bytes >= gs4d_render_bwd_workspace_size(n, n_views),
                     "gs4d_render_bwd: workspace too small");
        g2d = static_cast<float *>(ws);
    }
    if (n == 0) return GS4D_OK;
    hipStream_t st = as_stream(stream);
    GS4D_TRY(launch_fill<float>(g2d, 0.0f, n * n_views * 9, st));
    const int64_t n_tiles = (int64_t)vp.tiles_per_view * n_views;
    render_bwd_kernel<256><<<(unsigned)n_tiles, RT_THREADS, 0, st>>>(
        reinterpret_cast<const float4 *>(rec), n, vals, reinterpret_cast<const int2 *>(ranges), vp,
        dL_dimage, T_final, last, g2d);
    GS4D_LAUNCH_CHECK("gs4d_render_bwd");
    return launch_preprocess_bwd(params, n, vp, touched, g2d, dparams, st);
}
