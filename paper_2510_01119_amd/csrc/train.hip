// Optimisation-loop kernels: Adam, L1, SSIM, squared error.
//
// The method trains with a single photometric loss using the loss weights
// and optimiser of 3D Gaussian splatting, with the position learning rate
// lowered to 1e-5 and the schedule stretched to the iteration budget
// (Sec. 4.1).  Readings: Adam with bias correction; per-row exponential
// learning-rate decay lr0^(1-u) lr1^u; SSIM with an 11x11 Gaussian window
// (sigma 1.5), C1 = 0.01^2, C2 = 0.03^2 and zero padding.
#include "common.hpp"

#include <cmath>

namespace gs4d {
namespace {

// Sum over a 256-thread block; the result is valid in thread 0.
__device__ __forceinline__ float block_sum(float x) {
    __shared__ float ws[4];
    x = wave_sum(x);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = x;
    __syncthreads();
    return ws[0] + ws[1] + ws[2] + ws[3];
}

// ---------------------------------------------------------------- Adam
__global__ void __launch_bounds__(256)
adam_kernel(float *__restrict__ P, const float *__restrict__ Gr, float *__restrict__ M,
            float *__restrict__ Vv, int64_t n, gs4d_adam_cfg cfg, const int32_t *__restrict__ step) {
    __shared__ float lr[GS4D_N_FIELDS];
    __shared__ float bc1, bc2;
    const int s = *step + 1;
    if (threadIdx.x < (unsigned)cfg.rows) {
        const int r = threadIdx.x;
        float u = cfg.budget > 0 ? (float)s / (float)cfg.budget : 1.0f;
        u = fminf(fmaxf(u, 0.0f), 1.0f);
        const float a = cfg.lr0[r], b = cfg.lr1[r];
        lr[r] = (a > 0.0f && b > 0.0f) ? expf(logf(a) * (1.0f - u) + logf(b) * u) : a;
    }
    if (threadIdx.x == 0) {
        bc1 = 1.0f - powf(cfg.beta1, (float)s);
        bc2 = 1.0f - powf(cfg.beta2, (float)s);
    }
    __syncthreads();
    const int64_t total = (int64_t)cfg.rows * n;
    const float b1 = cfg.beta1, b2 = cfg.beta2, eps = cfg.eps;
    const float ib1 = 1.0f / bc1, ib2 = 1.0f / bc2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / n);
        const float rate = lr[r];
        if (rate == 0.0f) continue;
        const float g = Gr[i];
        const float m = b1 * M[i] + (1.0f - b1) * g;
        const float v = b2 * Vv[i] + (1.0f - b2) * g * g;
        M[i] = m;
        Vv[i] = v;
        P[i] -= rate * (m * ib1) / (sqrtf(v * ib2) + eps);
    }
}

__global__ void tick_kernel(int32_t *step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

// ---------------------------------------------------------------- L1 / SSE
__global__ void __launch_bounds__(256)
l1_kernel(const float *__restrict__ x, const float *__restrict__ y, int64_t count, float weight,
          float *__restrict__ loss, float *__restrict__ dx) {
    const float scale = weight / (float)count;
    float s = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float d = x[i] - y[i];
        s += fabsf(d);
        if (dx) dx[i] += d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
    }
    s = block_sum(s);
    if (threadIdx.x == 0 && s != 0.0f) atomicAdd(loss, s * scale);
}

__global__ void __launch_bounds__(256)
sse_kernel(const float *__restrict__ x, const float *__restrict__ y, int64_t count,
           double *__restrict__ out) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)x[i] - (double)y[i];
        s += d * d;
    }
    s = wave_sum_d(s);
    __shared__ double ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double tot = ws[0] + ws[1] + ws[2] + ws[3];
        if (tot != 0.0) atomicAdd(out, tot);
    }
}

// ---------------------------------------------------------------- SSIM
constexpr int SS_R = 5;               // window radius (11 taps)
constexpr int SS_K = 2 * SS_R + 1;
constexpr int SS_T = 32;              // output tile edge
constexpr int SS_E = SS_T + 2 * SS_R; // staged edge (42)
constexpr int SS_EP = 44;             // staged row stride (float4-aligned rows)
constexpr int SS_O = 4;               // adjacent outputs per thread in each pass
constexpr int SS_W = SS_O + 2 * SS_R; // inputs one thread reads per pass (14)
constexpr float SS_C1 = 0.01f * 0.01f;
constexpr float SS_C2 = 0.03f * 0.03f;
static_assert(SS_T * SS_T / SS_O == 256, "one vertical strip per thread");

struct Win {
    float g[SS_K];
};

// Both passes are register-blocked: a thread filters SS_O adjacent outputs
// from the SS_W inputs they share.  Horizontal pass: item (row r, column
// group j) covers columns 4j..4j+3 of row r, read as four float4 from the
// staged rows; vertical pass: thread (column c, row group) covers rows
// 4g..4g+3 of column c.  Taps are summed in the same order as a plain
// 11-tap loop.
__device__ __forceinline__ void load_row14(const float *row, int c0, float v[16]) {
    const float4 *p = reinterpret_cast<const float4 *>(row + c0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const float4 q = p[m];
        v[4 * m] = q.x;
        v[4 * m + 1] = q.y;
        v[4 * m + 2] = q.z;
        v[4 * m + 3] = q.w;
    }
}

// The tile (column, row, plane) of this block.  Workgroups go to the 8 XCDs
// in turn; block b takes tile (b mod 8) (nb8 / 8) + b div 8 of the first
// nb8 = 8 floor(nb / 8) tiles in row-major order (the rest stay in place), so
// that each XCD's blocks cover a run of neighbouring tiles and find the
// halo rows they share in its own L2.
__device__ __forceinline__ uint3 ssim_tile() {
    const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
    const unsigned b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const unsigned nb8 = nb & ~7u;
    const unsigned t = b < nb8 ? (b & 7u) * (nb8 >> 3) + (b >> 3) : b;
    const unsigned q = t / gridDim.x;
    return make_uint3(t - q * gridDim.x, q % gridDim.y, q / gridDim.y);
}

// Forward: per pixel SSIM and its partial derivatives with respect to the
// windowed statistics mu_x, E[x^2], E[xy] (written to three maps).  Each
// block stores its SSIM sum (and, when fused, its L1 sum) as a partial;
// partial_sum_kernel adds them up, so no block ever waits on another.  With
// l1_grad set, the kernel also writes dL/dimg = l1_scale sign(x - y)
// (overwriting), the L1 term of the photometric loss.
__global__ void __launch_bounds__(256)
ssim_fwd_kernel(const float *__restrict__ X, const float *__restrict__ Y, int h, int w, Win win,
                float *__restrict__ P1, float *__restrict__ P2, float *__restrict__ P3,
                float *__restrict__ part_ssim, float *__restrict__ part_l1, float l1_scale,
                float *__restrict__ l1_grad) {
    __shared__ __align__(16) float sx[SS_E][SS_EP];
    __shared__ __align__(16) float sy[SS_E][SS_EP];
    // row-filtered statistics, three planes: (mu_x, mu_y, E[x^2]) first, then
    // (E[y^2], E[xy]) -- 30.9 KB of LDS in all
    __shared__ __align__(16) float hs[3][SS_E][SS_T];
    const int t = threadIdx.x;
    const uint3 tb = ssim_tile();
    const int ox = tb.x * SS_T - SS_R, oy = tb.y * SS_T - SS_R;
    const int64_t plane = (int64_t)tb.z * h * w;
    {
        // every load issued before the first is used: outside the image (or
        // in a row's padding) a load reads the plane's first pixel and its
        // value is replaced by 0
        constexpr int SS_LD = (SS_E * SS_EP + 255) / 256;
        float xl[SS_LD], yl[SS_LD];
        bool inl[SS_LD];
#pragma unroll
        for (int k = 0; k < SS_LD; ++k) {
            const int i = t + 256 * k;
            const int r = i / SS_EP, c = i - r * SS_EP;
            const int gy = oy + r, gx = ox + c;
            inl[k] = i < SS_E * SS_EP && c < SS_E && gx >= 0 && gx < w && gy >= 0 && gy < h;
            const int64_t idx = inl[k] ? plane + (int64_t)gy * w + gx : plane;
            xl[k] = X[idx];
            yl[k] = Y[idx];
        }
#pragma unroll
        for (int k = 0; k < SS_LD; ++k) {
            const int i = t + 256 * k;
            if (i < SS_E * SS_EP) {
                const int r = i / SS_EP, c = i - r * SS_EP;
                sx[r][c] = inl[k] ? xl[k] : 0.0f;
                sy[r][c] = inl[k] ? yl[k] : 0.0f;
            }
        }
    }
    __syncthreads();
    const int c = t % SS_T, r0 = (t / SS_T) * SS_O;
    float m[5][SS_O] = {};
#pragma unroll
    for (int grp = 0; grp < 2; ++grp) {
        if (grp > 0) __syncthreads();   // the first group's column pass has read hs
        for (int i = t; i < SS_E * (SS_T / SS_O); i += 256) {
            const int r = i / (SS_T / SS_O), c0 = (i - r * (SS_T / SS_O)) * SS_O;
            float xv[16], yv[16];
            load_row14(sx[r], c0, xv);
            load_row14(sy[r], c0, yv);
            float s0[SS_O] = {}, s1[SS_O] = {}, s2[SS_O] = {};
#pragma unroll
            for (int k = 0; k < SS_K; ++k) {
                const float g = win.g[k];
#pragma unroll
                for (int o = 0; o < SS_O; ++o) {
                    const float x = xv[o + k], y = yv[o + k];
                    if (grp == 0) {
                        s0[o] += g * x;
                        s1[o] += g * y;
                        s2[o] += g * x * x;
                    } else {
                        s0[o] += g * y * y;
                        s1[o] += g * x * y;
                    }
                }
            }
            *reinterpret_cast<float4 *>(&hs[0][r][c0]) = make_float4(s0[0], s0[1], s0[2], s0[3]);
            *reinterpret_cast<float4 *>(&hs[1][r][c0]) = make_float4(s1[0], s1[1], s1[2], s1[3]);
            if (grp == 0)
                *reinterpret_cast<float4 *>(&hs[2][r][c0]) =
                    make_float4(s2[0], s2[1], s2[2], s2[3]);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (grp == 1 && q == 2) continue;
            float v[SS_W];
#pragma unroll
            for (int k = 0; k < SS_W; ++k) v[k] = hs[q][r0 + k][c];
            float acc[SS_O] = {};
#pragma unroll
            for (int k = 0; k < SS_K; ++k) {
                const float g = win.g[k];
#pragma unroll
                for (int o = 0; o < SS_O; ++o) acc[o] += g * v[o + k];
            }
#pragma unroll
            for (int o = 0; o < SS_O; ++o) m[grp == 0 ? q : 3 + q][o] = acc[o];
        }
    }
    float sv = 0.0f, lv = 0.0f;
    const int gx = tb.x * SS_T + c;
#pragma unroll
    for (int o = 0; o < SS_O; ++o) {
        const int r = r0 + o, gy = tb.y * SS_T + r;
        if (gx < w && gy < h) {
            const float mx = m[0][o], my = m[1][o];
            const float sxx = m[2][o] - mx * mx, syy = m[3][o] - my * my, sxy = m[4][o] - mx * my;
            const float A1 = 2.f * mx * my + SS_C1, A2 = 2.f * sxy + SS_C2;
            const float B1 = mx * mx + my * my + SS_C1, B2 = sxx + syy + SS_C2;
            // one hardware reciprocal (about 1 ulp) per factor instead of seven
            // correctly rounded divisions
            const float iA1 = __builtin_amdgcn_rcpf(A1), iA2 = __builtin_amdgcn_rcpf(A2);
            const float iB1 = __builtin_amdgcn_rcpf(B1), iB2 = __builtin_amdgcn_rcpf(B2);
            const float S = (A1 * A2) * (iB1 * iB2);
            sv += S;
            const int64_t po = plane + (int64_t)gy * w + gx;
            if (P1) {
                P1[po] = S * (2.f * my * iA1 - 2.f * mx * iB1 - 2.f * my * iA2 + 2.f * mx * iB2);
                P2[po] = -S * iB2;
                P3[po] = 2.f * S * iA2;
            }
            if (part_l1) {
                const float d = sx[r + SS_R][c + SS_R] - sy[r + SS_R][c + SS_R];
                lv += fabsf(d);
                if (l1_grad) l1_grad[po] = d > 0.0f ? l1_scale : (d < 0.0f ? -l1_scale : 0.0f);
            }
        }
    }
    const unsigned bid = tb.x + gridDim.x * (tb.y + gridDim.y * tb.z);
    sv = block_sum(sv);
    if (part_l1) lv = block_sum(lv);
    if (t == 0) {
        part_ssim[bid] = sv;
        if (part_l1) part_l1[bid] = lv;
    }
}

// One block: out[0] += a * sum(pa) + b * sum(pb) + c (pb may be NULL); with
// overwrite set the output is replaced instead of accumulated.  Partial
// sums are added in a fixed order, so the result is deterministic.
__device__ __forceinline__ void sum_partials(const float *__restrict__ pa,
                                             const float *__restrict__ pb, int count, float a,
                                             float b, float c, float *__restrict__ out,
                                             int overwrite) {
    float sa = 0.0f, sb = 0.0f;
    for (int i = threadIdx.x; i < count; i += 256) {
        sa += pa[i];
        if (pb) sb += pb[i];
    }
    sa = block_sum(sa);
    sb = block_sum(sb);
    if (threadIdx.x == 0) {
        const float v = a * sa + b * sb + c;
        out[0] = overwrite ? v : out[0] + v;
    }
}

__global__ void __launch_bounds__(256)
partial_sum_kernel(const float *__restrict__ pa, const float *__restrict__ pb, int count, float a,
                   float b, float c, float *__restrict__ out, int overwrite) {
    sum_partials(pa, pb, count, a, b, c, out, overwrite);
}

// The final loss sum of partial_sum_kernel, done instead by the first block
// of the SSIM backward before its own tile (the partials are complete once
// the forward has finished; no block waits on another).
struct LossSum {
    const float *pa, *pb;
    int count;
    float a, b, c;
    float *out;   // NULL: nothing to sum
};

// Backward: dSSIM/dx(q) = (G*P1)(q) + 2 x(q) (G*P2)(q) + y(q) (G*P3)(q),
// the window being symmetric (its adjoint is itself).
__global__ void __launch_bounds__(256)
ssim_bwd_kernel(const float *__restrict__ X, const float *__restrict__ Y, int h, int w, Win win,
                float scale, const float *__restrict__ P1, const float *__restrict__ P2,
                const float *__restrict__ P3, float *__restrict__ dX, float l1_scale,
                int overwrite, LossSum ls) {
    if (ls.out && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0)
        sum_partials(ls.pa, ls.pb, ls.count, ls.a, ls.b, ls.c, ls.out, 1);
    // one map at a time (staged, filtered along rows, then along columns into
    // registers): 12.8 KB of LDS, so that more blocks share a CU; the next
    // map's values are loaded into registers while the current one is
    // filtered
    constexpr int SS_PER = (SS_E * SS_EP + 255) / 256;
    __shared__ __align__(16) float sp[SS_E][SS_EP];
    __shared__ __align__(16) float hs[SS_E][SS_T];
    const int t = threadIdx.x;
    const uint3 tb = ssim_tile();
    const int ox = tb.x * SS_T - SS_R, oy = tb.y * SS_T - SS_R;
    const int64_t plane = (int64_t)tb.z * h * w;
    const int c = t % SS_T, r0 = (t / SS_T) * SS_O;
    auto fetch = [&](const float *Pj, float (&pre)[SS_PER]) {
#pragma unroll
        for (int u = 0; u < SS_PER; ++u) {
            const int i = t + u * 256;
            const int r = i / SS_EP, cc = i - r * SS_EP;
            const int gy = oy + r, gx = ox + cc;
            const bool in = i < SS_E * SS_EP && cc < SS_E && gx >= 0 && gx < w && gy >= 0 && gy < h;
            pre[u] = in ? Pj[plane + (int64_t)gy * w + gx] : 0.0f;
        }
    };
    float pre[SS_PER];
    fetch(P1, pre);
    float q[3][SS_O] = {};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        // sp's last readers (the previous map's row pass) are behind a barrier
#pragma unroll
        for (int u = 0; u < SS_PER; ++u) {
            const int i = t + u * 256;
            if (i < SS_E * SS_EP) (&sp[0][0])[i] = pre[u];
        }
        __syncthreads();
        if (j < 2) fetch(j == 0 ? P2 : P3, pre);
        for (int i = t; i < SS_E * (SS_T / SS_O); i += 256) {
            const int r = i / (SS_T / SS_O), c0 = (i - r * (SS_T / SS_O)) * SS_O;
            float v[16];
            load_row14(sp[r], c0, v);
            float a[SS_O] = {};
#pragma unroll
            for (int k = 0; k < SS_K; ++k) {
                const float g = win.g[k];
#pragma unroll
                for (int o = 0; o < SS_O; ++o) a[o] += g * v[o + k];
            }
            *reinterpret_cast<float4 *>(&hs[r][c0]) = make_float4(a[0], a[1], a[2], a[3]);
        }
        __syncthreads();
        float v[SS_W];
#pragma unroll
        for (int k = 0; k < SS_W; ++k) v[k] = hs[r0 + k][c];
#pragma unroll
        for (int k = 0; k < SS_K; ++k) {
            const float g = win.g[k];
#pragma unroll
            for (int o = 0; o < SS_O; ++o) q[j][o] += g * v[o + k];
        }
        // the next map's row pass writes hs only after the barrier that
        // follows its staging, so this column pass needs none of its own
    }
    const int gx = tb.x * SS_T + c;
#pragma unroll
    for (int o = 0; o < SS_O; ++o) {
        const int gy = tb.y * SS_T + r0 + o;
        if (gx < w && gy < h) {
            const int64_t po = plane + (int64_t)gy * w + gx;
            const float x = X[po], y = Y[po];
            // overwrite: dX = l1_scale sign(x - y) + the SSIM term (the
            // photometric loss), else the SSIM term is added to dX
            const float base =
                overwrite ? (x > y ? l1_scale : (x < y ? -l1_scale : 0.0f)) : dX[po];
            dX[po] = base + scale * (q[0][o] + 2.f * x * q[1][o] + y * q[2][o]);
        }
    }
}

Win make_window() {
    Win wv;
    double g[2 * SS_R + 1], s = 0.0;
    for (int k = 0; k < 2 * SS_R + 1; ++k) {
        const double x = k - SS_R;
        g[k] = std::exp(-(x * x) / (2.0 * 1.5 * 1.5));
        s += g[k];
    }
    for (int k = 0; k < 2 * SS_R + 1; ++k) wv.g[k] = (float)(g[k] / s);
    return wv;
}

inline unsigned stride_grid(int64_t count) {
    int64_t b = (count + 255) / 256;
    if (b > 2048) b = 2048;
    return (unsigned)(b > 0 ? b : 1);
}

}  // namespace
}  // namespace gs4d

using namespace gs4d;

extern "C" int gs4d_adam_step(float *params, const float *grads, float *m, float *v, int64_t n,
                              const gs4d_adam_cfg *cfg, int32_t *step, void *stream) {
    GS4D_REQUIRE(cfg && step, "gs4d_adam_step: null cfg / step");
    GS4D_REQUIRE(cfg->rows >= 1 && cfg->rows <= GS4D_N_FIELDS, "gs4d_adam_step: rows out of range");
    GS4D_REQUIRE(n >= 0, "gs4d_adam_step: n < 0");
    GS4D_REQUIRE(n == 0 || (params && grads && m && v), "gs4d_adam_step: null pointer");
    hipStream_t st = as_stream(stream);
    if (n > 0) {
        adam_kernel<<<stride_grid((int64_t)cfg->rows * n), 256, 0, st>>>(params, grads, m, v, n, *cfg,
                                                                          step);
        GS4D_LAUNCH_CHECK("gs4d_adam_step");
    }
    tick_kernel<<<1, 64, 0, st>>>(step);
    GS4D_LAUNCH_CHECK("gs4d_adam_step tick");
    return GS4D_OK;
}

extern "C" int gs4d_loss_l1(const float *img, const float *target, int64_t count, float weight,
                            float *loss, float *dL_dimg, void *stream) {
    GS4D_REQUIRE(count >= 0 && loss, "gs4d_loss_l1: bad arguments");
    if (count == 0) return GS4D_OK;
    GS4D_REQUIRE(img && target, "gs4d_loss_l1: null pointer");
    // four blocks per CU: enough loads in flight, few same-address atomics
    const unsigned blocks = stride_grid(count) < 1024 ? stride_grid(count) : 1024;
    l1_kernel<<<blocks, 256, 0, as_stream(stream)>>>(img, target, count, weight, loss, dL_dimg);
    GS4D_LAUNCH_CHECK("gs4d_loss_l1");
    return GS4D_OK;
}

extern "C" int gs4d_sse(const float *img, const float *target, int64_t count, double *sse,
                        void *stream) {
    GS4D_REQUIRE(count >= 0 && sse, "gs4d_sse: bad arguments");
    if (count == 0) return GS4D_OK;
    GS4D_REQUIRE(img && target, "gs4d_sse: null pointer");
    const unsigned blocks = stride_grid(count) < 256 ? stride_grid(count) : 256;
    sse_kernel<<<blocks, 256, 0, as_stream(stream)>>>(img, target, count, sse);
    GS4D_LAUNCH_CHECK("gs4d_sse");
    return GS4D_OK;
}

extern "C" size_t gs4d_ssim_workspace_size(int32_t b, int32_t c, int32_t h, int32_t w) {
    const size_t blocks = (size_t)((w + 15) / 16) * ((h + 15) / 16) * b * c;
    return (size_t)3 * (size_t)b * c * h * w * sizeof(float) + 2 * blocks * sizeof(float) + 6 * 256;
}

namespace {
struct SsimWs {
    float *P1, *P2, *P3, *part_ssim, *part_l1;
    dim3 grid;
};

SsimWs carve_ssim(void *ws, size_t ws_bytes, int32_t b, int32_t c, int32_t h, int32_t w) {
    SsimWs S;
    const int64_t count = (int64_t)b * c * h * w;
    Carve cv(ws, ws_bytes);
    S.P1 = cv.take<float>((size_t)count);
    S.P2 = cv.take<float>((size_t)count);
    S.P3 = cv.take<float>((size_t)count);
    S.grid = dim3((unsigned)((w + SS_T - 1) / SS_T), (unsigned)((h + SS_T - 1) / SS_T),
                  (unsigned)(b * c));
    const size_t nb = (size_t)S.grid.x * S.grid.y * S.grid.z;
    S.part_ssim = cv.take<float>(nb);
    S.part_l1 = cv.take<float>(nb);
    return S;
}
}  // namespace

extern "C" int gs4d_ssim(const float *img, const float *target, int32_t b, int32_t c, int32_t h,
                         int32_t w, float weight, float *ssim_sum, float *dL_dimg, void *ws,
                         size_t ws_bytes, void *stream) {
    GS4D_REQUIRE(b > 0 && c > 0 && h > 0 && w > 0, "gs4d_ssim: bad shape");
    GS4D_REQUIRE((int64_t)b * c <= 65535, "gs4d_ssim: too many planes");
    GS4D_REQUIRE(img && target, "gs4d_ssim: null image");
    GS4D_REQUIRE(ws && ws_bytes >= gs4d_ssim_workspace_size(b, c, h, w),
                 "gs4d_ssim: workspace too small");
    hipStream_t st = as_stream(stream);
    const int64_t count = (int64_t)b * c * h * w;
    SsimWs S = carve_ssim(ws, ws_bytes, b, c, h, w);
    const Win win = make_window();
    ssim_fwd_kernel<<<S.grid, 256, 0, st>>>(img, target, h, w, win, dL_dimg ? S.P1 : nullptr, S.P2,
                                            S.P3, S.part_ssim, nullptr, 0.0f, nullptr);
    GS4D_LAUNCH_CHECK("gs4d_ssim fwd");
    if (ssim_sum) {
        partial_sum_kernel<<<1, 256, 0, st>>>(S.part_ssim, nullptr, (int)(S.grid.x * S.grid.y * S.grid.z),
                                              weight / (float)count, 0.0f, 0.0f, ssim_sum, 0);
        GS4D_LAUNCH_CHECK("gs4d_ssim sum");
    }
    if (dL_dimg) {
        ssim_bwd_kernel<<<S.grid, 256, 0, st>>>(img, target, h, w, win, weight / (float)count, S.P1,
                                                S.P2, S.P3, dL_dimg, 0.0f, 0, LossSum{});
        GS4D_LAUNCH_CHECK("gs4d_ssim bwd");
    }
    return GS4D_OK;
}

extern "C" size_t gs4d_photometric_loss_workspace_size(int32_t b, int32_t c, int32_t h, int32_t w) {
    return gs4d_ssim_workspace_size(b, c, h, w);
}

extern "C" int gs4d_photometric_loss(const float *img, const float *target, int32_t b, int32_t c,
                                     int32_t h, int32_t w, float w_l1, float w_ssim, float *loss,
                                     float *dL_dimg, void *ws, size_t ws_bytes, void *stream) {
    GS4D_REQUIRE(b > 0 && c > 0 && h > 0 && w > 0, "gs4d_photometric_loss: bad shape");
    GS4D_REQUIRE((int64_t)b * c <= 65535, "gs4d_photometric_loss: too many planes");
    GS4D_REQUIRE(img && target && loss && dL_dimg, "gs4d_photometric_loss: null pointer");
    GS4D_REQUIRE(ws && ws_bytes >= gs4d_photometric_loss_workspace_size(b, c, h, w),
                 "gs4d_photometric_loss: workspace too small");
    hipStream_t st = as_stream(stream);
    const int64_t count = (int64_t)b * c * h * w;
    const float inv = 1.0f / (float)count;
    SsimWs S = carve_ssim(ws, ws_bytes, b, c, h, w);
    const Win win = make_window();
    // with an SSIM term the backward writes the L1 gradient together with its
    // own, else the forward writes it
    ssim_fwd_kernel<<<S.grid, 256, 0, st>>>(img, target, h, w, win, S.P1, S.P2, S.P3, S.part_ssim,
                                            S.part_l1, w_l1 * inv,
                                            w_ssim != 0.0f ? nullptr : dL_dimg);
    GS4D_LAUNCH_CHECK("gs4d_photometric_loss fwd");
    // loss = w_l1 mean|x - y| + w_ssim (1 - mean SSIM), summed by the first
    // block of the backward (or its own launch when there is no backward)
    const LossSum ls{S.part_l1, S.part_ssim, (int)(S.grid.x * S.grid.y * S.grid.z), w_l1 * inv,
                     -w_ssim * inv, w_ssim, loss};
    if (w_ssim != 0.0f) {
        ssim_bwd_kernel<<<S.grid, 256, 0, st>>>(img, target, h, w, win, -w_ssim * inv, S.P1, S.P2,
                                                S.P3, dL_dimg, w_l1 * inv, 1, ls);
        GS4D_LAUNCH_CHECK("gs4d_photometric_loss bwd");
    } else {
        partial_sum_kernel<<<1, 256, 0, st>>>(ls.pa, ls.pb, ls.count, ls.a, ls.b, ls.c, loss, 1);
        GS4D_LAUNCH_CHECK("gs4d_photometric_loss sum");
    }
    return GS4D_OK;
}
