// Static / dynamic split of a motion-probability map by Otsu's threshold
// (Sec. 3.2: the motion probabilities are thresholded with Otsu's method
// into a binary mask that decides each back-projected point's class; Otsu,
// "A threshold selection method from gray-level histograms", 1979).
//
// 256 uniform bins on [0, 1]: a value x (clamped to [0, 1], NaN as 0) falls
// in bin min(255, floor(256 x)) -- 256 x is exact in FP32.  For a split k
// (class 0 = bins below k, class 1 = the rest) with S0 = count and S1 = sum
// of (2i + 1) over the bins below k (bin centres (2i + 1) / 512), N and T the
// totals, the between-class variance is proportional to
//     A^2 / (S0 (N - S0)),   A = T S0 - S1 N   (integers, |A| < 2^53),
// evaluated in FP64 as (A * A) / (S0 * (N - S0)) -- one rounding each, so the
// same value on any IEEE machine (N <= 4,000,000 keeps A exact).  k* is the
// first k in 1..255 with the largest value (a split with an empty class has
// none; with no split at all k* = 256, everything static); the mask is
// bin(x) >= k*, an integer decision.  All device arithmetic here is exact or
// fixed in order (file compiled without FP contraction).
#include "common.hpp"

namespace gs4d {
namespace {

constexpr int OT_BINS = 256;

__device__ __forceinline__ int otsu_bin(float x) {
    x = x > 0.0f ? (x < 1.0f ? x : 1.0f) : 0.0f;   // NaN compares false -> 0
    const int b = (int)(x * 256.0f);
    return b < OT_BINS - 1 ? b : OT_BINS - 1;
}

__global__ void __launch_bounds__(256)
otsu_hist_kernel(const float *__restrict__ prob, int64_t count, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[OT_BINS];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[otsu_bin(prob[i])], 1u);
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// One block of 256 threads: thread k evaluates split k.
__global__ void __launch_bounds__(256)
otsu_select_kernel(const uint32_t *__restrict__ hist, int32_t *__restrict__ kstar,
                   float *__restrict__ threshold) {
    __shared__ int64_t s0[OT_BINS + 1], s1[OT_BINS + 1];
    __shared__ double best_v[OT_BINS / 64];
    __shared__ int best_k[OT_BINS / 64];
    const int k = threadIdx.x, l = k & 63, w = k >> 6;
    // exclusive prefix sums over the bins below each k, and the totals (one
    // thread, 256 integer additions)
    if (k == 0) {
        int64_t a = 0, b = 0;
        for (int i = 0; i < OT_BINS; ++i) {
            s0[i] = a;
            s1[i] = b;
            a += hist[i];
            b += (int64_t)hist[i] * (2 * i + 1);
        }
        s0[OT_BINS] = a;
        s1[OT_BINS] = b;
    }
    __syncthreads();
    const int64_t N = s0[OT_BINS], T = s1[OT_BINS];
    double v = -1.0;
    if (k >= 1) {
        const int64_t S0 = s0[k], S1 = s1[k];
        if (S0 > 0 && S0 < N) {
            const double A = (double)(T * S0 - S1 * N);
            v = (A * A) / ((double)S0 * (double)(N - S0));
        }
    }
    // first maximum: the largest value, the smallest k among equal values
    int bk = k;
    double bv = v;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int ok = __shfl_xor(bk, off, 64);
        if (ov > bv || (ov == bv && ok < bk)) {
            bv = ov;
            bk = ok;
        }
    }
    if (l == 0) {
        best_v[w] = bv;
        best_k[w] = bk;
    }
    __syncthreads();
    if (k == 0) {
        double fv = best_v[0];
        int fk = best_k[0];
        for (int i = 1; i < OT_BINS / 64; ++i)
            if (best_v[i] > fv || (best_v[i] == fv && best_k[i] < fk)) {
                fv = best_v[i];
                fk = best_k[i];
            }
        if (!(fv >= 0.0)) fk = OT_BINS;   // no split with two classes: all static
        *kstar = fk;
        if (threshold) *threshold = (float)fk / 256.0f;
    }
}

__global__ void __launch_bounds__(256)
otsu_mask_kernel(const float *__restrict__ prob, int64_t count, const int32_t *__restrict__ kstar,
                 uint8_t *__restrict__ mask) {
    const int k = *kstar;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        mask[i] = otsu_bin(prob[i]) >= k ? 1 : 0;
}

// mask = bin(x) >= k for a threshold k / 256 written by gs4d_otsu_mask
__global__ void __launch_bounds__(256)
threshold_mask_kernel(const float *__restrict__ prob, int64_t count,
                      const float *__restrict__ threshold, uint8_t *__restrict__ mask) {
    const int k = (int)(*threshold * 256.0f);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        mask[i] = otsu_bin(prob[i]) >= k ? 1 : 0;
}

struct OtsuWs {
    uint32_t *hist;
    int32_t *kstar;
};

OtsuWs carve_otsu(void *ws) {
    Carve c(ws, ~size_t(0));
    OtsuWs W;
    W.hist = c.take<uint32_t>(OT_BINS);
    W.kstar = c.take<int32_t>(1);
    return W;
}

}  // namespace
}  // namespace gs4d

using namespace gs4d;

extern "C" size_t gs4d_otsu_workspace_size(void) {
    Carve c(nullptr, 0);
    c.take<uint32_t>(OT_BINS);
    c.take<int32_t>(1);
    return c.used + 256;
}

extern "C" int gs4d_otsu_mask(const float *prob, int64_t count, float *threshold, uint8_t *mask,
                              void *ws, size_t ws_bytes, void *stream) {
    GS4D_REQUIRE(count >= 0, "gs4d_otsu_mask: count < 0");
    // 511 count^2 < 2^53 keeps the class sums' cross products exact in FP64
    GS4D_REQUIRE(count <= 4000000, "gs4d_otsu_mask: count above 4,000,000");
    GS4D_REQUIRE(count == 0 || prob, "gs4d_otsu_mask: null prob");
    GS4D_REQUIRE(threshold || mask, "gs4d_otsu_mask: no output");
    GS4D_REQUIRE(ws && ws_bytes >= gs4d_otsu_workspace_size(), "gs4d_otsu_mask: workspace too small");
    hipStream_t st = as_stream(stream);
    OtsuWs W = carve_otsu(ws);
    GS4D_TRY(launch_fill<uint32_t>(W.hist, 0u, OT_BINS, st));
    int64_t blocks = (count + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    if (count > 0) {
        otsu_hist_kernel<<<(unsigned)blocks, 256, 0, st>>>(prob, count, W.hist);
        GS4D_LAUNCH_CHECK("gs4d_otsu_mask hist");
    }
    otsu_select_kernel<<<1, OT_BINS, 0, st>>>(W.hist, W.kstar, threshold);
    GS4D_LAUNCH_CHECK("gs4d_otsu_mask select");
    if (mask && count > 0) {
        otsu_mask_kernel<<<(unsigned)blocks, 256, 0, st>>>(prob, count, W.kstar, mask);
        GS4D_LAUNCH_CHECK("gs4d_otsu_mask mask");
    }
    return GS4D_OK;
}

extern "C" int gs4d_threshold_mask(const float *prob, int64_t count, const float *threshold,
                                   uint8_t *mask, void *stream) {
    GS4D_REQUIRE(count >= 0, "gs4d_threshold_mask: count < 0");
    if (count == 0) return GS4D_OK;
    GS4D_REQUIRE(prob && threshold && mask, "gs4d_threshold_mask: null pointer");
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    threshold_mask_kernel<<<(unsigned)blocks, 256, 0, as_stream(stream)>>>(prob, count, threshold,
                                                                           mask);
    GS4D_LAUNCH_CHECK("gs4d_threshold_mask");
    return GS4D_OK;
}
