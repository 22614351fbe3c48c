// Internal helpers shared by the gs4d HIP translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "gs4d.h"

namespace gs4d {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);

#define GS4D_REQUIRE(cond, ...)                 \
    do {                                        \
        if (!(cond)) {                          \
            ::gs4d::set_error(__VA_ARGS__);     \
            return GS4D_ERR_INVALID_ARG;        \
        }                                       \
    } while (0)

#define GS4D_LAUNCH_CHECK(what)                                                        \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess) {                                                        \
            ::gs4d::set_error("%s: launch failed: %s", what, hipGetErrorString(e_));   \
            return GS4D_ERR_HIP;                                                       \
        }                                                                              \
    } while (0)

#define GS4D_TRY(expr)              \
    do {                            \
        int s_ = (expr);            \
        if (s_ != GS4D_OK) return s_; \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- views
// All views of one call travel by value in the kernel arguments.
struct ViewPack {
    gs4d_view v[GS4D_MAX_VIEWS];
    int32_t n_views;
    int32_t width, height;
    int32_t tiles_x, tiles_y;
    int32_t tiles_per_view;
};

int make_view_pack(const gs4d_view *views, int32_t n_views, ViewPack *pack);

// ---------------------------------------------------------------- workspace
// Bump allocator over a caller-provided workspace (256-byte aligned slices).
struct Carve {
    char *base;
    size_t size;
    size_t used = 0;
    Carve(void *b, size_t s) : base(static_cast<char *>(b)), size(s) {}
    template <class T>
    T *take(size_t count) {
        used = (used + 255) & ~size_t(255);
        T *p = reinterpret_cast<T *>(base ? base + used : nullptr);
        used += count * sizeof(T);
        return p;
    }
    bool ok() const { return used <= size; }
};

// ---------------------------------------------------------------- device utils
__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <class T>
__global__ void fill_kernel(T *dst, T value, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) dst[i] = value;
}

template <class T>
inline int launch_fill(T *dst, T value, int64_t count, hipStream_t st) {
    if (count <= 0) return GS4D_OK;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    fill_kernel<T><<<(unsigned)blocks, 256, 0, st>>>(dst, value, count);
    GS4D_LAUNCH_CHECK("fill");
    return GS4D_OK;
}

// Wave64 sum; every lane receives the total.
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Project-defined FP32 exp and ln.  Every per-Gaussian value that decides
// an integer (cull, footprint, tile rectangle, sort-key depth, the alpha
// >= 1/255 floor of compositing) uses these two, with a fixed operation
// order and no contraction, so that the result is reproducible bit for bit.
// exp(x): Cody-Waite reduction x = k ln2 + r (ln2 split so k * ln2_hi is
// exact), degree-7 Taylor polynomial of e^r in Horner form, scale by 2^k.
__device__ __forceinline__ float fixed_exp(float x) {
#pragma clang fp contract(off)
    if (x != x) return x;
    if (x < -87.0f) return 0.0f;
    if (x > 88.0f) return __builtin_huge_valf();
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

// ln(x): x = m 2^e with m in [1/sqrt2, sqrt2); ln m = 2 atanh(u),
// u = (m - 1) / (m + 1), series through u^9.
__device__ __forceinline__ float fixed_log(float x) {
#pragma clang fp contract(off)
    if (x != x) return x;
    if (x < 0.0f) return __builtin_nanf("");
    if (x == 0.0f) return -__builtin_huge_valf();
    if (x == __builtin_huge_valf()) return x;
    int e;
    float m = frexpf(x, &e);
    if (m < 0.70710678118654752f) {
        m = m * 2.0f;
        e = e - 1;
    }
    const float u = (m - 1.0f) / (m + 1.0f);
    const float u2 = u * u;
    float s = 1.0f / 9.0f;
    s = fmaf(s, u2, 1.0f / 7.0f);
    s = fmaf(s, u2, 1.0f / 5.0f);
    s = fmaf(s, u2, 1.0f / 3.0f);
    s = fmaf(s, u2, 1.0f);
    return fmaf((float)e, 0.693147180559945309f, (2.0f * u) * s);
}

// Exclusive prefix sums (radix sort, scans) ---------------------------------
struct ScanWs;   // defined in binsort.hip

// Device-wide exclusive scan of int32 values (count <= 2^31 - 1).  out may
// alias nothing.  total (device int64) receives the sum.  ws from
// scan_workspace_size(count).
size_t scan_workspace_size(int64_t count);
int exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t count, int64_t *total, void *ws,
                       hipStream_t st);

// Stable LSD radix sort of (key, value) pairs on bits [bit_lo, bit_hi).
// Count is read from *count_dev if not NULL, else count_host.  Capacity
// bounds the launch.  Buffers ping-pong between (k0, v0) and (k1, v1); the
// result lands in (k0, v0) if the number of 8-bit passes is even, else in
// (k1, v1): *result_in_alt reports which.
size_t radix_workspace_size(int64_t capacity);
int radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, const int64_t *count_dev,
                   int64_t count_host, int64_t capacity, int bit_lo, int bit_hi, void *ws,
                   hipStream_t st, int *result_in_alt);

}  // namespace gs4d
