// Learned initialisation: exact 8 nearest neighbours over a sorted cell
// grid, the point features, the 16-64-64-64-4 SiLU network (BF16
// parameters, FP32 accumulation) forward / backward / Adam, and the map
// between a 4D Gaussian's motion (log s_t, velocity) and its rotor form.
//
// The network is tiny (19k multiply-adds per point): one lane per point,
// the parameters are wave-uniform and reach the ALU through scalar loads,
// activations stay in registers.  The weight gradient is a contraction
// over points, so the backward stages each layer's activations and deltas
// of its 64 points in LDS and turns the lanes around (lane = output row);
// per-chunk partials are summed in a fixed order by a second kernel.
#include <cmath>

#include "common.hpp"

namespace gs4d {
namespace {

// ---------------------------------------------------------------- kNN
constexpr int KNN = 8;
constexpr int KNN_RINGS = 8;
constexpr int CELL_BIAS = 1 << 20;
constexpr uint64_t INVALID_KEY = ~0ull;

__device__ __forceinline__ uint64_t cell_key(int ix, int iy, int iz) {
    return ((uint64_t)(uint32_t)(ix + CELL_BIAS) << 42) | ((uint64_t)(uint32_t)(iy + CELL_BIAS) << 21) |
           (uint64_t)(uint32_t)(iz + CELL_BIAS);
}

__device__ __forceinline__ bool cell_of(float x, float cell, int &c) {
    const float q = floorf(x / cell);
    if (!(q >= (float)(-CELL_BIAS + 1) && q <= (float)(CELL_BIAS - 2))) return false;
    c = (int)q;
    return true;
}

__global__ void knn_keys_kernel(const float *__restrict__ xyz, int64_t n, float cell,
                                uint64_t *__restrict__ keys, uint32_t *__restrict__ idx,
                                int32_t *__restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int ix, iy, iz;
    const bool ok = cell_of(xyz[i], cell, ix) && cell_of(xyz[n + i], cell, iy) &&
                    cell_of(xyz[2 * n + i], cell, iz);
    keys[i] = ok ? cell_key(ix, iy, iz) : INVALID_KEY;
    idx[i] = (uint32_t)i;
    if (!ok) atomicOr(status, 1);
}

// first position in keys[0, n) with keys[pos] >= k
__device__ __forceinline__ int64_t lower_bound(const uint64_t *__restrict__ keys, int64_t n, uint64_t k) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

struct Best {
    float d[KNN];
    int32_t id[KNN];
    __device__ void reset() {
#pragma unroll
        for (int k = 0; k < KNN; ++k) {
            d[k] = __builtin_inff();
            id[k] = -1;
        }
    }
    // (d, id) ordering; keeps the 8 smallest
    __device__ __forceinline__ void offer(float dd, int32_t ii) {
        if (!(dd < d[KNN - 1] || (dd == d[KNN - 1] && (uint32_t)ii < (uint32_t)id[KNN - 1]))) return;
        d[KNN - 1] = dd;
        id[KNN - 1] = ii;
#pragma unroll
        for (int k = KNN - 1; k > 0; --k) {
            const bool lt = d[k] < d[k - 1] || (d[k] == d[k - 1] && (uint32_t)id[k] < (uint32_t)id[k - 1]);
            if (lt) {
                const float td = d[k];
                d[k] = d[k - 1];
                d[k - 1] = td;
                const int32_t ti = id[k];
                id[k] = id[k - 1];
                id[k - 1] = ti;
            }
        }
    }
};

__device__ __forceinline__ float dist2(float ax, float ay, float az, float bx, float by, float bz) {
    const float dx = bx - ax, dy = by - ay, dz = bz - az;
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// One thread per sorted position: neighbouring threads query nearby cells.
__global__ void knn_query_kernel(const float *__restrict__ xyz, int64_t n, float cell,
                                 const uint64_t *__restrict__ skeys, const uint32_t *__restrict__ sidx,
                                 int32_t *__restrict__ nbr, float *__restrict__ d2out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t q = sidx[s];
    Best best;
    best.reset();
    const uint64_t qkey = skeys[s];
    if (qkey != INVALID_KEY) {
        const float px = xyz[q], py = xyz[n + q], pz = xyz[2 * n + q];
        int cx, cy, cz;
        cell_of(px, cell, cx);
        cell_of(py, cell, cy);
        cell_of(pz, cell, cz);
        bool done = false;
        for (int r = 0; r <= KNN_RINGS && !done; ++r) {
            for (int dx = -r; dx <= r; ++dx) {
                for (int dy = -r; dy <= r; ++dy) {
                    const bool full = (dx == -r || dx == r || dy == -r || dy == r);
                    for (int part = 0; part < (full ? 1 : 2); ++part) {
                        const int z0 = full ? -r : (part == 0 ? -r : r);
                        const int z1 = full ? r : z0;
                        const int gx = cx + dx, gy = cy + dy;
                        const int gz0 = cz + z0, gz1 = cz + z1;
                        if (gx < -CELL_BIAS || gx >= CELL_BIAS || gy < -CELL_BIAS || gy >= CELL_BIAS)
                            continue;
                        const int lz0 = gz0 < -CELL_BIAS ? -CELL_BIAS : gz0;
                        const int lz1 = gz1 >= CELL_BIAS ? CELL_BIAS - 1 : gz1;
                        if (lz0 > lz1) continue;
                        const int64_t b = lower_bound(skeys, n, cell_key(gx, gy, lz0));
                        const int64_t e = lower_bound(skeys, n, cell_key(gx, gy, lz1) + 1);
                        for (int64_t j = b; j < e; ++j) {
                            const uint32_t o = sidx[j];
                            if (o == q) continue;
                            best.offer(dist2(px, py, pz, xyz[o], xyz[n + o], xyz[2 * n + o]), (int32_t)o);
                        }
                    }
                }
            }
            // every unvisited point lies outside the cube of cells [c - r, c + r]
            const float lo_x = (float)(cx - r) * cell, hi_x = (float)(cx + r + 1) * cell;
            const float lo_y = (float)(cy - r) * cell, hi_y = (float)(cy + r + 1) * cell;
            const float lo_z = (float)(cz - r) * cell, hi_z = (float)(cz + r + 1) * cell;
            float bnd = fminf(fminf(px - lo_x, hi_x - px), fminf(fminf(py - lo_y, hi_y - py),
                                                                  fminf(pz - lo_z, hi_z - pz)));
            // margin for the rounding of the cell assignment and of the distances
            const float mag = fmaxf(fmaxf(fabsf(px), fabsf(py)), fabsf(pz)) + (float)(r + 1) * cell;
            bnd -= 4e-6f * mag;
            if (best.id[KNN - 1] >= 0 && bnd > 0.0f && best.d[KNN - 1] < bnd * bnd) done = true;
        }
        if (!done) {
            // far from everything: exact scan of all points
            best.reset();
            for (int64_t j = 0; j < n; ++j) {
                if (skeys[j] == INVALID_KEY) break;
                const uint32_t o = sidx[j];
                if (o == q) continue;
                best.offer(dist2(px, py, pz, xyz[o], xyz[n + o], xyz[2 * n + o]), (int32_t)o);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KNN; ++k) {
        nbr[(int64_t)k * n + q] = best.id[k];
        d2out[(int64_t)k * n + q] = best.d[k];
    }
}

struct Std16 {
    float shift[16];
    float scale[16];
};

__global__ void features_kernel(const float *__restrict__ xyz, const float *__restrict__ attr,
                                const uint8_t *__restrict__ dyn, const int32_t *__restrict__ nbr,
                                int64_t n, Std16 st, float *__restrict__ feat) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float px = xyz[i], py = xyz[n + i], pz = xyz[2 * n + i];
    const float pt = attr[3 * n + i];
    float ox[KNN], oy[KNN], oz[KNN], ot[KNN];
    int cnt = 0;
    float mx = 0.0f, my = 0.0f, mz = 0.0f, mt = 0.0f;
#pragma unroll
    for (int k = 0; k < KNN; ++k) {
        const int32_t j = nbr[(int64_t)k * n + i];
        const bool ok = j >= 0;
        ox[k] = ok ? xyz[j] - px : 0.0f;
        oy[k] = ok ? xyz[n + j] - py : 0.0f;
        oz[k] = ok ? xyz[2 * n + j] - pz : 0.0f;
        ot[k] = ok ? attr[3 * n + j] - pt : 0.0f;
        cnt += ok ? 1 : 0;
        mx += ox[k];
        my += oy[k];
        mz += oz[k];
        mt += ot[k];
    }
    const float inv = cnt > 0 ? 1.0f / (float)cnt : 0.0f;
    mx *= inv;
    my *= inv;
    mz *= inv;
    mt *= inv;
    // (co)variances of the space-time offsets: per spatial axis, each
    // spatial axis with time, and time
    float vx = 0.0f, vy = 0.0f, vz = 0.0f, cx = 0.0f, cy = 0.0f, cz = 0.0f, vt = 0.0f;
#pragma unroll
    for (int k = 0; k < KNN; ++k) {
        const bool ok = nbr[(int64_t)k * n + i] >= 0;
        const float ax = ox[k] - mx, ay = oy[k] - my, az = oz[k] - mz, at = ot[k] - mt;
        vx += ok ? ax * ax : 0.0f;
        vy += ok ? ay * ay : 0.0f;
        vz += ok ? az * az : 0.0f;
        cx += ok ? ax * at : 0.0f;
        cy += ok ? ay * at : 0.0f;
        cz += ok ? az * at : 0.0f;
        vt += ok ? at * at : 0.0f;
    }
    float f[16];
    f[0] = px;
    f[1] = py;
    f[2] = pz;
    f[3] = attr[4 * n + i];
    f[4] = attr[5 * n + i];
    f[5] = mx;
    f[6] = my;
    f[7] = mz;
    f[8] = vx * inv;
    f[9] = vy * inv;
    f[10] = vz * inv;
    f[11] = cx * inv;
    f[12] = cy * inv;
    f[13] = cz * inv;
    f[14] = vt * inv;
    f[15] = (dyn != nullptr && dyn[i] != 0) ? 1.0f : 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) feat[(int64_t)k * n + i] = (f[k] - st.shift[k]) * st.scale[k];
}

// ---------------------------------------------------------------- network
constexpr int NIN = 16, NH = 64, NOUT = 4;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + NH * NIN;      // 1024
constexpr int OFF_W2 = OFF_B1 + NH;            // 1088
constexpr int OFF_B2 = OFF_W2 + NH * NH;       // 5184
constexpr int OFF_W3 = OFF_B2 + NH;            // 5248
constexpr int OFF_B3 = OFF_W3 + NH * NH;       // 9344
constexpr int OFF_W4 = OFF_B3 + NH;            // 9408
constexpr int OFF_B4 = OFF_W4 + NOUT * NH;     // 9664
constexpr int NPARAM = OFF_B4 + NOUT;          // 9668
static_assert(NPARAM == GS4D_MLP_PARAMS, "parameter count");

// BF16 -> FP32 is exact: the pattern is the upper half of the FP32 one.
__device__ __forceinline__ float bf(const uint16_t *__restrict__ w, int k) {
    return __uint_as_float((uint32_t)w[k] << 16);
}

__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// z[j] = b[j] + sum_i W[j][i] in[i], i in order, fused multiply-adds
template <int FI, int FO>
__device__ __forceinline__ void dense(const uint16_t *__restrict__ w, int offW, int offB,
                                      const float (&in)[FI], float (&z)[FO]) {
#pragma unroll
    for (int j = 0; j < FO; ++j) {
        float acc = bf(w, offB + j);
#pragma unroll
        for (int i = 0; i < FI; ++i) acc = fmaf(bf(w, offW + j * FI + i), in[i], acc);
        z[j] = acc;
    }
}

// g_in[i] = sum_j W[j][i] g_out[j]
template <int FI, int FO>
__device__ __forceinline__ void dense_t(const uint16_t *__restrict__ w, int offW, const float (&g)[FO],
                                        float (&out)[FI]) {
#pragma unroll
    for (int i = 0; i < FI; ++i) out[i] = 0.0f;
#pragma unroll
    for (int j = 0; j < FO; ++j)
#pragma unroll
        for (int i = 0; i < FI; ++i) out[i] = fmaf(bf(w, offW + j * FI + i), g[j], out[i]);
}

__global__ void __launch_bounds__(256) mlp_fwd_kernel(const uint16_t *__restrict__ w,
                                                      const float *__restrict__ x, int64_t n,
                                                      float *__restrict__ y) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float h0[NIN], a[NH], b[NH], o[NOUT];
#pragma unroll
    for (int i = 0; i < NIN; ++i) h0[i] = x[(int64_t)i * n + p];
    dense<NIN, NH>(w, OFF_W1, OFF_B1, h0, a);
#pragma unroll
    for (int i = 0; i < NH; ++i) a[i] = silu(a[i]);
    dense<NH, NH>(w, OFF_W2, OFF_B2, a, b);
#pragma unroll
    for (int i = 0; i < NH; ++i) b[i] = silu(b[i]);
    dense<NH, NH>(w, OFF_W3, OFF_B3, b, a);
#pragma unroll
    for (int i = 0; i < NH; ++i) a[i] = silu(a[i]);
    dense<NH, NOUT>(w, OFF_W4, OFF_B4, a, o);
#pragma unroll
    for (int k = 0; k < NOUT; ++k) y[(int64_t)k * n + p] = o[k];
}

// Partial gradients of one 64-point chunk are written in "storage order":
// each weight block transposed ([in][out]) so that lanes write consecutive
// addresses; the reduction maps them back to the flat [out][in] order.
constexpr int CHUNK = 64;    // points per wave (one wave per workgroup)
constexpr int LDS_STRIDE = NH + 4;

struct OutW {
    float w[NOUT];
};

// Stage one layer's weight gradient: dW[j][i] = sum_p D[p][j] H[p][i] over
// the chunk, lane = j (rows), written transposed into part.
template <int FI, int FO>
__device__ __forceinline__ void weight_grad(const float *H, const float *D, float *__restrict__ part,
                                            int offW, int offB, int lane) {
    if (lane < FO) {
        float acc[FI];
#pragma unroll
        for (int i = 0; i < FI; ++i) acc[i] = 0.0f;
        float bsum = 0.0f;
        for (int p = 0; p < CHUNK; ++p) {
            const float d = D[p * LDS_STRIDE + lane];
            bsum += d;
#pragma unroll
            for (int i = 0; i < FI; ++i) acc[i] = fmaf(d, H[p * LDS_STRIDE + i], acc[i]);
        }
#pragma unroll
        for (int i = 0; i < FI; ++i) part[offW + i * FO + lane] = acc[i];
        part[offB + lane] = bsum;
    }
}

__global__ void __launch_bounds__(CHUNK) mlp_bwd_kernel(const uint16_t *__restrict__ w,
                                                        const float *__restrict__ x, int64_t n,
                                                        const float *__restrict__ dy,
                                                        const float *__restrict__ target, OutW ow,
                                                        float inv_n, float *__restrict__ partial,
                                                        float *__restrict__ loss_part,
                                                        float *__restrict__ dx) {
    __shared__ float H[CHUNK * LDS_STRIDE];    // a layer's inputs, [point][i]
    __shared__ float D[CHUNK * LDS_STRIDE];    // its output deltas, [point][j]
    __shared__ float Z1[CHUNK * LDS_STRIDE];   // pre-activations of layers 1, 2 (own row)
    __shared__ float Z2[CHUNK * LDS_STRIDE];
    const int lane = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int64_t p = c * CHUNK + lane;
    const bool valid = p < n;
    float *part = partial + c * NPARAM;
    float *z1 = Z1 + lane * LDS_STRIDE;
    float *z2 = Z2 + lane * LDS_STRIDE;

    float h0[NIN], z[NH], t[NH], g[NH], o[NOUT];
#pragma unroll
    for (int i = 0; i < NIN; ++i) h0[i] = valid ? x[(int64_t)i * n + p] : 0.0f;
    dense<NIN, NH>(w, OFF_W1, OFF_B1, h0, z);
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        z1[i] = z[i];
        t[i] = silu(z[i]);
    }
    dense<NH, NH>(w, OFF_W2, OFF_B2, t, z);
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        z2[i] = z[i];
        t[i] = silu(z[i]);
    }
    dense<NH, NH>(w, OFF_W3, OFF_B3, t, z);      // z = pre-activation of layer 3
#pragma unroll
    for (int i = 0; i < NH; ++i) t[i] = silu(z[i]);
    dense<NH, NOUT>(w, OFF_W4, OFF_B4, t, o);

    float d4[NOUT];
    float lp = 0.0f;
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
        if (target != nullptr) {
            const float e = valid ? o[k] - target[(int64_t)k * n + p] : 0.0f;
            lp = fmaf(ow.w[k] * e, e, lp);
            d4[k] = 2.0f * ow.w[k] * e * inv_n;
        } else {
            d4[k] = valid ? dy[(int64_t)k * n + p] : 0.0f;
        }
    }
    if (target != nullptr && loss_part != nullptr) {
        const float s = wave_sum(lp);
        if (lane == 0) loss_part[c] = s;
    }

    // layer 4: lanes are the 64 inputs of W4 (4 outputs)
#pragma unroll
    for (int i = 0; i < NH; ++i) H[lane * LDS_STRIDE + i] = t[i];
#pragma unroll
    for (int k = 0; k < NOUT; ++k) D[lane * LDS_STRIDE + k] = d4[k];
    __syncthreads();
    {
        float acc[NOUT] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int q = 0; q < CHUNK; ++q) {
            const float h = H[q * LDS_STRIDE + lane];
#pragma unroll
            for (int k = 0; k < NOUT; ++k) acc[k] = fmaf(D[q * LDS_STRIDE + k], h, acc[k]);
        }
#pragma unroll
        for (int k = 0; k < NOUT; ++k) part[OFF_W4 + lane * NOUT + k] = acc[k];
        if (lane < NOUT) {
            float bs = 0.0f;
            for (int q = 0; q < CHUNK; ++q) bs += D[q * LDS_STRIDE + lane];
            part[OFF_B4 + lane] = bs;
        }
    }
    __syncthreads();

    // delta of layer 3
    dense_t<NH, NOUT>(w, OFF_W4, d4, g);
#pragma unroll
    for (int i = 0; i < NH; ++i) g[i] *= dsilu(z[i]);
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        H[lane * LDS_STRIDE + i] = silu(z2[i]);
        D[lane * LDS_STRIDE + i] = g[i];
    }
    __syncthreads();
    weight_grad<NH, NH>(H, D, part, OFF_W3, OFF_B3, lane);
    __syncthreads();

    // delta of layer 2
    dense_t<NH, NH>(w, OFF_W3, g, t);
#pragma unroll
    for (int i = 0; i < NH; ++i) t[i] *= dsilu(z2[i]);
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        H[lane * LDS_STRIDE + i] = silu(z1[i]);
        D[lane * LDS_STRIDE + i] = t[i];
    }
    __syncthreads();
    weight_grad<NH, NH>(H, D, part, OFF_W2, OFF_B2, lane);
    __syncthreads();

    // delta of layer 1
    dense_t<NH, NH>(w, OFF_W2, t, g);
#pragma unroll
    for (int i = 0; i < NH; ++i) g[i] *= dsilu(z1[i]);
#pragma unroll
    for (int i = 0; i < NIN; ++i) H[lane * LDS_STRIDE + i] = h0[i];
#pragma unroll
    for (int i = 0; i < NH; ++i) D[lane * LDS_STRIDE + i] = g[i];
    __syncthreads();
    weight_grad<NIN, NH>(H, D, part, OFF_W1, OFF_B1, lane);

    if (dx != nullptr && valid) {
        float gx[NIN];
        dense_t<NIN, NH>(w, OFF_W1, g, gx);
#pragma unroll
        for (int i = 0; i < NIN; ++i) dx[(int64_t)i * n + p] = gx[i];
    }
}

// grad[k] = sum over chunks, in chunk order; thread s reads storage slot s.
__global__ void mlp_reduce_kernel(const float *__restrict__ partial, int64_t chunks,
                                  float *__restrict__ grad, const float *__restrict__ loss_part,
                                  float inv_n, float *__restrict__ loss) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < NPARAM) {
        float acc = 0.0f;
        for (int64_t c = 0; c < chunks; ++c) acc += partial[c * NPARAM + s];
        // invert storage_pos: scan the block the slot belongs to
        int k;
        if (s < OFF_B1) k = OFF_W1 + (s - OFF_W1) % NH * NIN + (s - OFF_W1) / NH;
        else if (s < OFF_W2) k = s;
        else if (s < OFF_B2) k = OFF_W2 + (s - OFF_W2) % NH * NH + (s - OFF_W2) / NH;
        else if (s < OFF_W3) k = s;
        else if (s < OFF_B3) k = OFF_W3 + (s - OFF_W3) % NH * NH + (s - OFF_W3) / NH;
        else if (s < OFF_W4) k = s;
        else if (s < OFF_B4) k = OFF_W4 + (s - OFF_W4) % NOUT * NH + (s - OFF_W4) / NOUT;
        else k = s;
        grad[k] = acc;
    } else if (s == NPARAM && loss != nullptr && loss_part != nullptr) {
        float acc = 0.0f;
        for (int64_t c = 0; c < chunks; ++c) acc += loss_part[c];
        *loss = acc * inv_n;
    }
}

__global__ void mlp_adam_kernel(float *__restrict__ master, const float *__restrict__ grad,
                                float *__restrict__ m, float *__restrict__ v,
                                uint16_t *__restrict__ wb, int64_t count, float lr, float b1, float b2,
                                float eps, const int32_t *__restrict__ step) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int s = *step + 1;
    const float g = grad[k];
    const float mk = b1 * m[k] + (1.0f - b1) * g;
    const float vk = b2 * v[k] + (1.0f - b2) * g * g;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / (1.0f - powf(b1, (float)s));
    const float vh = vk / (1.0f - powf(b2, (float)s));
    const float p = master[k] - lr * mh / (sqrtf(vh) + eps);
    master[k] = p;
    wb[k] = to_bf16(p);
}

__global__ void step_tick_kernel(int32_t *step) { *step += 1; }

__global__ void to_bf16_kernel(const float *__restrict__ src, uint16_t *__restrict__ dst, int64_t count) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) dst[k] = to_bf16(src[k]);
}

// ---------------------------------------------------------------- motion map
__device__ __forceinline__ void qmul(const float a[4], const float b[4], float out[4]) {
    out[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    out[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    out[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    out[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

__global__ void motion_init_kernel(float *__restrict__ params, const float *__restrict__ pred, int64_t n) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const float ls = params[4 * n + g];
    const float lst = pred[g];
    const float vx = pred[n + g], vy = pred[2 * n + g], vz = pred[3 * n + g];
    // no usable prediction: the heuristic parameters stand
    if (!(isfinite(ls) && isfinite(lst) && isfinite(vx) && isfinite(vy) && isfinite(vz))) return;
    const float s2 = expf(2.0f * ls);
    const float st2 = expf(2.0f * lst);
    const float vn = sqrtf(vx * vx + vy * vy + vz * vz);
    // The rotation nearest to identity with the right eigenvectors: the
    // spatial axis k closest to +-v carries the moving eigenvector (a
    // spatial rotation of at most ~55 degrees takes e_k to d = sign * v/|v|),
    // then a rotation in the (e_k, t) plane.  v = 0 gives identity rotors.
    int k = 0;
    float qs[4] = {1.0f, 0.0f, 0.0f, 0.0f};
    float bsign = 1.0f;
    if (vn > 0.0f) {
        const float u[3] = {vx / vn, vy / vn, vz / vn};
        k = (fabsf(u[1]) > fabsf(u[0])) ? 1 : 0;
        k = (fabsf(u[2]) > fabsf(u[k])) ? 2 : k;
        bsign = u[k] < 0.0f ? -1.0f : 1.0f;
        const float d[3] = {bsign * u[0], bsign * u[1], bsign * u[2]};
        // quaternion taking e_k to d: (1 + e_k . d, e_k x d), normalised
        float c3[3];
        c3[0] = (k == 1 ? d[2] : 0.0f) + (k == 2 ? -d[1] : 0.0f);
        c3[1] = (k == 0 ? -d[2] : 0.0f) + (k == 2 ? d[0] : 0.0f);
        c3[2] = (k == 0 ? d[1] : 0.0f) + (k == 1 ? -d[0] : 0.0f);
        const float w0 = 1.0f + d[k];
        const float nq = sqrtf(w0 * w0 + c3[0] * c3[0] + c3[1] * c3[1] + c3[2] * c3[2]);
        qs[0] = w0 / nq;
        qs[1] = c3[0] / nq;
        qs[2] = c3[1] / nq;
        qs[3] = c3[2] / nq;
    }
    // 2x2 block of Sigma in the plane spanned by (d, 0) and the t axis
    const float a = fmaf(st2 * vn, vn, s2), c = st2, b = bsign * st2 * vn;
    const float half = 0.5f * (a - c);
    const float rad = sqrtf(half * half + b * b);
    const float lam_big = 0.5f * (a + c) + rad;
    const float lam_small = (s2 * st2) / lam_big;      // det = s^2 s_t^2, no cancellation
    float phi = 0.5f * atan2f(2.0f * b, a - c);        // eigenvector of lam_big
    float lam_k = lam_big, lam_t = lam_small;
    const float quarter = 0.785398163397448f;
    if (fabsf(phi) > quarter) {                        // keep the rotation small
        phi -= copysignf(2.0f * quarter, phi);
        lam_k = lam_small;
        lam_t = lam_big;
    }
    // (e_k, t) plane rotation taking e_k to cos(phi) e_k + sin(phi) t: the
    // rotor (cos th/2, sin th/2 e_k) on both sides with th = -phi
    float axt[4] = {cosf(-0.5f * phi), 0.0f, 0.0f, 0.0f};
    axt[1 + k] = sinf(-0.5f * phi);
    const float qsc[4] = {qs[0], -qs[1], -qs[2], -qs[3]};
    float ql[4], qr[4];
    qmul(qs, axt, ql);
    qmul(axt, qsc, qr);
#pragma unroll
    for (int j = 0; j < 3; ++j) params[(4 + j) * n + g] = (j == k) ? 0.5f * logf(lam_k) : ls;
    params[7 * n + g] = 0.5f * logf(lam_t);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        params[(8 + j) * n + g] = ql[j];
        params[(12 + j) * n + g] = qr[j];
    }
}

__global__ void motion_of_kernel(const float *__restrict__ params, int64_t n, float *__restrict__ out) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    float p[20];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 20; ++k) {
        p[k] = params[(int64_t)k * n + g];
        ok = ok && isfinite(p[k]);
    }
    const float nl = sqrtf(p[8] * p[8] + p[9] * p[9] + p[10] * p[10] + p[11] * p[11]);
    const float nr = sqrtf(p[12] * p[12] + p[13] * p[13] + p[14] * p[14] + p[15] * p[15]);
    ok = ok && nl > 0.0f && nr > 0.0f;
    float res[4] = {__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""), __builtin_nanf("")};
    if (ok) {
        float a[4], b[4], s[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] = p[8 + k] / nl;
            b[k] = p[12 + k] / nr;
            s[k] = expf(p[4 + k]);
        }
        // column c of R diag(s): the image of the basis quaternion of axis c
        // (x, y, z, t <-> i, j, k, 1) under q -> a q b, times s[c]; the
        // image's components (1, i, j, k) are its (t, x, y, z) coordinates
        const float basis[4][4] = {{0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}};
        float M[4][4];   // M[row][col], rows/cols in (x, y, z, t) order
#pragma unroll
        for (int col = 0; col < 4; ++col) {
            float t1[4], t2[4];
            qmul(a, basis[col], t1);
            qmul(t1, b, t2);
            M[0][col] = t2[1] * s[col];
            M[1][col] = t2[2] * s[col];
            M[2][col] = t2[3] * s[col];
            M[3][col] = t2[0] * s[col];
        }
        float Stt = 0.0f, Sxt[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            Stt = fmaf(M[3][k], M[3][k], Stt);
#pragma unroll
            for (int r = 0; r < 3; ++r) Sxt[r] = fmaf(M[r][k], M[3][k], Sxt[r]);
        }
        if (Stt > 0.0f) {
            res[0] = 0.5f * logf(Stt);
            res[1] = Sxt[0] / Stt;
            res[2] = Sxt[1] / Stt;
            res[3] = Sxt[2] / Stt;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) out[(int64_t)k * n + g] = res[k];
}

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace
}  // namespace gs4d

using namespace gs4d;

extern "C" {

size_t gs4d_knn8_workspace_size(int64_t n) {
    if (n < 0) return 0;
    Carve cv(nullptr, 0);
    cv.take<uint64_t>((size_t)n);
    cv.take<uint32_t>((size_t)n);
    cv.take<uint64_t>((size_t)n);
    cv.take<uint32_t>((size_t)n);
    cv.take<char>(radix_workspace_size(n));
    return cv.used + 256;
}

int gs4d_knn8(const float *xyz, int64_t n, float cell, int32_t *nbr, float *d2, int32_t *status,
              void *ws, size_t ws_bytes, void *stream) {
    GS4D_REQUIRE(n >= 0 && n < (int64_t(1) << 31), "gs4d_knn8: n out of range");
    GS4D_REQUIRE(cell > 0.0f && std::isfinite(cell), "gs4d_knn8: cell must be positive");
    if (n == 0) return GS4D_OK;
    GS4D_REQUIRE(xyz && nbr && d2 && status && ws, "gs4d_knn8: null pointer");
    GS4D_REQUIRE(ws_bytes >= gs4d_knn8_workspace_size(n), "gs4d_knn8: workspace too small");
    hipStream_t st = as_stream(stream);
    Carve cv(ws, ws_bytes);
    uint64_t *k0 = cv.take<uint64_t>((size_t)n);
    uint32_t *v0 = cv.take<uint32_t>((size_t)n);
    uint64_t *k1 = cv.take<uint64_t>((size_t)n);
    uint32_t *v1 = cv.take<uint32_t>((size_t)n);
    void *rws = cv.take<char>(radix_workspace_size(n));
    GS4D_TRY(launch_fill<int32_t>(status, 0, 1, st));
    knn_keys_kernel<<<blocks_for(n, 256), 256, 0, st>>>(xyz, n, cell, k0, v0, status);
    GS4D_LAUNCH_CHECK("knn_keys");
    int alt = 0;
    GS4D_TRY(radix_sort_u64(k0, v0, k1, v1, nullptr, n, n, 0, 64, rws, st, &alt));
    const uint64_t *sk = alt ? k1 : k0;
    const uint32_t *sv = alt ? v1 : v0;
    knn_query_kernel<<<blocks_for(n, 128), 128, 0, st>>>(xyz, n, cell, sk, sv, nbr, d2);
    GS4D_LAUNCH_CHECK("knn_query");
    return GS4D_OK;
}

int gs4d_init_features(const float *xyz, const float *attr, const uint8_t *dyn,
                       const int32_t *nbr, int64_t n, const float *shift, const float *scale,
                       float *feat, void *stream) {
    GS4D_REQUIRE(n >= 0, "gs4d_init_features: n < 0");
    if (n == 0) return GS4D_OK;
    GS4D_REQUIRE(xyz && attr && nbr && shift && scale && feat, "gs4d_init_features: null pointer");
    Std16 s;
    for (int k = 0; k < 16; ++k) {
        s.shift[k] = shift[k];
        s.scale[k] = scale[k];
    }
    hipStream_t st = as_stream(stream);
    features_kernel<<<blocks_for(n, 256), 256, 0, st>>>(xyz, attr, dyn, nbr, n, s, feat);
    GS4D_LAUNCH_CHECK("init_features");
    return GS4D_OK;
}

int gs4d_mlp_fwd(const uint16_t *w_bf16, const float *x, int64_t n, float *y, void *stream) {
    GS4D_REQUIRE(n >= 0, "gs4d_mlp_fwd: n < 0");
    if (n == 0) return GS4D_OK;
    GS4D_REQUIRE(w_bf16 && x && y, "gs4d_mlp_fwd: null pointer");
    hipStream_t st = as_stream(stream);
    mlp_fwd_kernel<<<blocks_for(n, 256), 256, 0, st>>>(w_bf16, x, n, y);
    GS4D_LAUNCH_CHECK("mlp_fwd");
    return GS4D_OK;
}

size_t gs4d_mlp_bwd_workspace_size(int64_t n) {
    if (n < 0) return 0;
    const int64_t chunks = (n + CHUNK - 1) / CHUNK;
    Carve cv(nullptr, 0);
    cv.take<float>((size_t)(chunks > 0 ? chunks : 1) * NPARAM);
    cv.take<float>((size_t)(chunks > 0 ? chunks : 1));
    return cv.used + 256;
}

int gs4d_mlp_bwd(const uint16_t *w_bf16, const float *x, int64_t n, const float *dy,
                 const float *target, const float *out_weight, float *grad, float *dx,
                 float *loss, void *ws, size_t ws_bytes, void *stream) {
    GS4D_REQUIRE(n >= 0 && n < (int64_t(1) << 31), "gs4d_mlp_bwd: n out of range");
    GS4D_REQUIRE(w_bf16 && grad, "gs4d_mlp_bwd: null pointer");
    hipStream_t st = as_stream(stream);
    if (n == 0) {   // no points: zero gradient and loss (dy / target may be empty)
        GS4D_TRY(launch_fill<float>(grad, 0.0f, NPARAM, st));
        if (loss) GS4D_TRY(launch_fill<float>(loss, 0.0f, 1, st));
        return GS4D_OK;
    }
    GS4D_REQUIRE((dy == nullptr) != (target == nullptr), "gs4d_mlp_bwd: exactly one of dy, target");
    GS4D_REQUIRE(target == nullptr || out_weight != nullptr, "gs4d_mlp_bwd: target needs out_weight");
    GS4D_REQUIRE(x && ws, "gs4d_mlp_bwd: null pointer");
    GS4D_REQUIRE(ws_bytes >= gs4d_mlp_bwd_workspace_size(n), "gs4d_mlp_bwd: workspace too small");
    const int64_t chunks = (n + CHUNK - 1) / CHUNK;
    Carve cv(ws, ws_bytes);
    float *partial = cv.take<float>((size_t)chunks * NPARAM);
    float *loss_part = cv.take<float>((size_t)chunks);
    OutW ow;
    for (int k = 0; k < NOUT; ++k) ow.w[k] = out_weight ? out_weight[k] : 0.0f;
    const float inv_n = 1.0f / (float)n;
    mlp_bwd_kernel<<<(unsigned)chunks, CHUNK, 0, st>>>(w_bf16, x, n, dy, target, ow, inv_n, partial,
                                                      target ? loss_part : nullptr, dx);
    GS4D_LAUNCH_CHECK("mlp_bwd");
    mlp_reduce_kernel<<<blocks_for(NPARAM + 1, 256), 256, 0, st>>>(
        partial, chunks, grad, target ? loss_part : nullptr, inv_n, target ? loss : nullptr);
    GS4D_LAUNCH_CHECK("mlp_reduce");
    return GS4D_OK;
}

int gs4d_mlp_adam(float *master, const float *grad, float *m, float *v, uint16_t *w_bf16,
                  int64_t count, float lr, float beta1, float beta2, float eps, int32_t *step,
                  void *stream) {
    GS4D_REQUIRE(count >= 0, "gs4d_mlp_adam: count < 0");
    if (count == 0) return GS4D_OK;
    GS4D_REQUIRE(master && grad && m && v && w_bf16 && step, "gs4d_mlp_adam: null pointer");
    hipStream_t st = as_stream(stream);
    mlp_adam_kernel<<<blocks_for(count, 256), 256, 0, st>>>(master, grad, m, v, w_bf16, count, lr,
                                                           beta1, beta2, eps, step);
    GS4D_LAUNCH_CHECK("mlp_adam");
    step_tick_kernel<<<1, 1, 0, st>>>(step);
    GS4D_LAUNCH_CHECK("mlp_adam_tick");
    return GS4D_OK;
}

int gs4d_to_bf16(const float *src, uint16_t *dst, int64_t count, void *stream) {
    GS4D_REQUIRE(count >= 0, "gs4d_to_bf16: count < 0");
    if (count == 0) return GS4D_OK;
    GS4D_REQUIRE(src && dst, "gs4d_to_bf16: null pointer");
    hipStream_t st = as_stream(stream);
    to_bf16_kernel<<<blocks_for(count, 256), 256, 0, st>>>(src, dst, count);
    GS4D_LAUNCH_CHECK("to_bf16");
    return GS4D_OK;
}

int gs4d_motion_init(float *params, const float *pred, int64_t n, void *stream) {
    GS4D_REQUIRE(n >= 0, "gs4d_motion_init: n < 0");
    if (n == 0) return GS4D_OK;
    GS4D_REQUIRE(params && pred, "gs4d_motion_init: null pointer");
    hipStream_t st = as_stream(stream);
    motion_init_kernel<<<blocks_for(n, 256), 256, 0, st>>>(params, pred, n);
    GS4D_LAUNCH_CHECK("motion_init");
    return GS4D_OK;
}

int gs4d_motion_of(const float *params, int64_t n, float *out, void *stream) {
    GS4D_REQUIRE(n >= 0, "gs4d_motion_of: n < 0");
    if (n == 0) return GS4D_OK;
    GS4D_REQUIRE(params && out, "gs4d_motion_of: null pointer");
    hipStream_t st = as_stream(stream);
    motion_of_kernel<<<blocks_for(n, 256), 256, 0, st>>>(params, n, out);
    GS4D_LAUNCH_CHECK("motion_of");
    return GS4D_OK;
}

}  // extern "C"
