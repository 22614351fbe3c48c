// Scene preparation: back projection on consistent depth (Sec. 3.2),
// voxel grid pruning (Sec. 3.2 "Grid Pruning"; per-class voxel sizes of the
// Lite/Full presets, Sec. 4.1) and the heuristic initialisation of the
// pruned points (Sec. 4.1).
//
// Pruning:
// The paper aggregates the points of each occupied voxel through a hash map.
// Here the aggregation is sort-based, which also yields a deterministic
// output order:
//   1. one 64-bit key per point: class, an "unpruned" flag for classes whose
//      voxel edge is <= 0, and the three floor(fl32(x / S_v)) voxel indices
//      (20 bits each, biased by 2^19);
//   2. stable LSD radix sort of (key, point index);
//   3. segment heads (key changes) and their exclusive scan -> voxel ids;
//   4. per-voxel FP64 sums: each thread folds a run of 64 sorted points in
//      registers and flushes one atomic per voxel it touched;
//   5. keep voxels with at least min_count points, compact, write centroid,
//      attribute means, count and key.
#include "common.hpp"

namespace gs4d {
namespace {

constexpr int PR_CHUNK = 64;
constexpr int PR_MAX_ATTR = 16;
constexpr int64_t PR_BIAS = 524288;   // 2^19

__global__ void prune_keys_kernel(const float *__restrict__ xyz, const uint8_t *__restrict__ cls,
                                  int64_t m, float vs, float vd, uint64_t *__restrict__ keys,
                                  uint32_t *__restrict__ idx, int32_t *__restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint64_t c = (cls && cls[i]) ? 1ull : 0ull;
    const float v = c ? vd : vs;
    uint64_t key = c << 63;
    if (!(v > 0.0f)) {
        key |= (1ull << 62) | (uint64_t)i;
    } else {
        uint64_t q[3];
        for (int a = 0; a < 3; ++a) {
            const float f = floorf(xyz[(int64_t)a * m + i] / v);
            if (!(f >= -(float)PR_BIAS && f <= (float)(PR_BIAS - 1))) {
                *status = 2;
                q[a] = 0;
            } else {
                q[a] = (uint64_t)((int64_t)f + PR_BIAS);
            }
        }
        key |= (q[0] << 40) | (q[1] << 20) | q[2];
    }
    keys[i] = key;
    idx[i] = (uint32_t)i;
}

__global__ void seg_head_kernel(const uint64_t *__restrict__ keys, int64_t m,
                                int32_t *__restrict__ head) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// seg_excl: exclusive scan of head.  start[s] = first sorted index of segment s,
// start[S] = m.
__global__ void seg_start_kernel(const int32_t *__restrict__ head, const int32_t *__restrict__ excl,
                                 int64_t m, int32_t *__restrict__ start) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    if (head[i]) start[excl[i]] = (int32_t)i;
    if (i == m - 1) start[excl[i] + head[i]] = (int32_t)m;
}

__global__ void seg_sum_kernel(const uint32_t *__restrict__ order, const int32_t *__restrict__ head,
                               const int32_t *__restrict__ excl, const float *__restrict__ xyz,
                               const float *__restrict__ attr, int k_attr, int64_t m,
                               int64_t seg_stride, double *__restrict__ acc) {
    const int64_t c0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * PR_CHUNK;
    if (c0 >= m) return;
    const int64_t c1 = c0 + PR_CHUNK < m ? c0 + PR_CHUNK : m;
    const int nf = 3 + k_attr;
    double s[3 + PR_MAX_ATTR];
    for (int a = 0; a < nf; ++a) s[a] = 0.0;
    int64_t seg = excl[c0] + head[c0] - 1;
    for (int64_t i = c0; i < c1; ++i) {
        const int64_t sg = excl[i] + head[i] - 1;
        if (sg != seg) {
            for (int a = 0; a < nf; ++a) {
                atomicAdd(&acc[a * seg_stride + seg], s[a]);
                s[a] = 0.0;
            }
            seg = sg;
        }
        const int64_t p = order[i];
        for (int a = 0; a < 3; ++a) s[a] += (double)xyz[a * m + p];
        for (int a = 0; a < k_attr; ++a) s[3 + a] += (double)attr[a * m + p];
    }
    for (int a = 0; a < nf; ++a) atomicAdd(&acc[a * seg_stride + seg], s[a]);
}

__global__ void seg_keep_kernel(const int32_t *__restrict__ start, const int64_t *__restrict__ nseg,
                                int32_t min_count, int32_t *__restrict__ keep) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = *nseg;
    if (s >= S) return;
    keep[s] = (start[s + 1] - start[s]) >= min_count ? 1 : 0;
}

__global__ void seg_write_kernel(const int32_t *__restrict__ start, const int64_t *__restrict__ nseg,
                                 const int32_t *__restrict__ keep, const int32_t *__restrict__ kexcl,
                                 const int64_t *__restrict__ nkeep, const double *__restrict__ acc,
                                 int64_t seg_stride, const uint64_t *__restrict__ keys, int k_attr,
                                 int64_t capacity, float *__restrict__ out_xyz,
                                 float *__restrict__ out_attr, int32_t *__restrict__ out_count,
                                 uint64_t *__restrict__ out_key) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = *nseg;
    if (s >= S || !keep[s]) return;
    if (*nkeep > capacity) return;
    const int64_t j = kexcl[s];
    const int32_t cnt = start[s + 1] - start[s];
    const double inv = 1.0 / (double)cnt;
    for (int a = 0; a < 3; ++a) out_xyz[a * capacity + j] = (float)(acc[a * seg_stride + s] * inv);
    for (int a = 0; a < k_attr; ++a)
        out_attr[a * capacity + j] = (float)(acc[(3 + a) * seg_stride + s] * inv);
    out_count[j] = cnt;
    out_key[j] = keys[start[s]];
}

__global__ void prune_status_kernel(const int64_t *__restrict__ nkeep, int64_t capacity,
                                    int64_t *__restrict__ n_out, int32_t *__restrict__ status) {
    if (threadIdx.x || blockIdx.x) return;
    const int64_t k = *nkeep;
    *n_out = k;
    if (*status == 0 && k > capacity) *status = 1;
}

struct PruneLayout {
    uint64_t *k0, *k1;
    uint32_t *v0, *v1;
    int32_t *head, *excl, *start, *keep, *kexcl;
    int64_t *nseg, *nkeep;
    double *acc;
    void *scan_ws, *radix_ws;
};

PruneLayout carve_prune(void *ws, int64_t m, int32_t k_attr, size_t *used) {
    Carve c(ws, ~size_t(0));
    PruneLayout L;
    const size_t mm = (size_t)(m > 0 ? m : 1);
    L.k0 = c.take<uint64_t>(mm);
    L.k1 = c.take<uint64_t>(mm);
    L.v0 = c.take<uint32_t>(mm);
    L.v1 = c.take<uint32_t>(mm);
    L.head = c.take<int32_t>(mm);
    L.excl = c.take<int32_t>(mm);
    L.start = c.take<int32_t>(mm + 1);
    L.keep = c.take<int32_t>(mm);
    L.kexcl = c.take<int32_t>(mm);
    L.nseg = c.take<int64_t>(1);
    L.nkeep = c.take<int64_t>(1);
    L.acc = c.take<double>(mm * (size_t)(3 + k_attr));
    L.scan_ws = c.take<char>(scan_workspace_size(m));
    L.radix_ws = c.take<char>(radix_workspace_size(m));
    *used = c.used;
    return L;
}

inline unsigned blocks_for(int64_t count, int threads) {
    const int64_t b = (count + threads - 1) / threads;
    return (unsigned)(b > 0 ? b : 1);
}

// ------------------------------------------------------------ back projection
// X = R^T (D K^-1 (x + 1/2, y + 1/2, 1)^T - t) for the pixels whose
// accumulated alpha exceeds min_cover, D = depth_acc / cover (the
// alpha-weighted depth).
__global__ void bp_keep_kernel(const float *__restrict__ cover, int64_t hw, float min_cover,
                               int32_t *__restrict__ keep) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= hw) return;
    keep[i] = cover[i] > min_cover ? 1 : 0;
}

__global__ void bp_write_kernel(const float *__restrict__ depth_acc, const float *__restrict__ cover,
                                const int32_t *__restrict__ keep, const int32_t *__restrict__ excl,
                                gs4d_view V, int64_t capacity, float *__restrict__ out_xyz,
                                float *__restrict__ out_depth, int32_t *__restrict__ out_pixel,
                                double *__restrict__ depth_sum) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t hw = (int64_t)V.width * V.height;
    const bool kept = i < hw && keep[i];
    const float D = kept ? depth_acc[i] / cover[i] : 0.0f;
    if (depth_sum) {
        const double s = wave_sum_d((double)D);
        if (lane_id() == 0 && s != 0.0) atomicAdd(depth_sum, s);
    }
    if (!kept) return;
    const int64_t j = excl[i];
    if (j >= capacity) return;
    const int y = (int)(i / V.width), x = (int)(i - (int64_t)y * V.width);
    const float c0 = (((float)x + 0.5f) - V.cx) / V.fx * D;
    const float c1 = (((float)y + 0.5f) - V.cy) / V.fy * D;
    const float d0 = c0 - V.Rt[3], d1 = c1 - V.Rt[7], d2 = D - V.Rt[11];
    // R^T (xc - t): column j of R
    for (int a = 0; a < 3; ++a)
        out_xyz[a * capacity + j] = V.Rt[a] * d0 + V.Rt[4 + a] * d1 + V.Rt[8 + a] * d2;
    out_depth[j] = D;
    out_pixel[j] = (int32_t)i;
}

__global__ void bp_count_kernel(const int64_t *__restrict__ total, int64_t *__restrict__ n_out) {
    if (threadIdx.x || blockIdx.x) return;
    *n_out = *total;
}

// ------------------------------------------------------------ initialisation
__global__ void init_kernel(const float *__restrict__ xyz, const float *__restrict__ rgb,
                            const float *__restrict__ t, const float *__restrict__ depth,
                            const uint8_t *__restrict__ dyn, int64_t k, int64_t stride,
                            float log_vs, float log_vd, int pruned_s, int pruned_d,
                            float inv_focal, float log_st_dynamic, float logit0,
                            float *__restrict__ P) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    const bool d = dyn && dyn[i];
    // a class that is not pruned: the footprint of one back-projected pixel
    const float ls = (d ? pruned_d : pruned_s) ? (d ? log_vd : log_vs) : logf(depth[i] * inv_focal);
    for (int a = 0; a < 3; ++a) {
        P[a * k + i] = xyz[a * stride + i];
        P[(4 + a) * k + i] = ls;
        P[(17 + a) * k + i] = rgb[a * stride + i];
    }
    P[3 * k + i] = t[i];
    P[7 * k + i] = d ? log_st_dynamic : 0.0f;
    for (int a = 0; a < 4; ++a) {
        P[(8 + a) * k + i] = a == 0 ? 1.0f : 0.0f;
        P[(12 + a) * k + i] = a == 0 ? 1.0f : 0.0f;
    }
    P[16 * k + i] = logit0;
}

}  // namespace
}  // namespace gs4d

using namespace gs4d;

extern "C" size_t gs4d_grid_prune_workspace_size(int64_t m, int32_t k_attr) {
    size_t used = 0;
    carve_prune(nullptr, m, k_attr < 0 ? 0 : k_attr, &used);
    return used + 256;
}

extern "C" int gs4d_grid_prune(const float *xyz, const float *attr, int32_t k_attr,
                               const uint8_t *cls, int64_t m, float voxel_static,
                               float voxel_dynamic, int32_t min_count, int64_t capacity,
                               float *out_xyz, float *out_attr, int32_t *out_count,
                               uint64_t *out_key, int64_t *n_out, int32_t *status, void *ws,
                               size_t ws_bytes, void *stream) {
    GS4D_REQUIRE(m >= 0 && m < ((int64_t)1 << 31), "gs4d_grid_prune: m out of range");
    GS4D_REQUIRE(k_attr >= 0 && k_attr <= PR_MAX_ATTR, "gs4d_grid_prune: k_attr must be in [0, %d]",
                 PR_MAX_ATTR);
    GS4D_REQUIRE(min_count >= 1, "gs4d_grid_prune: min_count must be >= 1");
    GS4D_REQUIRE(capacity >= 0, "gs4d_grid_prune: capacity < 0");
    GS4D_REQUIRE(n_out && status, "gs4d_grid_prune: null n_out / status");
    GS4D_REQUIRE(m == 0 || xyz, "gs4d_grid_prune: null xyz");
    GS4D_REQUIRE(k_attr == 0 || m == 0 || attr, "gs4d_grid_prune: null attr");
    GS4D_REQUIRE(capacity == 0 || (out_xyz && out_count && out_key && (k_attr == 0 || out_attr)),
                 "gs4d_grid_prune: null output");
    GS4D_REQUIRE(ws && ws_bytes >= gs4d_grid_prune_workspace_size(m, k_attr),
                 "gs4d_grid_prune: workspace too small");
    hipStream_t st = as_stream(stream);
    GS4D_TRY(launch_fill<int32_t>(status, 0, 1, st));
    if (m == 0) return launch_fill<int64_t>(n_out, (int64_t)0, 1, st);
    size_t used = 0;
    PruneLayout L = carve_prune(ws, m, k_attr, &used);
    prune_keys_kernel<<<blocks_for(m, 256), 256, 0, st>>>(xyz, cls, m, voxel_static, voxel_dynamic,
                                                          L.k0, L.v0, status);
    GS4D_LAUNCH_CHECK("prune keys");
    int alt = 0;
    GS4D_TRY(radix_sort_u64(L.k0, L.v0, L.k1, L.v1, nullptr, m, m, 0, 64, L.radix_ws, st, &alt));
    const uint64_t *keys = alt ? L.k1 : L.k0;
    const uint32_t *order = alt ? L.v1 : L.v0;
    seg_head_kernel<<<blocks_for(m, 256), 256, 0, st>>>(keys, m, L.head);
    GS4D_LAUNCH_CHECK("prune heads");
    GS4D_TRY(exclusive_scan_i32(L.head, L.excl, m, L.nseg, L.scan_ws, st));
    seg_start_kernel<<<blocks_for(m, 256), 256, 0, st>>>(L.head, L.excl, m, L.start);
    GS4D_LAUNCH_CHECK("prune starts");
    GS4D_TRY(launch_fill<double>(L.acc, 0.0, m * (int64_t)(3 + k_attr), st));
    seg_sum_kernel<<<blocks_for((m + PR_CHUNK - 1) / PR_CHUNK, 128), 128, 0, st>>>(
        order, L.head, L.excl, xyz, attr, k_attr, m, m, L.acc);
    GS4D_LAUNCH_CHECK("prune sums");
    // the scan below covers keep[0..m): entries past the segment count stay 0
    GS4D_TRY(launch_fill<int32_t>(L.keep, 0, m, st));
    seg_keep_kernel<<<blocks_for(m, 256), 256, 0, st>>>(L.start, L.nseg, min_count, L.keep);
    GS4D_LAUNCH_CHECK("prune keep");
    GS4D_TRY(exclusive_scan_i32(L.keep, L.kexcl, m, L.nkeep, L.scan_ws, st));
    seg_write_kernel<<<blocks_for(m, 256), 256, 0, st>>>(L.start, L.nseg, L.keep, L.kexcl, L.nkeep,
                                                         L.acc, m, keys, k_attr, capacity, out_xyz,
                                                         out_attr, out_count, out_key);
    GS4D_LAUNCH_CHECK("prune write");
    prune_status_kernel<<<1, 64, 0, st>>>(L.nkeep, capacity, n_out, status);
    GS4D_LAUNCH_CHECK("prune status");
    return GS4D_OK;
}

extern "C" size_t gs4d_backproject_workspace_size(int64_t hw) {
    Carve c(nullptr, ~size_t(0));
    const size_t n = (size_t)(hw > 0 ? hw : 1);
    c.take<int32_t>(n);
    c.take<int32_t>(n);
    c.take<int64_t>(1);
    c.take<char>(scan_workspace_size(hw));
    return c.used + 256;
}

extern "C" int gs4d_backproject(const float *depth_acc, const float *cover, const gs4d_view *view,
                                float min_cover, int64_t capacity, float *out_xyz, float *out_depth,
                                int32_t *out_pixel, int64_t *n_out, double *depth_sum, void *ws,
                                size_t ws_bytes, void *stream) {
    GS4D_REQUIRE(view, "gs4d_backproject: null view");
    const int64_t hw = (int64_t)view->width * view->height;
    GS4D_REQUIRE(view->width > 0 && view->height > 0 && hw < ((int64_t)1 << 31),
                 "gs4d_backproject: bad image size %d x %d", view->width, view->height);
    GS4D_REQUIRE(view->fx != 0.0f && view->fy != 0.0f, "gs4d_backproject: zero focal length");
    GS4D_REQUIRE(min_cover > 0.0f, "gs4d_backproject: min_cover must be > 0");
    GS4D_REQUIRE(capacity >= 0, "gs4d_backproject: capacity < 0");
    GS4D_REQUIRE(depth_acc && cover && n_out, "gs4d_backproject: null input");
    GS4D_REQUIRE(capacity == 0 || (out_xyz && out_depth && out_pixel), "gs4d_backproject: null output");
    GS4D_REQUIRE(ws && ws_bytes >= gs4d_backproject_workspace_size(hw),
                 "gs4d_backproject: workspace too small");
    hipStream_t st = as_stream(stream);
    Carve c(ws, ws_bytes);
    int32_t *keep = c.take<int32_t>((size_t)hw);
    int32_t *excl = c.take<int32_t>((size_t)hw);
    int64_t *total = c.take<int64_t>(1);
    void *scan_ws = c.take<char>(scan_workspace_size(hw));
    bp_keep_kernel<<<blocks_for(hw, 256), 256, 0, st>>>(cover, hw, min_cover, keep);
    GS4D_LAUNCH_CHECK("backproject keep");
    GS4D_TRY(exclusive_scan_i32(keep, excl, hw, total, scan_ws, st));
    bp_write_kernel<<<blocks_for(hw, 256), 256, 0, st>>>(depth_acc, cover, keep, excl, *view,
                                                         capacity, out_xyz, out_depth, out_pixel,
                                                         depth_sum);
    GS4D_LAUNCH_CHECK("backproject write");
    bp_count_kernel<<<1, 64, 0, st>>>(total, n_out);
    GS4D_LAUNCH_CHECK("backproject count");
    return GS4D_OK;
}

extern "C" int gs4d_heuristic_init(const float *xyz, const float *rgb, const float *t,
                                   const float *depth, const uint8_t *dynamic, int64_t k,
                                   int64_t stride, float voxel_static, float voxel_dynamic,
                                   float focal, int32_t frames, float *params, void *stream) {
    GS4D_REQUIRE(k >= 0 && k < ((int64_t)1 << 31), "gs4d_heuristic_init: k out of range");
    GS4D_REQUIRE(stride >= k, "gs4d_heuristic_init: stride < k");
    GS4D_REQUIRE(frames >= 2, "gs4d_heuristic_init: frames must be >= 2");
    if (k == 0) return GS4D_OK;
    GS4D_REQUIRE(xyz && rgb && t && params, "gs4d_heuristic_init: null pointer");
    const bool unpruned = !(voxel_static > 0.0f) || (dynamic && !(voxel_dynamic > 0.0f));
    GS4D_REQUIRE(!unpruned || (depth && focal > 0.0f),
                 "gs4d_heuristic_init: a class that is not pruned needs depth and focal > 0");
    const int ps = voxel_static > 0.0f, pd = voxel_dynamic > 0.0f;
    const float log_vs = ps ? logf(voxel_static) : 0.0f;
    const float log_vd = pd ? logf(voxel_dynamic) : 0.0f;
    const float inv_focal = focal > 0.0f ? 1.0f / focal : 0.0f;
    const float log_st_dynamic = logf(2.0f / (float)frames);
    const float logit0 = logf(0.1f / 0.9f);
    init_kernel<<<blocks_for(k, 256), 256, 0, as_stream(stream)>>>(
        xyz, rgb, t, depth, dynamic, k, stride, log_vs, log_vd, ps, pd, inv_focal, log_st_dynamic,
        logit0, params);
    GS4D_LAUNCH_CHECK("gs4d_heuristic_init");
    return GS4D_OK;
}
