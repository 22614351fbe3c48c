// Tile binning and sorting (the tile-based splatting renderer of Sec. 3.1).
//
// Result: every visible (view, Gaussian) duplicated once per touched 16x16
// tile, as (key, value) = ((global tile << 32) | bits(FP32 depth), Gaussian)
// sorted ascending by (key, value).
//
// Counting (the default while tiles hold up to a few thousand pairs and a
// view has at most 8,192 tiles): per-(tile, block of Gaussians) pair counts,
// their scan, every pair written straight into its tile, then the per-tile
// depth sort of step 5 below, which also puts equal depths in Gaussian
// order -- four launches; see "counting strategy" further down.
//
// Per-tile radix (for larger tile grids):
//   1. device-wide exclusive scan of tiles-touched over the (view, Gaussian)
//      items -> each item's first pair slot, the pair count P and the
//      capacity flag (on device).
//   2. emit pairs in item order (and zero the tile ranges).
//   3. stable LSD radix sort of the P pairs on the tile bits only (1-2 digit
//      passes); inside one tile the pairs stay in Gaussian order.
//   4. tile ranges from adjacent key differences.
//   5. one workgroup per tile sorts its pairs stably on the 32 depth bits,
//      which yields exactly the ascending (key, value) order.
// Presort (for tiles of tens of thousands of pairs): a stable radix sort of
// the items on their depth bits (the first histogram pass builds the keys
// and zeroes the ranges), the scan of step 1 read in that order, emission in
// depth order, then steps 3 and 4; the pairs are then in order already.
//
// Radix sort: 8-bit digits; per pass a histogram kernel (per-block digit
// counts), a scan kernel (one wave per digit over the blocks, giving each
// digit's total), and a scatter kernel that ranks keys stably with wave ballots,
// regroups them by digit in LDS and writes each digit run contiguously.
#include "common.hpp"

#include <mutex>

namespace gs4d {
namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
// keys per block = 256 threads x ITEMS, by capacity: short blocks for the
// sorts of a few hundred thousand keys a training step makes, so that they
// still spread over all 256 compute units; long ones for tens of millions
constexpr int RS_TINY_ITEMS = 2;
constexpr int RS_SMALL_ITEMS = 4;
constexpr int RS_LARGE_ITEMS = 8;
constexpr int64_t RS_TINY_LIMIT = 1 << 18;
constexpr int64_t RS_SMALL_LIMIT = 1 << 22;

__device__ __forceinline__ int64_t read_count(const int64_t *count_dev, int64_t count_host,
                                              int64_t capacity) {
    int64_t n = count_dev ? *count_dev : count_host;
    if (n > capacity) n = capacity;
    if (n < 0) n = 0;
    return n;
}

// the digit of a pass: key bits [shift, shift + nbits), nbits <= 8 (the
// last pass of a sort on bits [lo, hi) takes only the bits below hi)
template <class K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, int nbits) {
    return (uint32_t)((key >> shift) & (K)((1u << nbits) - 1u));
}

// Block b covers keys [b*TILE, (b+1)*TILE), TILE = 256 * ITEMS.  Wave w owns
// the contiguous 64*ITEMS keys starting at b*TILE + w*64*ITEMS; item i of
// lane l is key w*64*ITEMS + i*64 + l, so every wave load reads 64
// consecutive keys.
template <class K, int RS_ITEMS>
__global__ void __launch_bounds__(RS_THREADS)
rs_hist_kernel(const K *__restrict__ keys, const int64_t *count_dev, int64_t count_host,
               int64_t capacity, int shift, int nbits, uint32_t *__restrict__ hist) {
    constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
    const int64_t n = read_count(count_dev, count_host, capacity);
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    const int64_t b = blockIdx.x;
    if (b >= nb) return;
    __shared__ uint32_t cnt[RS_WAVES][256];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    for (int i = t; i < RS_WAVES * 256; i += RS_THREADS) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t base = b * RS_TILE + (int64_t)w * (RS_TILE / RS_WAVES);
#pragma unroll 4
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t idx = base + i * 64 + l;
        if (idx < n) atomicAdd(&cnt[w][digit_of(keys[idx], shift, nbits)], 1u);
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < RS_WAVES; ++k) c += cnt[k][t];
    hist[(int64_t)t * nb + b] = c;
}

// Presort strategy: the items (view, Gaussian) as the source of the depth
// sort's first pass: item o's key is
// the bits of its FP32 depth (culled items, no tile touched: 0xFFFFFFFF, so
// they sort last) and its value o.  The first histogram pass builds keys
// and values itself (same block layout as rs_hist_kernel), and zeroes the
// tile ranges in the same launch (a tile no pair reaches stays (0, 0)).
struct ItemSource {
    const float4 *rec;
    const int32_t *touched;
    int32_t *ranges;
    int64_t n_range_ints;
};

template <int RS_ITEMS>
__global__ void __launch_bounds__(RS_THREADS)
rs_hist_items_kernel(ItemSource src, int64_t m, uint32_t *__restrict__ keys,
                     uint32_t *__restrict__ vals, uint32_t *__restrict__ hist) {
    constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    for (int64_t i = (int64_t)blockIdx.x * RS_THREADS + t; i < src.n_range_ints;
         i += (int64_t)gridDim.x * RS_THREADS)
        src.ranges[i] = 0;
    const int64_t nb = (m + RS_TILE - 1) / RS_TILE;
    const int64_t b = blockIdx.x;
    if (b >= nb) return;
    __shared__ uint32_t cnt[RS_WAVES][256];
    for (int i = t; i < RS_WAVES * 256; i += RS_THREADS) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t base = b * RS_TILE + (int64_t)w * (RS_TILE / RS_WAVES);
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t o = base + i * 64 + l;
        if (o < m) {
            const uint32_t key =
                src.touched[o] > 0 ? __float_as_uint(src.rec[3 * o + 1].z) : 0xFFFFFFFFu;
            keys[o] = key;
            vals[o] = (uint32_t)o;
            atomicAdd(&cnt[w][key & 0xFFu], 1u);
        }
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < RS_WAVES; ++k) c += cnt[k][t];
    hist[(int64_t)t * nb + b] = c;
}

// One wave per digit: exclusive prefix of hist[d][0..nb) in place and the
// digit's total count in row_total[d] (the offsets between digits are left to
// the scatter blocks, so no kernel needs device-wide atomics).
constexpr int RS_SCAN_LOADS = 16;

__global__ void __launch_bounds__(64)
rs_scan_kernel(uint32_t *__restrict__ hist, uint32_t *__restrict__ row_total,
               const int64_t *count_dev, int64_t count_host, int64_t capacity, int RS_TILE) {
    const int64_t n = read_count(count_dev, count_host, capacity);
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    if (nb == 0) return;
    const int d = blockIdx.x, l = threadIdx.x;
    uint32_t running = 0;
    uint32_t *row = hist + (int64_t)d * nb;
    // RS_SCAN_LOADS loads per lane in flight per step: the loop is bound by
    // load latency, not by the wave scans
    for (int64_t c0 = 0; c0 < nb; c0 += 64 * RS_SCAN_LOADS) {
        uint32_t x[RS_SCAN_LOADS];
#pragma unroll
        for (int i = 0; i < RS_SCAN_LOADS; ++i) {
            const int64_t idx = c0 + i * 64 + l;
            x[i] = idx < nb ? row[idx] : 0u;
        }
#pragma unroll
        for (int i = 0; i < RS_SCAN_LOADS; ++i) {
            uint32_t incl = x[i];
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off, 64);
                if (l >= off) incl += y;
            }
            const int64_t idx = c0 + i * 64 + l;
            if (idx < nb) row[idx] = running + incl - x[i];
            running += __shfl(incl, 63, 64);
        }
    }
    if (l == 0) row_total[d] = running;
}

template <class K, int RS_ITEMS>
__global__ void __launch_bounds__(RS_THREADS)
rs_scatter_kernel(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                  K *__restrict__ kout, uint32_t *__restrict__ vout, const int64_t *count_dev,
                  int64_t count_host, int64_t capacity, int shift, int nbits,
                  const uint32_t *__restrict__ hist, const uint32_t *__restrict__ row_total) {
    constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
    const int64_t n = read_count(count_dev, count_host, capacity);
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    const int64_t b = blockIdx.x;
    if (b >= nb) return;
    __shared__ K sk[RS_TILE];
    __shared__ uint32_t sv[RS_TILE];
    __shared__ uint32_t wcnt[RS_WAVES][256];   // per-wave running digit counts
    __shared__ uint32_t dstart[256];           // block-local start of each digit
    __shared__ uint32_t gbase[256];            // global start of this block's digit run
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    for (int i = t; i < RS_WAVES * 256; i += RS_THREADS) (&wcnt[0][0])[i] = 0;
    __syncthreads();

    const int64_t base = b * RS_TILE + (int64_t)w * (RS_TILE / RS_WAVES);
    const uint64_t lt_mask = (l == 0) ? 0ull : (~0ull >> (64 - l));
    K key[RS_ITEMS];
    uint32_t val[RS_ITEMS], rank[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t idx = base + i * 64 + l;
        const bool valid = idx < n;
        key[i] = valid ? kin[idx] : (K)0;
        val[i] = valid ? vin[idx] : 0u;
        const uint32_t d = digit_of(key[i], shift, nbits);
        // lanes holding the same digit: per significant digit bit, the lane's
        // bit as an all-ones / zero word, its ballot, and the lanes that agree
        // (xnor) in both halves of the mask
        const uint64_t vmask = __ballot(valid);
        uint32_t plo = (uint32_t)vmask, phi = (uint32_t)(vmask >> 32);
        for (int bit = 0; bit < nbits; ++bit) {
            const uint32_t own = (uint32_t)__builtin_amdgcn_sbfe((int)d, bit, 1);
            const uint64_t m = __ballot(own != 0u);
            plo &= ~((uint32_t)m ^ own);
            phi &= ~((uint32_t)(m >> 32) ^ own);
        }
        const uint64_t peers = ((uint64_t)phi << 32) | plo;
        const uint32_t before = __popcll(peers & lt_mask);
        uint32_t r = 0;
        if (valid) r = wcnt[w][d] + before;
        const bool leader = valid && before == 0;
        // all lanes have read wcnt[w][d] before the leader updates it
        __builtin_amdgcn_wave_barrier();
        if (leader) wcnt[w][d] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        rank[i] = valid ? r : 0xFFFFFFFFu;
    }
    __syncthreads();
    // per digit: prefix over waves, block-local start, global start (the
    // keys of all smaller digits plus this digit's keys in earlier blocks)
    {
        const int d = t;
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < RS_WAVES; ++k) {
            const uint32_t c = wcnt[k][d];
            wcnt[k][d] = run;
            run += c;
        }
        // block exclusive scans over the 256 digits of this block's counts
        // and of the digit totals
        const uint32_t tot = row_total[d];
        uint32_t incl = run, tincl = tot;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            const uint32_t z = __shfl_up(tincl, off, 64);
            if (l >= off) { incl += y; tincl += z; }
        }
        __shared__ uint32_t wsum[2][RS_WAVES];
        if (l == 63) { wsum[0][w] = incl; wsum[1][w] = tincl; }
        const uint32_t in_row = hist[(int64_t)d * nb + b];
        __syncthreads();
        uint32_t off = 0, toff = 0;
        for (int k = 0; k < w; ++k) { off += wsum[0][k]; toff += wsum[1][k]; }
        dstart[d] = off + incl - run;
        gbase[d] = toff + tincl - tot + in_row;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        if (rank[i] != 0xFFFFFFFFu) {
            const uint32_t d = digit_of(key[i], shift, nbits);
            const uint32_t pos = dstart[d] + wcnt[w][d] + rank[i];
            sk[pos] = key[i];
            sv[pos] = val[i];
        }
    }
    __syncthreads();
    const int64_t nvalid = (n - b * RS_TILE) < RS_TILE ? (n - b * RS_TILE) : RS_TILE;
#pragma unroll 4
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int idx = i * RS_THREADS + t;
        if (idx < nvalid) {
            const K k = sk[idx];
            const uint32_t d = digit_of(k, shift, nbits);
            const uint32_t dst = gbase[d] + (uint32_t)idx - dstart[d];
            kout[dst] = k;
            vout[dst] = sv[idx];
        }
    }
}

// ---------------------------------------------------------------- scan
// values per block = 256 threads x ITEMS: 4 up to 2^20 values, so that the
// few hundred thousand of a training step still make enough blocks, else 16
constexpr int SC_THREADS = 256;
constexpr int SC_SMALL_ITEMS = 4;
constexpr int SC_LARGE_ITEMS = 16;
constexpr int64_t SC_SMALL_LIMIT = 1 << 20;

__device__ __forceinline__ int64_t block_excl_scan(int64_t x, int64_t *total) {
    __shared__ int64_t ws[SC_THREADS / 64];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    int64_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(incl, off, 64);
        if (l >= off) incl += y;
    }
    if (l == 63) ws[w] = incl;
    __syncthreads();
    int64_t off = 0, tot = 0;
    for (int k = 0; k < SC_THREADS / 64; ++k) {
        if (k < w) off += ws[k];
        tot += ws[k];
    }
    __syncthreads();
    *total = tot;
    return off + incl - x;
}

// value i of a scan input: in[i], or in[gather[i]] when a gather index is given
__device__ __forceinline__ int32_t scan_in(const int32_t *__restrict__ in,
                                           const uint32_t *__restrict__ gather, int64_t i) {
    return gather ? in[gather[i]] : in[i];
}

template <int ITEMS>
__global__ void __launch_bounds__(SC_THREADS)
scan_reduce_kernel(const int32_t *__restrict__ in, const uint32_t *__restrict__ gather,
                   int64_t count, int64_t *__restrict__ bsum) {
    const int64_t b = blockIdx.x;
    const int64_t base = b * (SC_THREADS * ITEMS);
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = base + (int64_t)i * SC_THREADS + threadIdx.x;
        if (idx < count) s += scan_in(in, gather, idx);
    }
    int64_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) bsum[b] = tot;
}

// Exclusive scan of the block sums; with `n_pairs`, also the pair count and
// the capacity flag of the binning (the scanned values are pair counts).
__global__ void __launch_bounds__(SC_THREADS)
scan_top_kernel(int64_t *__restrict__ bsum, int64_t nblocks, int64_t *__restrict__ total,
                int64_t capacity, int64_t *__restrict__ n_pairs, int32_t *__restrict__ overflow) {
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nblocks; c0 += SC_THREADS) {
        const int64_t idx = c0 + threadIdx.x;
        const int64_t x = idx < nblocks ? bsum[idx] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(x, &tot);
        if (idx < nblocks) bsum[idx] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        *total = carry;
        if (n_pairs) {
            *n_pairs = carry;
            *overflow = carry > capacity ? 1 : 0;
        }
    }
}

// Scans of at most SC_FUSE_BLOCKS blocks skip scan_top_kernel: each
// down-sweep block adds up the block sums before its own (at most a few
// thousand values), and the last block writes the total (and, for the
// binning, the pair count and capacity flag).
constexpr int64_t SC_FUSE_BLOCKS = 2048;

struct ScanTop {
    int self_prefix;   // 1: bsum holds plain block sums; 0: scanned by scan_top_kernel
    int64_t nblocks;
    int64_t *total;
    int64_t capacity;
    int64_t *n_pairs;   // optional, with overflow
    int32_t *overflow;
};

// Loads and stores are coalesced (value i*256 + thread of the block); the
// scan itself runs over ITEMS consecutive values per thread, regrouped in LDS.
template <int ITEMS>
__global__ void __launch_bounds__(SC_THREADS)
scan_down_kernel(const int32_t *__restrict__ in, const uint32_t *__restrict__ gather,
                 int32_t *__restrict__ out, int64_t count, const int64_t *__restrict__ bsum,
                 ScanTop top) {
    constexpr int TILE = SC_THREADS * ITEMS;
    __shared__ int32_t tile[TILE];
    const int64_t b = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t base = b * TILE;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = base + (int64_t)i * SC_THREADS + t;
        tile[i * SC_THREADS + t] = idx < count ? scan_in(in, gather, idx) : 0;
    }
    __syncthreads();
    int32_t v[ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        v[i] = tile[t * ITEMS + i];
        s += v[i];
    }
    // every thread has read its values before the scan's barriers
    int64_t prefix;
    if (top.self_prefix) {
        int64_t part = 0;
        for (int64_t i = t; i < b; i += SC_THREADS) part += bsum[i];
        block_excl_scan(part, &prefix);
    } else {
        prefix = bsum[b];
    }
    int64_t tot;
    int64_t run = prefix + block_excl_scan(s, &tot);
    if (top.self_prefix && b == top.nblocks - 1 && t == 0) {
        const int64_t all = prefix + tot;
        *top.total = all;
        if (top.n_pairs) {
            *top.n_pairs = all;
            *top.overflow = all > top.capacity ? 1 : 0;
        }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        tile[t * ITEMS + i] = (int32_t)run;
        run += v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = base + (int64_t)i * SC_THREADS + t;
        if (idx < count) out[idx] = tile[i * SC_THREADS + t];
    }
}

inline int sc_items(int64_t count) {
    return count <= SC_SMALL_LIMIT ? SC_SMALL_ITEMS : SC_LARGE_ITEMS;
}

inline int64_t sc_blocks(int64_t count) {
    const int64_t tile = (int64_t)SC_THREADS * sc_items(count);
    return (count + tile - 1) / tile;
}

// the launches of one scan: block sums, (for many blocks) their scan with
// the optional binning outputs, the down-sweep
int scan_launch(const int32_t *in, const uint32_t *gather, int32_t *out, int64_t count,
                int64_t *total, int64_t *bsum, int64_t capacity, int64_t *n_pairs,
                int32_t *overflow, hipStream_t st) {
    const int64_t nb = sc_blocks(count);
    const bool fused = nb <= SC_FUSE_BLOCKS;
    const ScanTop top{fused ? 1 : 0, nb, total, capacity, n_pairs, overflow};
    if (sc_items(count) == SC_SMALL_ITEMS)
        scan_reduce_kernel<SC_SMALL_ITEMS><<<(unsigned)nb, SC_THREADS, 0, st>>>(in, gather, count, bsum);
    else
        scan_reduce_kernel<SC_LARGE_ITEMS><<<(unsigned)nb, SC_THREADS, 0, st>>>(in, gather, count, bsum);
    if (!fused)
        scan_top_kernel<<<1, SC_THREADS, 0, st>>>(bsum, nb, total, capacity, n_pairs, overflow);
    if (sc_items(count) == SC_SMALL_ITEMS)
        scan_down_kernel<SC_SMALL_ITEMS><<<(unsigned)nb, SC_THREADS, 0, st>>>(in, gather, out, count,
                                                                             bsum, top);
    else
        scan_down_kernel<SC_LARGE_ITEMS><<<(unsigned)nb, SC_THREADS, 0, st>>>(in, gather, out, count,
                                                                             bsum, top);
    return GS4D_OK;
}

// ---------------------------------------------------------------- binning kernels
// The pairs of one wave's items.  An item's pairs are its rectangle's tiles
// in row-major order from slot off on: key (global tile << 32) | depth bits,
// value g.  The lanes hold items that are consecutive in the pair-offset
// scan, so their pairs fill one contiguous slot range [S, S + total); the
// wave writes it 64 slots per step (coalesced stores), lane j taking slot
// C + j.  The item owning a slot is the highest lane whose first slot is at
// or before it: the lanes whose item starts inside the step mark their start
// in the wave's 64 LDS slots, a prefix maximum over the lanes spreads each
// mark to the slots after it, and the lane whose item started before the step
// covers the slots ahead of the first mark.  Every lane of the wave calls
// this; `mark` holds -1 in all 64 slots on entry and again on return.  Slots
// outside [0, capacity) are not written.
constexpr int EMIT_THREADS = 128;

__device__ __forceinline__ void emit_wave_pairs(bool valid, int32_t off, int32_t cnt, int4 r,
                                                uint32_t lo, uint32_t g, uint32_t tbase,
                                                int32_t tiles_x, int64_t capacity, int32_t *mark,
                                                uint64_t *__restrict__ keys,
                                                uint32_t *__restrict__ vals) {
    const int lane = threadIdx.x & 63;
    valid = valid && cnt > 0;
    const uint64_t vm = __ballot(valid);
    if (vm == 0) return;
    const int64_t S = __builtin_amdgcn_readlane(off, __builtin_ctzll(vm));
    int32_t total = valid ? cnt : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) total += __shfl_xor(total, d, 64);
    for (int64_t C = S; C < S + total; C += 64) {
        const int64_t rel = (int64_t)off - C;
        if (valid && rel >= 0 && rel < 64) mark[rel] = lane;
        __builtin_amdgcn_wave_barrier();
        int own = mark[lane];
        __builtin_amdgcn_wave_barrier();
        mark[lane] = -1;
        const uint64_t before = __ballot(valid && rel < 0);
        const int carry = before ? 63 - __builtin_clzll(before) : -1;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(own, d, 64);
            if (lane >= d) own = max(own, y);
        }
        own = max(own, carry);
        const int src = own < 0 ? 0 : own;
        const int32_t ooff = __shfl(off, src, 64);
        const int x0 = __shfl(r.x, src, 64), y0 = __shfl(r.y, src, 64);
        const int w = __shfl(r.z, src, 64) - x0;
        const uint32_t olo = (uint32_t)__shfl((int)lo, src, 64);
        const uint32_t og = (uint32_t)__shfl((int)g, src, 64);
        const uint32_t otb = (uint32_t)__shfl((int)tbase, src, 64);
        const int64_t slot = C + lane;
        if (own >= 0 && w > 0 && slot < S + total && slot >= 0 && slot < capacity) {
            const int local = (int)(slot - ooff);
            const int ty = local / w, tx = local - ty * w;
            const uint64_t tile = (uint64_t)otb + (uint64_t)(y0 + ty) * tiles_x + (x0 + tx);
            keys[slot] = (tile << 32) | olo;
            vals[slot] = og;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Item o = view vi * n + Gaussian g (grid: x over g, y over vi) writes its
// touched[o] pairs from offs[o] on.  The grid also zeroes the tile ranges (a
// tile no pair reaches stays (0, 0)).
__global__ void __launch_bounds__(EMIT_THREADS)
emit_kernel(const float4 *__restrict__ rec, const int32_t *__restrict__ touched,
            const int32_t *__restrict__ offs, const int4 *__restrict__ rect, int64_t n,
            int32_t tiles_x, int32_t tiles_per_view, int64_t capacity, uint64_t *__restrict__ keys,
            uint32_t *__restrict__ vals, int32_t *__restrict__ ranges, int64_t n_range_ints) {
    __shared__ int32_t mark[EMIT_THREADS / 64][64];
    mark[threadIdx.x >> 6][threadIdx.x & 63] = -1;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t vi = blockIdx.y;
    const int64_t stride = (int64_t)gridDim.x * gridDim.y * blockDim.x;
    for (int64_t i = g + (int64_t)vi * gridDim.x * blockDim.x; i < n_range_ints; i += stride)
        ranges[i] = 0;
    bool valid = false;
    int32_t cnt = 0, off = 0;
    int4 r = make_int4(0, 0, 0, 0);
    uint32_t lo = 0;
    if (g < n) {
        const int64_t o = (int64_t)vi * n + g;
        cnt = touched[o];
        if (cnt > 0) {
            valid = true;
            off = offs[o];
            r = rect[o];
            lo = __float_as_uint(rec[3 * o + 1].z);
        }
    }
    __builtin_amdgcn_wave_barrier();
    emit_wave_pairs(valid, off, cnt, r, lo, (uint32_t)g, vi * (uint32_t)tiles_per_view, tiles_x,
                    capacity, mark[threadIdx.x >> 6], keys, vals);
}

// Presort strategy: items in depth order k (order[k] = item o) write their
// pairs from offs[k] on; inside one tile they are then ascending in (depth
// bits, Gaussian) already.
__global__ void __launch_bounds__(EMIT_THREADS)
emit_depth_order_kernel(const uint32_t *__restrict__ dkeys, const uint32_t *__restrict__ order,
                        const int32_t *__restrict__ touched, const int32_t *__restrict__ offs,
                        const int4 *__restrict__ rect, int64_t m, int64_t n, int32_t tiles_x,
                        int32_t tiles_per_view, int64_t capacity, uint64_t *__restrict__ keys,
                        uint32_t *__restrict__ vals) {
    __shared__ int32_t mark[EMIT_THREADS / 64][64];
    mark[threadIdx.x >> 6][threadIdx.x & 63] = -1;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool valid = false;
    int32_t cnt = 0, off = 0;
    int4 r = make_int4(0, 0, 0, 0);
    uint32_t lo = 0, g = 0, tbase = 0;
    if (k < m) {
        const uint32_t o = order[k];
        cnt = touched[o];
        if (cnt > 0) {
            valid = true;
            off = offs[k];
            const uint32_t vi = (uint32_t)(o / (uint64_t)n);
            g = (uint32_t)(o - (uint64_t)vi * (uint64_t)n);
            r = rect[o];
            lo = dkeys[k];
            tbase = vi * (uint32_t)tiles_per_view;
        }
    }
    __builtin_amdgcn_wave_barrier();
    emit_wave_pairs(valid, off, cnt, r, lo, g, tbase, tiles_x, capacity, mark[threadIdx.x >> 6],
                    keys, vals);
}

// Tile ranges from adjacent key differences: where the tile changes between
// pairs i - 1 and i, the earlier tile ends and the later one starts at i; the
// last pair closes its tile.  Each thread takes RG_UNROLL pairs one grid
// stride apart, so a wave's loads stay coalesced and several are in flight
// (the kernel is bound by load latency otherwise).  Only a key's upper word
// (the tile) is read; the tile of pair i - 1 comes from the next lower lane,
// lane 0 reads it.
constexpr int RG_UNROLL = 4;

__global__ void ranges_kernel(const uint64_t *__restrict__ keys, const int64_t *__restrict__ n_pairs,
                              int64_t capacity, int64_t n_tiles, int2 *__restrict__ ranges) {
    const int64_t n = *n_pairs;
    if (n > capacity) return;   // overflow: every tile stays empty (0, 0)
    const uint32_t *hi = reinterpret_cast<const uint32_t *>(keys) + 1;   // word 2 i + 1
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b - lane < n;
         b += RG_UNROLL * stride) {
        uint32_t cur[RG_UNROLL], prv[RG_UNROLL];
#pragma unroll
        for (int u = 0; u < RG_UNROLL; ++u) {
            const int64_t i = b + u * stride;
            cur[u] = i < n ? hi[2 * i] : ~0u;
            prv[u] = (lane == 0 && i > 0 && i <= n) ? hi[2 * (i - 1)] : ~0u;
        }
#pragma unroll
        for (int u = 0; u < RG_UNROLL; ++u) {
            const uint32_t up = __shfl_up(cur[u], 1, 64);
            if (lane > 0) prv[u] = up;
        }
#pragma unroll
        for (int u = 0; u < RG_UNROLL; ++u) {
            const int64_t i = b + u * stride;
            if (i >= n) break;
            const uint32_t tile = cur[u], prev = prv[u];
            if (tile != prev) {
                if (tile < (uint64_t)n_tiles) ranges[tile].x = (int32_t)i;
                if (prev < (uint64_t)n_tiles) ranges[prev].y = (int32_t)i;
            }
            if (i == n - 1 && tile < (uint64_t)n_tiles) ranges[tile].y = (int32_t)n;
        }
    }
}

// ---------------------------------------------------------------- per-tile depth order
// One workgroup per tile sorts its pairs stably on the 32 depth bits (LSD,
// 8-bit digits); runs of equal depth bits are then put in Gaussian order
// (the pairs may arrive in any order), giving the ascending (depth bits,
// Gaussian) order inside the tile.  A tile of at most SEG_CAP pairs is
// sorted in registers and LDS; a longer one passes through global memory
// SEG_CAP pairs at a time, with the spare pair buffer as the other side of
// each pass.  A digit pass in which
// every pair has the same digit leaves the order as it is and is skipped.
//
// Pair layout inside a chunk of R * 256 pairs: wave w owns pairs
// [w*64*R, (w+1)*64*R); item i of lane l is pair (w*R + i)*64 + l.  A pair's
// place in a pass: the start of its digit, plus the pairs of that digit in
// earlier waves (and earlier chunks), plus its rank among the earlier pairs
// of its wave with that digit (wave ballots).
constexpr int SEG_THREADS = 256;
constexpr int SEG_WAVES = SEG_THREADS / 64;
constexpr int SEG_ITEMS = 8;
constexpr int SEG_CAP = SEG_THREADS * SEG_ITEMS;
constexpr int SEG_RUN = 32;   // longest run of equal keys put in order in place

struct SegShared {
    uint32_t key[SEG_CAP];
    uint32_t val[SEG_CAP];
    uint32_t cnt[2][SEG_WAVES][256];   // per (wave, digit): counts, then starts
    uint32_t base[256];                // long tiles: start of each digit's next run
    uint32_t kmin[SEG_WAVES], kmax[SEG_WAVES];
    int skip;
    int ties;   // equal depth keys seen in the tile
};

template <int CTRL, int ROW_MASK, bool MAX>
__device__ __forceinline__ uint32_t dpp_extreme(uint32_t x) {
    const uint32_t y =
        (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, ROW_MASK, 0xF, false);
    return MAX ? (x > y ? x : y) : (x < y ? x : y);
}

// minimum (or maximum) over the 64 lanes of a wave, in every lane
template <bool MAX>
__device__ __forceinline__ uint32_t wave_extreme(uint32_t x) {
    x = dpp_extreme<0x111, 0xF, MAX>(x);   // row_shr:1
    x = dpp_extreme<0x112, 0xF, MAX>(x);   // row_shr:2
    x = dpp_extreme<0x114, 0xF, MAX>(x);   // row_shr:4
    x = dpp_extreme<0x118, 0xF, MAX>(x);   // row_shr:8
    x = dpp_extreme<0x142, 0xA, MAX>(x);   // row_bcast:15
    x = dpp_extreme<0x143, 0xC, MAX>(x);   // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// lanes of this wave that are valid and hold the same digit, bits
// [shift, shift + nbits) of k, as this lane: per bit, the lane's bit as an
// all-ones / zero word, its ballot, and the lanes that agree with it
// (xnor), in both halves of the mask
__device__ __forceinline__ uint64_t same_digit(uint32_t k, int shift, bool valid, int nbits) {
    const uint64_t v = __ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    for (int bit = 0; bit < nbits; ++bit) {
        const uint32_t own = (uint32_t)__builtin_amdgcn_sbfe((int)k, shift + bit, 1);
        const uint64_t m = __ballot(own != 0u);
        lo &= ~((uint32_t)m ^ own);
        hi &= ~((uint32_t)(m >> 32) ^ own);
    }
    return ((uint64_t)hi << 32) | lo;
}

// Rank of each item of this thread among the earlier items of its wave with
// the same digit; c[w][d] counts the wave's items of digit d (zero on entry).
// Per round, the first lane of each digit's run adds the run's length with a
// returning LDS atomic (a wave's LDS operations take effect in order, so the
// rounds need not wait for each other) and its peers read the old count
// from it.
__device__ __forceinline__ void rank_items(const uint32_t (&k)[SEG_ITEMS],
                                           uint32_t (&rank)[SEG_ITEMS], int R, int first,
                                           int len, int shift, int nbits, uint32_t (*c)[256]) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const uint64_t lt_mask = (l == 0) ? 0ull : (~0ull >> (64 - l));
    uint32_t old[SEG_ITEMS];
    int lead[SEG_ITEMS];
#pragma unroll
    for (int i = 0; i < SEG_ITEMS; ++i) {
        if (i < R) {
            const bool valid = first + (w * R + i) * 64 + l < len;
            const uint32_t d = (k[i] >> shift) & 0xFFu;
            const uint64_t peers = same_digit(k[i], shift, valid, nbits);
            const uint32_t before = (uint32_t)__popcll(peers & lt_mask);
            uint32_t o = 0;
            if (valid && before == 0) o = atomicAdd(&c[w][d], (uint32_t)__popcll(peers));
            old[i] = o;
            rank[i] = before;
            lead[i] = valid ? (int)__builtin_ctzll(peers) : l;
        }
    }
#pragma unroll
    for (int i = 0; i < SEG_ITEMS; ++i)
        if (i < R) rank[i] += (uint32_t)__shfl((int)old[i], lead[i], 64);
}

// inclusive prefix sum over the 64 lanes of a wave: shifts inside rows of
// 16 lanes, then the row totals broadcast into the rows above (DPP)
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
}

// Wave 0: exclusive scan of the 256 digit totals tot(d) (lane l holds digits
// l, l+64, l+128, l+192) into start(d); returns, in every lane, whether one
// digit holds all `len` pairs.
__device__ __forceinline__ bool wave_digit_scan(const uint32_t (&tot)[4], uint32_t (&start)[4],
                                                int len) {
    uint32_t carry = 0;
    bool whole = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t incl = wave_incl_scan(tot[j]);
        start[j] = carry + incl - tot[j];
        carry += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        whole |= tot[j] == (uint32_t)len;
    }
    return __ballot(whole) != 0;
}

// pair j of the segment from the output arrays (at == 0) or the spare buffer
__device__ __forceinline__ void seg_load(const uint64_t *keys, const uint32_t *vals,
                                         const uint64_t *spill, bool in_spill, int64_t j,
                                         uint32_t &k, uint32_t &v) {
    if (in_spill) {
        const uint64_t x = spill[j];
        k = (uint32_t)x;
        v = (uint32_t)(x >> 32);
    } else {
        k = (uint32_t)keys[j];
        v = vals[j];
    }
}

__device__ __forceinline__ void seg_store(uint64_t *keys, uint32_t *vals, uint64_t *spill,
                                          bool to_spill, int64_t j, uint64_t tile_hi,
                                          uint32_t k, uint32_t v) {
    if (to_spill) {
        spill[j] = (uint64_t)k | ((uint64_t)v << 32);
    } else {
        keys[j] = tile_hi | k;
        vals[j] = v;
    }
}

// Four 8-bit passes through global memory for a tile longer than SEG_CAP,
// keyed on the depth bits or (BY_VALUE) on the Gaussian index; the pairs
// start and end in the output arrays.
template <bool BY_VALUE>
__device__ __forceinline__ void long_tile_passes(SegShared &sh, uint64_t *__restrict__ keys,
                                 uint32_t *__restrict__ vals, uint64_t *__restrict__ spill,
                                 int64_t start, int len, uint64_t tile_hi) {
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    bool in_spill = false;
    uint32_t k[SEG_ITEMS], v[SEG_ITEMS], rank[SEG_ITEMS];
    for (int p = 0; p < 4; ++p) {
        const int shift = 8 * p;
        sh.base[t] = 0;
        for (int i = t; i < 2 * SEG_WAVES * 256; i += SEG_THREADS) (&sh.cnt[0][0][0])[i] = 0;
        __syncthreads();
        for (int e = t; e < len; e += SEG_THREADS) {
            uint32_t ke, ve;
            seg_load(keys, vals, spill, in_spill, start + e, ke, ve);
            atomicAdd(&sh.base[((BY_VALUE ? ve : ke) >> shift) & 0xFFu], 1u);
        }
        __syncthreads();
        if (w == 0) {
            uint32_t tot[4], st[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) tot[j] = sh.base[j * 64 + l];
            const bool whole = wave_digit_scan(tot, st, len);
#pragma unroll
            for (int j = 0; j < 4; ++j) sh.base[j * 64 + l] = st[j];
            if (l == 0) sh.skip = whole ? 1 : 0;
        }
        __syncthreads();
        if (sh.skip) continue;
        for (int c0 = 0, ci = 0; c0 < len; c0 += SEG_CAP, ++ci) {
            uint32_t (*c)[256] = sh.cnt[ci & 1];
#pragma unroll
            for (int i = 0; i < SEG_ITEMS; ++i) {
                const int e = c0 + (w * SEG_ITEMS + i) * 64 + l;
                if (e < len) {
                    seg_load(keys, vals, spill, in_spill, start + e, k[i], v[i]);
                } else {
                    k[i] = 0;
                    v[i] = 0;
                }
            }
            rank_items(BY_VALUE ? v : k, rank, SEG_ITEMS, c0, len, shift, 8, c);
            __syncthreads();
            // digit t: starts of its run in each wave of this chunk; the next
            // chunk's counters are cleared
            {
                uint32_t run = sh.base[t];
#pragma unroll
                for (int ww = 0; ww < SEG_WAVES; ++ww) {
                    const uint32_t x = c[ww][t];
                    c[ww][t] = run;
                    run += x;
                }
                sh.base[t] = run;
#pragma unroll
                for (int ww = 0; ww < SEG_WAVES; ++ww) sh.cnt[(ci + 1) & 1][ww][t] = 0;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < SEG_ITEMS; ++i) {
                const int e = c0 + (w * SEG_ITEMS + i) * 64 + l;
                if (e < len) {
                    const uint32_t d = ((BY_VALUE ? v[i] : k[i]) >> shift) & 0xFFu;
                    const uint32_t pos = c[w][d] + rank[i];
                    seg_store(keys, vals, spill, !in_spill, start + pos, tile_hi, k[i], v[i]);
                }
            }
        }
        // the pass's stores are complete before the next pass reads them
        __syncthreads();
        in_spill = !in_spill;
    }
    if (in_spill) {
        for (int e = t; e < len; e += SEG_THREADS) {
            uint32_t ke, ve;
            seg_load(keys, vals, spill, true, start + e, ke, ve);
            seg_store(keys, vals, spill, false, start + e, tile_hi, ke, ve);
        }
    }
    __syncthreads();
}

// a long tile: sorted on the depth bits; where equal depths remain, sorted
// again on (Gaussian, then depth), so that equal depths end up in Gaussian
// order whatever order the pairs arrived in
__device__ __forceinline__ void long_tile_sort(SegShared &sh, uint64_t *__restrict__ keys,
                               uint32_t *__restrict__ vals, uint64_t *__restrict__ spill,
                               int64_t start, int len, uint64_t tile_hi) {
    long_tile_passes<false>(sh, keys, vals, spill, start, len, tile_hi);
    bool tie = false;
    for (int e = threadIdx.x + 1; e < len; e += SEG_THREADS)
        tie |= (uint32_t)keys[start + e] == (uint32_t)keys[start + e - 1];
    if (__ballot(tie) != 0 && (threadIdx.x & 63) == 0) sh.ties = 1;
    __syncthreads();
    if (!sh.ties) return;
    long_tile_passes<true>(sh, keys, vals, spill, start, len, tile_hi);
    long_tile_passes<false>(sh, keys, vals, spill, start, len, tile_hi);
}

// One stable LSD sort of a short tile held in registers (item i of lane l
// of wave w: pair (w*R + i)*64 + l) on the `bits` low bits of key[], with
// pay[] carried along; the counter set `par & 1` is zero on entry.  Returns
// the counter parity for the next sort.
__device__ __forceinline__ int seg_lsd(SegShared &sh, uint32_t (&key)[SEG_ITEMS],
                                       uint32_t (&pay)[SEG_ITEMS], int R, int len, int bits,
                                       int par, bool &tie) {
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    uint32_t rank[SEG_ITEMS];
    for (int p = 0; 8 * p < bits; ++p, ++par) {
        const int shift = 8 * p;
        const int nbits = bits - shift < 8 ? bits - shift : 8;
        uint32_t (*c)[256] = sh.cnt[par & 1];
        rank_items(key, rank, R, 0, len, shift, nbits, c);
        __syncthreads();
        // wave 0 turns the counts into starts; the next pass's counters are
        // cleared meanwhile
#pragma unroll
        for (int ww = 0; ww < SEG_WAVES; ++ww) sh.cnt[(par + 1) & 1][ww][t] = 0;
        if (w == 0) {
            uint32_t tot[4], st[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int d = j * 64 + l;
                tot[j] = 0;
#pragma unroll
                for (int ww = 0; ww < SEG_WAVES; ++ww) tot[j] += c[ww][d];
            }
            const bool whole = wave_digit_scan(tot, st, len);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int d = j * 64 + l;
                uint32_t run = st[j];
#pragma unroll
                for (int ww = 0; ww < SEG_WAVES; ++ww) {
                    const uint32_t x = c[ww][d];
                    c[ww][d] = run;
                    run += x;
                }
            }
            if (l == 0) sh.skip = whole ? 1 : 0;
        }
        __syncthreads();
        if (sh.skip) continue;
#pragma unroll
        for (int i = 0; i < SEG_ITEMS; ++i) {
            if (i < R && (w * R + i) * 64 + l < len) {
                const uint32_t pos = c[w][(key[i] >> shift) & 0xFFu] + rank[i];
                sh.key[pos] = key[i];
                sh.val[pos] = pay[i];
            }
        }
        __syncthreads();
        // read back in sorted order; `tie`: this thread's pair equals the one
        // before it (the last pass that moved the pairs decides)
        tie = false;
#pragma unroll
        for (int i = 0; i < SEG_ITEMS; ++i) {
            const int e = (w * R + i) * 64 + l;
            if (i < R && e < len) {
                key[i] = sh.key[e];
                pay[i] = sh.val[e];
                tie |= e >= 1 && sh.key[e - 1] == key[i];
            }
        }
    }
    return par;
}

// minimum of lo and maximum of hi over the block (every thread passes its
// values; all get the results); earlier readers of kmin / kmax must be done
__device__ __forceinline__ void block_min_max(SegShared &sh, uint32_t &lo, uint32_t &hi) {
    const int w = threadIdx.x >> 6;
    lo = wave_extreme<false>(lo);
    hi = wave_extreme<true>(hi);
    if ((threadIdx.x & 63) == 0) {
        sh.kmin[w] = lo;
        sh.kmax[w] = hi;
    }
    __syncthreads();
    lo = sh.kmin[0];
    hi = sh.kmax[0];
#pragma unroll
    for (int ww = 1; ww < SEG_WAVES; ++ww) {
        lo = sh.kmin[ww] < lo ? sh.kmin[ww] : lo;
        hi = sh.kmax[ww] > hi ? sh.kmax[ww] : hi;
    }
}

// five waves per SIMD (96 VGPRs): with the run fix for equal depths the
// kernel needs more than the 80 VGPRs of six waves, and spilling there wrote
// about 70 B of scratch per lane back to HBM (27 MB per launch at scene
// scale); the batched set's 16k tiles took 162 us at six waves, 152 at five
// Where the pairs' depth bits come from when only their values were written
// (GATHER): item (view, g)'s word, view = tile / tiles_per_view.
struct DepthSource {
    const uint32_t *dbits = nullptr;   // [view][n] depth bits of the visible items
    int64_t n = 0;
    int32_t tiles_per_view = 1;
};

__device__ __forceinline__ uint32_t gathered_depth(const DepthSource &src, int64_t vi,
                                                   uint32_t g) {
    return src.dbits[vi * src.n + g];
}

template <bool GATHER>
__global__ void __launch_bounds__(SEG_THREADS) __attribute__((amdgpu_waves_per_eu(5)))
tile_depth_sort_kernel(uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                       const int2 *__restrict__ ranges, uint64_t *__restrict__ spill,
                       DepthSource src) {
    __shared__ SegShared sh;
    const int2 r = ranges[blockIdx.x];
    const int len = r.y - r.x;
    const int64_t start = r.x;
    const uint64_t tile_hi = (uint64_t)blockIdx.x << 32;
    const int64_t vi = GATHER ? (int64_t)(blockIdx.x / (uint32_t)src.tiles_per_view) : 0;
    if (len <= 0) return;
    if (len == 1) {
        if (GATHER && threadIdx.x == 0) keys[start] = tile_hi | gathered_depth(src, vi, vals[start]);
        return;
    }
    if (threadIdx.x == 0) sh.ties = 0;
    if (len > SEG_CAP) {
        if (GATHER) {
            for (int e = threadIdx.x; e < len; e += SEG_THREADS)
                keys[start + e] = tile_hi | gathered_depth(src, vi, vals[start + e]);
            __syncthreads();
        }
        long_tile_sort(sh, keys, vals, spill, start, len, tile_hi);
        return;
    }
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int R = (len + SEG_THREADS - 1) / SEG_THREADS;   // items per lane, <= SEG_ITEMS
    uint32_t k[SEG_ITEMS], v[SEG_ITEMS];
    uint32_t lo = 0xFFFFFFFFu, hi = 0;
#pragma unroll
    for (int i = 0; i < SEG_ITEMS; ++i) {
        const int e = (w * R + i) * 64 + l;
        k[i] = 0;
        v[i] = 0;
        if (i < R && e < len) {
            v[i] = vals[start + e];
            k[i] = GATHER ? gathered_depth(src, vi, v[i]) : (uint32_t)keys[start + e];
            lo = k[i] < lo ? k[i] : lo;
            hi = k[i] > hi ? k[i] : hi;
        }
    }
    for (int i = t; i < 2 * SEG_WAVES * 256; i += SEG_THREADS) (&sh.cnt[0][0][0])[i] = 0;
    // The tile's keys lie in [kmin, kmax]: sorting k - kmin on its
    // bit_width(kmax - kmin) low bits gives the same order in fewer digit
    // bits (depths inside one tile span a narrow range).
    block_min_max(sh, lo, hi);
    const uint32_t kmin = lo, kmax = hi;
    const int bits = kmax == kmin ? 0 : 32 - __builtin_clz(kmax - kmin);
#pragma unroll
    for (int i = 0; i < SEG_ITEMS; ++i) k[i] -= kmin;
    // all keys equal (bits 0): every pair ties
    bool tie = bits == 0;
    int par = seg_lsd(sh, k, v, R, len, bits, 0, tie);
    // Equal depths: their pairs may have arrived in any order and must end
    // in Gaussian order.  A run of at most SEG_RUN equal keys is put in order
    // in place (each pair's place in its run = run start + the number of its
    // run's values below its own); a tile with a longer run is sorted again,
    // on the Gaussian index (minus its minimum) first and on the depth after.
    if (__syncthreads_or(tie)) {
#pragma unroll
        for (int i = 0; i < SEG_ITEMS; ++i) {
            const int e = (w * R + i) * 64 + l;
            if (i < R && e < len) {
                sh.key[e] = k[i];
                sh.val[e] = v[i];
            }
        }
        __syncthreads();
        // the counters are free now: they take the values of the runs in
        // their new order
        uint32_t *perm = &sh.cnt[0][0][0];
        uint32_t moved = 0;   // bit i: item i is in a run, its value at perm[e]
        bool long_run = false;
#pragma unroll
        for (int i = 0; i < SEG_ITEMS; ++i) {
            const int e = (w * R + i) * 64 + l;
            if (i < R && e < len) {
                const bool in_run = (e >= 1 && sh.key[e - 1] == k[i]) ||
                                    (e + 1 < len && sh.key[e + 1] == k[i]);
                if (in_run) {
                    int s0 = e, s1 = e;
                    while (s0 > 0 && e - s0 < SEG_RUN && sh.key[s0 - 1] == k[i]) --s0;
                    while (s1 + 1 < len && s1 - e < SEG_RUN && sh.key[s1 + 1] == k[i]) ++s1;
                    if (s1 - s0 + 1 > SEG_RUN) {
                        long_run = true;
                    } else {
                        int below = 0;
                        for (int j = s0; j <= s1; ++j) below += sh.val[j] < v[i] ? 1 : 0;
                        perm[s0 + below] = v[i];
                        moved |= 1u << i;
                    }
                }
            }
        }
        if (__syncthreads_or(long_run)) {
            for (int i = t; i < 2 * SEG_WAVES * 256; i += SEG_THREADS) (&sh.cnt[0][0][0])[i] = 0;
            uint32_t vlo = 0xFFFFFFFFu, vhi = 0;
#pragma unroll
            for (int i = 0; i < SEG_ITEMS; ++i) {
                if (i < R && (w * R + i) * 64 + l < len) {
                    vlo = v[i] < vlo ? v[i] : vlo;
                    vhi = v[i] > vhi ? v[i] : vhi;
                }
            }
            block_min_max(sh, vlo, vhi);
            const uint32_t vmin = vlo, vmax = vhi;
            const int vbits = vmax == vmin ? 0 : 32 - __builtin_clz(vmax - vmin);
#pragma unroll
            for (int i = 0; i < SEG_ITEMS; ++i) v[i] -= vmin;
            bool unused = false;
            par = seg_lsd(sh, v, k, R, len, vbits, par, unused);
#pragma unroll
            for (int i = 0; i < SEG_ITEMS; ++i) v[i] += vmin;
            seg_lsd(sh, k, v, R, len, bits, par, unused);
        } else {
#pragma unroll
            for (int i = 0; i < SEG_ITEMS; ++i)
                if ((moved >> i) & 1u) v[i] = perm[(w * R + i) * 64 + l];
        }
    }
#pragma unroll
    for (int i = 0; i < SEG_ITEMS; ++i) {
        const int e = (w * R + i) * 64 + l;
        if (i < R && e < len) {
            keys[start + e] = tile_hi | (k[i] + kmin);
            vals[start + e] = v[i];
        }
    }
}

// ---------------------------------------------------------------- counting strategy
// Binning without a sort on the tile bits.  The items of one view are cut
// into blocks of CT_THREADS * ipt; with hist[T][e] the number of pairs of
// block e in global tile T:
//   1. ct_count_kernel: each block counts its pairs per tile in LDS and
//      writes its column of hist, and the depth bits of its items into a
//      compact array (one word per item).
//   2. ct_scan_kernel: one wave per tile turns its row of hist into
//      exclusive prefixes and writes the row total.
//   3. ct_emit_kernel: each block scans the row totals of its view into the
//      tiles' first slots (adding the pairs of earlier views), walks its
//      pairs again and writes each one's value (the Gaussian) to its tile's
//      next slot (a per-tile LDS cursor started at tile start + hist
//      prefix); block 0 of each view writes that view's ranges, the first
//      block the pair count and the capacity flag.  Scattered stores bound
//      this kernel, so the keys are left to step 4.
//   4. tile_depth_sort_kernel reads each pair's depth bits from the compact
//      array, orders the tile by (depth bits, Gaussian) and writes the keys.
// Inside a tile the pairs of a block arrive in no fixed order; the depth
// sort resolves equal depths by the Gaussian index, so the output is the
// same (key, value) order as the other strategies, bit for bit.
//
// Launch: a 1-D grid of n_views * nbp blocks (nbp = blocks per view rounded
// up to a multiple of 8; the extra blocks hold no items).  Workgroups go to
// the 8 XCDs in turn, so block b is given column (b % 8) * (grid / 8) + b / 8:
// neighbouring columns of hist -- one cache line of a row -- are written and
// read by blocks of one XCD, whose L2 merges them.
constexpr int CT_THREADS = 512;
constexpr int CT_WAVES = CT_THREADS / 64;
constexpr int CT_MAX_TPV = 8192;         // tiles per view held as LDS counters
constexpr int CT_MAX_IPT = 128;          // items per thread and block
constexpr int64_t CT_TARGET_BLOCKS = 2048;
constexpr int CT_SCAN_LOADS = 16;
constexpr int CT_LOADS = 8;
constexpr int CT_XCDS = 8;

// (view, column) of block b of a grid of nb blocks (nb a multiple of 8)
__device__ __forceinline__ void ct_block(int64_t nbp, int64_t &vi, int64_t &e) {
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t c = (b % CT_XCDS) * (nb / CT_XCDS) + b / CT_XCDS;
    vi = c / nbp;
    e = c - vi * nbp;
}

// exclusive prefix sum over the block; *total gets the block's sum
__device__ __forceinline__ int64_t ct_block_scan(int64_t x, int64_t *total) {
    __shared__ int64_t ws[CT_WAVES];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    int64_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(incl, off, 64);
        if (l >= off) incl += y;
    }
    if (l == 63) ws[w] = incl;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < CT_WAVES; ++k) {
        if (k < w) off += ws[k];
        tot += ws[k];
    }
    __syncthreads();
    *total = tot;
    return off + incl - x;
}

// The tiles of one wave's items, one pair per lane and step.  The wave's
// pairs are numbered in lane order (item j's from the exclusive prefix of
// the counts over lanes < j on); at step C lane l takes pair C + l, owned by
// the highest lane whose first pair is at or before it (found as in
// emit_wave_pairs).  Every lane calls f(active, src, tile) at every step:
// src is the owning lane, tile the tile's index inside the view.
template <class F>
__device__ __forceinline__ void wave_tiles(bool valid, int32_t cnt, int4 r, int32_t tiles_x,
                                           int32_t *mark, F &&f) {
    const int lane = threadIdx.x & 63;
    valid = valid && cnt > 0;
    const uint32_t c = valid ? (uint32_t)cnt : 0u;
    const uint32_t incl = wave_incl_scan(c);
    const int32_t off = (int32_t)(incl - c);
    const int32_t total = __builtin_amdgcn_readlane((int)incl, 63);
    for (int32_t C = 0; C < total; C += 64) {
        const int32_t rel = off - C;
        if (valid && rel >= 0 && rel < 64) mark[rel] = lane;
        __builtin_amdgcn_wave_barrier();
        int own = mark[lane];
        __builtin_amdgcn_wave_barrier();
        mark[lane] = -1;
        const uint64_t before = __ballot(valid && rel < 0);
        const int carry = before ? 63 - __builtin_clzll(before) : -1;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(own, d, 64);
            if (lane >= d) own = max(own, y);
        }
        own = max(own, carry);
        const int src = own < 0 ? 0 : own;
        const int32_t ooff = __shfl(off, src, 64);
        const int x0 = __shfl(r.x, src, 64), y0 = __shfl(r.y, src, 64);
        const int w = __shfl(r.z, src, 64) - x0;
        const int32_t slot = C + lane;
        const bool active = own >= 0 && w > 0 && slot < total;
        int tile = 0;
        if (active) {
            const int local = slot - ooff;
            const int ty = local / w, tx = local - ty * w;
            tile = (y0 + ty) * tiles_x + (x0 + tx);
        }
        f(active, src, tile);
    }
}

__global__ void __launch_bounds__(CT_THREADS)
ct_count_kernel(const float4 *__restrict__ rec, const int32_t *__restrict__ touched,
                const int4 *__restrict__ rect, int64_t n, int32_t tiles_x, int32_t tpv,
                int32_t ipt, int64_t nbp, uint32_t *__restrict__ hist,
                uint32_t *__restrict__ dbits) {
    __shared__ uint32_t cnt[CT_MAX_TPV];
    __shared__ int32_t mark[CT_WAVES][64];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    int64_t vi, e;
    ct_block(nbp, vi, e);
    for (int i = t; i < tpv; i += CT_THREADS) cnt[i] = 0;
    mark[w][l] = -1;
    __syncthreads();
    for (int r = 0; r < ipt; ++r) {
        const int64_t g = (e * ipt + r) * CT_THREADS + t;
        int32_t c = 0;
        int4 rc = make_int4(0, 0, 0, 0);
        if (g < n) {
            const int64_t o = vi * n + g;
            c = touched[o];
            if (c > 0) {
                rc = rect[o];
                dbits[o] = __float_as_uint(rec[3 * o + 1].z);
            }
        }
        wave_tiles(c > 0, c, rc, tiles_x, mark[w], [&](bool active, int, int tile) {
            if (active && (unsigned)tile < (unsigned)tpv) atomicAdd(&cnt[tile], 1u);
        });
    }
    __syncthreads();
    for (int i = t; i < tpv; i += CT_THREADS) hist[(vi * tpv + i) * nbp + e] = cnt[i];
}

// grid ceil(n_tiles / CT_WAVES): wave w of block b scans tile CT_WAVES b + w
__global__ void __launch_bounds__(CT_THREADS)
ct_scan_kernel(uint32_t *__restrict__ hist, int64_t nbp, int64_t n_tiles,
               uint32_t *__restrict__ row_total) {
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int64_t T = (int64_t)blockIdx.x * CT_WAVES + w;
    if (T >= n_tiles) return;
    uint32_t running = 0;
    uint32_t *row = hist + T * nbp;
    for (int64_t c0 = 0; c0 < nbp; c0 += 64 * CT_SCAN_LOADS) {
        // clamped indexes: unconditional loads, all in flight together
        uint32_t x[CT_SCAN_LOADS];
#pragma unroll
        for (int i = 0; i < CT_SCAN_LOADS; ++i) {
            const int64_t idx = c0 + i * 64 + l;
            x[i] = row[idx < nbp ? idx : nbp - 1];
        }
#pragma unroll
        for (int i = 0; i < CT_SCAN_LOADS; ++i) {
            if (c0 + i * 64 + l >= nbp) x[i] = 0u;
            const uint32_t incl = wave_incl_scan(x[i]);
            const int64_t idx = c0 + i * 64 + l;
            if (idx < nbp) row[idx] = running + incl - x[i];
            running += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        }
    }
    if (l == 0) row_total[T] = running;
}

// the grid of ct_count_kernel
__global__ void __launch_bounds__(CT_THREADS)
ct_emit_kernel(const int32_t *__restrict__ touched, const int4 *__restrict__ rect, int64_t n,
               int32_t n_views, int32_t tiles_x, int32_t tpv, int32_t ipt, int64_t nbp,
               const uint32_t *__restrict__ hist, const uint32_t *__restrict__ row_total,
               int64_t capacity, int64_t *__restrict__ n_pairs, int32_t *__restrict__ overflow,
               uint32_t *__restrict__ vals, int2 *__restrict__ ranges) {
    __shared__ uint32_t next[CT_MAX_TPV];
    __shared__ int32_t mark[CT_WAVES][64];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    int64_t vi, e;
    ct_block(nbp, vi, e);
    const int64_t t0 = vi * tpv, n_tiles = (int64_t)n_views * tpv;
    // this view's tiles: first slots inside the view (next[]) and its total;
    // CT_LOADS loads per thread at a time, at clamped indexes so that all
    // are in flight together
    int64_t carry = 0;
    for (int i0 = 0; i0 < tpv; i0 += CT_THREADS * CT_LOADS) {
        const int b0 = i0 + t * CT_LOADS;   // CT_LOADS consecutive tiles per thread
        uint32_t x[CT_LOADS];
        int64_t sx = 0;
#pragma unroll
        for (int j = 0; j < CT_LOADS; ++j) x[j] = row_total[t0 + (b0 + j < tpv ? b0 + j : tpv - 1)];
#pragma unroll
        for (int j = 0; j < CT_LOADS; ++j) {
            if (b0 + j >= tpv) x[j] = 0u;
            sx += x[j];
        }
        int64_t tot;
        int64_t run = carry + ct_block_scan(sx, &tot);
#pragma unroll
        for (int j = 0; j < CT_LOADS; ++j) {
            if (b0 + j < tpv) next[b0 + j] = (uint32_t)run;
            run += x[j];
        }
        carry += tot;
    }
    // pairs of the earlier views and of all views
    int64_t before = 0, all = carry;
    if (n_views > 1) {
        int64_t sb = 0, sa = 0;
        for (int64_t i0 = 0; i0 < n_tiles; i0 += (int64_t)CT_THREADS * CT_LOADS) {
            uint32_t x[CT_LOADS];
#pragma unroll
            for (int j = 0; j < CT_LOADS; ++j) {
                const int64_t i = i0 + (int64_t)j * CT_THREADS + t;
                x[j] = row_total[i < n_tiles ? i : n_tiles - 1];
            }
#pragma unroll
            for (int j = 0; j < CT_LOADS; ++j) {
                const int64_t i = i0 + (int64_t)j * CT_THREADS + t;
                if (i < t0) sb += x[j];
                else if (i >= t0 + tpv && i < n_tiles) sa += x[j];
            }
        }
        int64_t tb, ta;
        ct_block_scan(sb, &tb);
        ct_block_scan(sa, &ta);
        before = tb;
        all = tb + carry + ta;
    }
    const bool over = all > capacity;
    if (vi == 0 && e == 0 && t == 0) {
        *n_pairs = all;
        *overflow = over ? 1 : 0;
    }
    __syncthreads();   // next[] complete
    if (e == 0) {
        // over capacity, every tile stays empty
        for (int i0 = 0; i0 < tpv; i0 += CT_THREADS * CT_LOADS) {
            uint32_t c[CT_LOADS];
#pragma unroll
            for (int j = 0; j < CT_LOADS; ++j) {
                const int i = i0 + j * CT_THREADS + t;
                c[j] = row_total[t0 + (i < tpv ? i : tpv - 1)];
            }
#pragma unroll
            for (int j = 0; j < CT_LOADS; ++j) {
                const int i = i0 + j * CT_THREADS + t;
                if (i < tpv) {
                    const int64_t s0 = before + next[i];
                    const bool empty = over || c[j] == 0 || s0 + c[j] > capacity;
                    ranges[t0 + i] = empty ? make_int2(0, 0) : make_int2((int)s0, (int)(s0 + c[j]));
                }
            }
        }
    }
    if (over) return;
    for (int i0 = 0; i0 < tpv; i0 += CT_THREADS * CT_LOADS) {
        uint32_t h[CT_LOADS];
#pragma unroll
        for (int j = 0; j < CT_LOADS; ++j) {
            const int i = i0 + j * CT_THREADS + t;
            h[j] = hist[(t0 + (i < tpv ? i : tpv - 1)) * nbp + e];
        }
#pragma unroll
        for (int j = 0; j < CT_LOADS; ++j) {
            const int i = i0 + j * CT_THREADS + t;
            if (i < tpv) next[i] += (uint32_t)before + h[j];
        }
    }
    mark[w][l] = -1;
    __syncthreads();
    for (int r = 0; r < ipt; ++r) {
        const int64_t g = (e * ipt + r) * CT_THREADS + t;
        int32_t c = 0;
        int4 rc = make_int4(0, 0, 0, 0);
        if (g < n) {
            const int64_t o = vi * n + g;
            c = touched[o];
            if (c > 0) rc = rect[o];
        }
        wave_tiles(c > 0, c, rc, tiles_x, mark[w], [&](bool active, int src, int tile) {
            const uint32_t og = (uint32_t)__shfl((int)(uint32_t)g, src, 64);
            if (active && (unsigned)tile < (unsigned)tpv) {
                const uint32_t pos = atomicAdd(&next[tile], 1u);
                if ((int64_t)pos < capacity) vals[pos] = og;
            }
        });
    }
}

// items per thread of the counting strategy: the smallest power of two that
// keeps the block count at most CT_TARGET_BLOCKS.  Each thread walks its
// rounds one after another, so large sets want many blocks; beyond about
// 2,048 the count columns and the emit blocks' passes over the row totals
// cost more than the shorter walks save (8 views x 500k Gaussians: 435,
// 371, 334 and 367 us of binning kernels at 320, 1,024, 2,048 and 4,096).
inline int ct_ipt(int64_t n, int32_t n_views) {
    int ipt = 1;
    while (ipt < CT_MAX_IPT &&
           (int64_t)n_views * ((n + (int64_t)CT_THREADS * ipt - 1) / ((int64_t)CT_THREADS * ipt)) >
               CT_TARGET_BLOCKS)
        ipt *= 2;
    return ipt;
}

struct CountPlan {
    int ipt = 0;
    int64_t nbp = 0;   // columns of hist per view (a multiple of CT_XCDS)
    uint32_t *hist = nullptr, *row_total = nullptr, *dbits = nullptr;
};

// the counting strategy's buffers inside `bytes` of workspace at ws (false
// if they do not fit with any block size)
bool ct_plan(void *ws, size_t bytes, int64_t n, int32_t n_views, int64_t n_tiles, CountPlan *P) {
    for (int ipt = ct_ipt(n, n_views); ipt <= CT_MAX_IPT; ipt *= 2) {
        const int64_t nbv = (n + (int64_t)CT_THREADS * ipt - 1) / ((int64_t)CT_THREADS * ipt);
        const int64_t nbp = ((nbv > 0 ? nbv : 1) + CT_XCDS - 1) / CT_XCDS * CT_XCDS;
        Carve c(ws, bytes);
        P->dbits = c.take<uint32_t>((size_t)(n * n_views > 0 ? n * n_views : 1));
        P->hist = c.take<uint32_t>((size_t)(n_tiles * nbp));
        P->row_total = c.take<uint32_t>((size_t)n_tiles);
        if (c.ok()) {
            P->ipt = ipt;
            P->nbp = nbp;
            return true;
        }
    }
    return false;
}

inline unsigned grid_for(int64_t count, int threads) {
    int64_t b = (count + threads - 1) / threads;
    return (unsigned)(b > 0 ? b : 1);
}

template <class K, int ITEMS>
int radix_passes(K *k0, uint32_t *v0, K *k1, uint32_t *v1, const int64_t *count_dev,
                 int64_t count_host, int64_t capacity, int bit_lo, int bit_hi, uint32_t *hist,
                 uint32_t *totals, const ItemSource *items, hipStream_t st) {
    constexpr int TILE = RS_THREADS * ITEMS;
    const int64_t nb_max = (capacity + TILE - 1) / TILE;
    K *src = k0, *dst = k1;
    uint32_t *vsrc = v0, *vdst = v1;
    // ceil(bits / 8) passes.  64-bit (tile) keys split their bits evenly over
    // the passes (e.g. 7 + 7 for 14 tile bits rather than 8 + 6): a pass with
    // fewer buckets writes longer runs per block, and the widest pass sets the
    // cost.  32-bit keys take 8-bit digits from bit_lo up.
    const int bits = bit_hi - bit_lo, passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift, nbits;
        if constexpr (sizeof(K) == 8) {
            shift = bit_lo + p * bits / passes;
            nbits = bit_lo + (p + 1) * bits / passes - shift;
        } else {
            shift = bit_lo + 8 * p;
            nbits = bit_hi - shift < 8 ? bit_hi - shift : 8;
        }
        if constexpr (sizeof(K) == 4) {
            if (shift == bit_lo && items) {
                rs_hist_items_kernel<ITEMS><<<(unsigned)nb_max, RS_THREADS, 0, st>>>(
                    *items, count_host, src, vsrc, hist);
            } else {
                rs_hist_kernel<K, ITEMS><<<(unsigned)nb_max, RS_THREADS, 0, st>>>(
                    src, count_dev, count_host, capacity, shift, nbits, hist);
            }
        } else {
            rs_hist_kernel<K, ITEMS><<<(unsigned)nb_max, RS_THREADS, 0, st>>>(
                src, count_dev, count_host, capacity, shift, nbits, hist);
        }
        rs_scan_kernel<<<256, 64, 0, st>>>(hist, totals, count_dev, count_host, capacity, TILE);
        rs_scatter_kernel<K, ITEMS><<<(unsigned)nb_max, RS_THREADS, 0, st>>>(
            src, vsrc, dst, vdst, count_dev, count_host, capacity, shift, nbits, hist, totals);
        GS4D_LAUNCH_CHECK("radix pass");
        K *tk = src; src = dst; dst = tk;
        uint32_t *tv = vsrc; vsrc = vdst; vdst = tv;
    }
    return GS4D_OK;
}

inline int rs_items(int64_t capacity) {
    return capacity <= RS_TINY_LIMIT ? RS_TINY_ITEMS
                                     : capacity <= RS_SMALL_LIMIT ? RS_SMALL_ITEMS : RS_LARGE_ITEMS;
}

inline int64_t rs_blocks(int64_t capacity) {
    const int64_t tile = (int64_t)RS_THREADS * rs_items(capacity);
    const int64_t nb = (capacity + tile - 1) / tile;
    return nb > 0 ? nb : 1;
}

template <class K>
int radix_sort_impl(K *k0, uint32_t *v0, K *k1, uint32_t *v1, const int64_t *count_dev,
                    int64_t count_host, int64_t capacity, int bit_lo, int bit_hi, void *ws,
                    hipStream_t st, int *result_in_alt, const ItemSource *items = nullptr) {
    const int passes = (bit_hi - bit_lo + 7) / 8;
    *result_in_alt = passes & 1;
    if (passes <= 0 || capacity <= 0) return GS4D_OK;
    Carve c(ws, ~size_t(0));
    uint32_t *hist = c.take<uint32_t>((size_t)rs_blocks(capacity) * 256);
    uint32_t *totals = c.take<uint32_t>(256);
    switch (rs_items(capacity)) {
    case RS_TINY_ITEMS:
        return radix_passes<K, RS_TINY_ITEMS>(k0, v0, k1, v1, count_dev, count_host, capacity,
                                               bit_lo, bit_hi, hist, totals, items, st);
    case RS_SMALL_ITEMS:
        return radix_passes<K, RS_SMALL_ITEMS>(k0, v0, k1, v1, count_dev, count_host, capacity,
                                                bit_lo, bit_hi, hist, totals, items, st);
    default:
        return radix_passes<K, RS_LARGE_ITEMS>(k0, v0, k1, v1, count_dev, count_host, capacity,
                                                bit_lo, bit_hi, hist, totals, items, st);
    }
}

}  // namespace

size_t radix_workspace_size(int64_t capacity) {
    // enough block histograms for any capacity up to this one (a smaller
    // capacity may use shorter blocks, hence more of them)
    int64_t nb = rs_blocks(capacity);
    for (const int64_t lim : {RS_TINY_LIMIT, RS_SMALL_LIMIT}) {
        const int64_t q = rs_blocks(capacity < lim ? capacity : lim);
        nb = q > nb ? q : nb;
    }
    Carve c(nullptr, 0);
    c.take<uint32_t>((size_t)nb * 256);
    c.take<uint32_t>(256);
    return c.used + 256;
}

int radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, const int64_t *count_dev,
                   int64_t count_host, int64_t capacity, int bit_lo, int bit_hi, void *ws,
                   hipStream_t st, int *result_in_alt) {
    return radix_sort_impl<uint64_t>(k0, v0, k1, v1, count_dev, count_host, capacity, bit_lo,
                                     bit_hi, ws, st, result_in_alt);
}

size_t scan_workspace_size(int64_t count) {
    // enough block sums for any count up to this one
    int64_t nb = sc_blocks(count);
    const int64_t q = sc_blocks(count < SC_SMALL_LIMIT ? count : SC_SMALL_LIMIT);
    nb = q > nb ? q : nb;
    return (size_t)(nb > 0 ? nb : 1) * sizeof(int64_t) + 256;
}

int exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t count, int64_t *total, void *ws,
                       hipStream_t st) {
    if (count <= 0) {
        return launch_fill<int64_t>(total, (int64_t)0, 1, st);
    }
    scan_launch(in, nullptr, out, count, total, static_cast<int64_t *>(ws), 0, nullptr, nullptr, st);
    GS4D_LAUNCH_CHECK("exclusive_scan");
    return GS4D_OK;
}

namespace {
// Pair offsets of the items (taken in `order` when given): exclusive scan of
// touched, the pair count and the capacity flag (count >= 1).
int pair_offsets(const int32_t *touched, const uint32_t *order, int32_t *offs, int64_t count,
                 int64_t *total, void *ws, int64_t capacity, int64_t *n_pairs, int32_t *overflow,
                 hipStream_t st) {
    scan_launch(touched, order, offs, count, total, static_cast<int64_t *>(ws), capacity, n_pairs,
                overflow, st);
    GS4D_LAUNCH_CHECK("pair_offsets");
    return GS4D_OK;
}
}  // namespace

namespace {
struct BinLayout {
    uint32_t *ik0, *iv0, *ik1, *iv1;   // presort: item keys / values, two buffers
    int32_t *offs;
    void *scan_ws;
    int64_t *total;
    uint64_t *pk;                       // alternate pair buffers
    uint32_t *pv;
    void *radix_ws;
    size_t ct_bytes;                    // bytes from ik0 on free for the counting strategy
};

// The counting strategy reuses the span from ik0 to the end of ct_room (the
// item buffers it does not need) for its per-block tile counts; ct_room
// alone holds them for the smallest grid (CT_XCDS columns per view) at the
// largest tile grid.
BinLayout carve_bin(void *ws, int64_t m, int32_t n_views, int64_t cap, size_t *used) {
    Carve c(ws, ~size_t(0));
    BinLayout L;
    const size_t mm = (size_t)(m > 0 ? m : 1);
    L.ik0 = c.take<uint32_t>(mm);
    L.iv0 = c.take<uint32_t>(mm);
    L.ik1 = c.take<uint32_t>(mm);
    L.iv1 = c.take<uint32_t>(mm);
    L.offs = c.take<int32_t>(mm);
    L.scan_ws = c.take<char>(scan_workspace_size(m));
    L.total = c.take<int64_t>(1);
    c.take<char>((size_t)(n_views > 0 ? n_views : 1) * CT_MAX_TPV * (4 * CT_XCDS + 4) + 1024);
    L.ct_bytes = c.used;
    L.pk = c.take<uint64_t>((size_t)(cap > 0 ? cap : 1));
    L.pv = c.take<uint32_t>((size_t)(cap > 0 ? cap : 1));
    L.radix_ws = c.take<char>(radix_workspace_size(m > cap ? m : cap));
    *used = c.used;
    return L;
}

// binning strategy (gs4d_set_bin_strategy); automatic: per tile while the
// pair capacity averages at most BIN_PER_TILE_MAX_MEAN pairs per tile
int g_bin_strategy = GS4D_BIN_AUTO;
constexpr int64_t BIN_PER_TILE_MAX_MEAN = 4096;

int tile_bits_for(int64_t n_tiles) {
    int b = 1;
    while (((int64_t)1 << b) < n_tiles) ++b;
    return b;
}
}  // namespace

}  // namespace gs4d

using namespace gs4d;

extern "C" int gs4d_set_bin_strategy(int32_t strategy) {
    GS4D_REQUIRE(strategy == GS4D_BIN_AUTO || strategy == GS4D_BIN_PER_TILE ||
                     strategy == GS4D_BIN_PRESORT || strategy == GS4D_BIN_COUNT,
                 "gs4d_set_bin_strategy: strategy must be 0, 1, 2 or 3");
    g_bin_strategy = strategy;
    return GS4D_OK;
}

extern "C" size_t gs4d_bin_sort_workspace_size(int64_t n, int32_t n_views, int64_t pair_capacity) {
    size_t used = 0;
    carve_bin(nullptr, n * (int64_t)(n_views > 0 ? n_views : 1), n_views, pair_capacity, &used);
    return used + 256;
}

extern "C" int gs4d_bin_sort(const float *rec, const int32_t *rect, const int32_t *touched,
                             int64_t n, const gs4d_view *views, int32_t n_views,
                             int64_t pair_capacity, uint64_t *keys, uint32_t *vals,
                             int32_t *ranges, int64_t *n_pairs, int32_t *overflow, void *ws,
                             size_t ws_bytes, void *stream) {
    ViewPack vp;
    GS4D_TRY(make_view_pack(views, n_views, &vp));
    GS4D_REQUIRE(n >= 0 && n <= (int64_t)0x7fffffff, "gs4d_bin_sort: n out of range");
    GS4D_REQUIRE((int64_t)n * n_views <= (int64_t)0xffffffffLL, "gs4d_bin_sort: n * n_views >= 2^32");
    GS4D_REQUIRE(pair_capacity >= 0 && pair_capacity < ((int64_t)1 << 31),
                 "gs4d_bin_sort: pair_capacity out of range");
    GS4D_REQUIRE(ranges && n_pairs && overflow, "gs4d_bin_sort: null output pointer");
    GS4D_REQUIRE(n == 0 || (rec && rect && touched), "gs4d_bin_sort: null input pointer");
    GS4D_REQUIRE(pair_capacity == 0 || (keys && vals), "gs4d_bin_sort: null pair buffer");
    const int64_t m = n * n_views;
    size_t need = gs4d_bin_sort_workspace_size(n, n_views, pair_capacity);
    GS4D_REQUIRE(ws != nullptr && ws_bytes >= need, "gs4d_bin_sort: workspace too small (%zu < %zu)",
                 ws_bytes, need);
    hipStream_t st = as_stream(stream);
    size_t used = 0;
    BinLayout L = carve_bin(ws, m, n_views, pair_capacity, &used);
    const int64_t n_tiles = (int64_t)vp.tiles_per_view * n_views;

    if (m == 0) {
        GS4D_TRY(launch_fill<int32_t>(ranges, 0, 2 * n_tiles, st));
        GS4D_TRY(launch_fill<int64_t>(n_pairs, (int64_t)0, 1, st));
        GS4D_TRY(launch_fill<int32_t>(overflow, 0, 1, st));
        return GS4D_OK;
    }
    const int tbits = tile_bits_for(n_tiles);
    const int tpasses = (tbits + 7) / 8;
    uint64_t *ek = (tpasses & 1) ? L.pk : keys;
    uint32_t *ev = (tpasses & 1) ? L.pv : vals;
    uint64_t *ok = (tpasses & 1) ? keys : L.pk;
    uint32_t *ov = (tpasses & 1) ? vals : L.pv;
    // Both strategies give the same pairs in the same order.  Per tile: fewer
    // launches, and cheap while tiles hold up to a few thousand pairs.
    // Presort: one device-wide sort of the items by depth, which wins when
    // tiles hold tens of thousands of pairs (then the per-tile sorts pass
    // through global memory).  Automatic choice from the pair capacity per
    // tile, known on the host.
    const bool per_tile = g_bin_strategy == GS4D_BIN_PER_TILE ||
                          g_bin_strategy == GS4D_BIN_COUNT ||
                          (g_bin_strategy == GS4D_BIN_AUTO &&
                           pair_capacity <= (int64_t)BIN_PER_TILE_MAX_MEAN * n_tiles);
    // Counting: fewest launches; where it applies (tiles per view held in
    // LDS) it is the per-tile default.
    CountPlan cp;
    if (per_tile && g_bin_strategy != GS4D_BIN_PER_TILE && vp.tiles_per_view <= CT_MAX_TPV &&
        ct_plan(ws, L.ct_bytes, n, n_views, n_tiles, &cp)) {
        const unsigned grid = (unsigned)(cp.nbp * n_views);
        ct_count_kernel<<<grid, CT_THREADS, 0, st>>>(
            reinterpret_cast<const float4 *>(rec), touched, reinterpret_cast<const int4 *>(rect), n,
            vp.tiles_x, vp.tiles_per_view, cp.ipt, cp.nbp, cp.hist, cp.dbits);
        ct_scan_kernel<<<grid_for(n_tiles, CT_WAVES), CT_THREADS, 0, st>>>(cp.hist, cp.nbp, n_tiles,
                                                                          cp.row_total);
        ct_emit_kernel<<<grid, CT_THREADS, 0, st>>>(
            touched, reinterpret_cast<const int4 *>(rect), n, n_views, vp.tiles_x,
            vp.tiles_per_view, cp.ipt, cp.nbp, cp.hist, cp.row_total, pair_capacity, n_pairs,
            overflow, vals, reinterpret_cast<int2 *>(ranges));
        GS4D_LAUNCH_CHECK("count binning");
        if (pair_capacity == 0) return GS4D_OK;
        tile_depth_sort_kernel<true><<<(unsigned)n_tiles, SEG_THREADS, 0, st>>>(
            keys, vals, reinterpret_cast<const int2 *>(ranges), L.pk,
            DepthSource{cp.dbits, n, vp.tiles_per_view});
        GS4D_LAUNCH_CHECK("tile depth sort");
        return GS4D_OK;
    }
    int alt = 0;
    if (per_tile) {
        // pair offsets of the items, pair count and capacity flag
        GS4D_TRY(pair_offsets(touched, nullptr, L.offs, m, L.total, L.scan_ws, pair_capacity,
                              n_pairs, overflow, st));
        if (pair_capacity == 0) return launch_fill<int32_t>(ranges, 0, 2 * n_tiles, st);
        // emit in item order (zeroing the ranges), stable sort on the tile bits only
        emit_kernel<<<dim3(grid_for(n, EMIT_THREADS), (unsigned)n_views), EMIT_THREADS, 0, st>>>(
            reinterpret_cast<const float4 *>(rec), touched, L.offs,
            reinterpret_cast<const int4 *>(rect), n, vp.tiles_x, vp.tiles_per_view, pair_capacity,
            ek, ev, ranges, 2 * n_tiles);
        GS4D_LAUNCH_CHECK("emit");
    } else {
        // items sorted by depth bits; the first pass builds their keys and
        // zeroes the ranges
        const ItemSource items{reinterpret_cast<const float4 *>(rec), touched, ranges,
                               2 * n_tiles};
        GS4D_TRY(radix_sort_impl<uint32_t>(L.ik0, L.iv0, L.ik1, L.iv1, nullptr, m, m, 0, 32,
                                           L.radix_ws, st, &alt, &items));
        const uint32_t *dkeys = alt ? L.ik1 : L.ik0;
        const uint32_t *order = alt ? L.iv1 : L.iv0;
        // offsets in depth order, pair count and capacity flag
        GS4D_TRY(pair_offsets(touched, order, L.offs, m, L.total, L.scan_ws, pair_capacity,
                              n_pairs, overflow, st));
        if (pair_capacity == 0) return GS4D_OK;
        // emit in depth order: inside a tile the pairs are then in (depth, Gaussian) order
        emit_depth_order_kernel<<<grid_for(m, EMIT_THREADS), EMIT_THREADS, 0, st>>>(
            dkeys, order, touched, L.offs, reinterpret_cast<const int4 *>(rect), m, n,
            vp.tiles_x, vp.tiles_per_view, pair_capacity, ek, ev);
        GS4D_LAUNCH_CHECK("emit (depth order)");
    }
    GS4D_TRY(radix_sort_u64(ek, ev, ok, ov, n_pairs, 0, pair_capacity, 32, 32 + tbits, L.radix_ws,
                            st, &alt));
    // tile ranges; the pair count is on the device: a grid of at most 2,048
    // blocks strides over it
    const unsigned rblocks = grid_for((pair_capacity + RG_UNROLL - 1) / RG_UNROLL, 256);
    const unsigned rgrid = rblocks < 65536u ? rblocks : 65536u;
    ranges_kernel<<<rgrid, 256, 0, st>>>(keys, n_pairs, pair_capacity, n_tiles,
                                         reinterpret_cast<int2 *>(ranges));
    GS4D_LAUNCH_CHECK("ranges");
    if (per_tile) {
        // depth order inside each tile (the pair buffer L.pk is free again)
        tile_depth_sort_kernel<false><<<(unsigned)n_tiles, SEG_THREADS, 0, st>>>(
            keys, vals, reinterpret_cast<const int2 *>(ranges), L.pk, DepthSource{});
        GS4D_LAUNCH_CHECK("tile depth sort");
    }
    return GS4D_OK;
}

// ---------------------------------------------------------------------------
// gs4d_bin_sort_noalloc: the same binning for callers that cannot allocate
// (graph capture, serving loops): its scratch memory is this fixed device
// array of the library, one per GPU, held until the process ends.  On the
// host the array's name is only a stand-in, never a device address: its
// address on each device is looked up once with hipGetSymbolAddress (with
// that device current) and kept; only that pointer is passed to kernels.
// Calls that overlap on one GPU share the array and race; the binning
// writes every scratch word it reads, so a call needs nothing cleared.
static __device__ __align__(256) char scratch[GS4D_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

int scratch_for_current_device(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        gs4d::set_error("gs4d_bin_sort_noalloc: hipGetDevice: %s", hipGetErrorString(e));
        return GS4D_ERR_HIP;
    }
    GS4D_REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, "gs4d_bin_sort_noalloc: device %d out of range",
                 dev);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            gs4d::set_error("gs4d_bin_sort_noalloc: hipGetSymbolAddress(scratch): %s",
                            hipGetErrorString(e));
            return GS4D_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GS4D_OK;
}
}  // namespace

extern "C" int gs4d_bin_sort_noalloc(const float *rec, const int32_t *rect, const int32_t *touched,
                                     int64_t n, const gs4d_view *views, int32_t n_views,
                                     int64_t pair_capacity, uint64_t *keys, uint32_t *vals,
                                     int32_t *ranges, int64_t *n_pairs, int32_t *overflow,
                                     void *stream) {
    GS4D_REQUIRE(n >= 0 && n <= (int64_t)0x7fffffff, "gs4d_bin_sort_noalloc: n out of range");
    GS4D_REQUIRE(n_views >= 1 && n_views <= GS4D_MAX_VIEWS, "gs4d_bin_sort_noalloc: n_views out of range");
    GS4D_REQUIRE(pair_capacity >= 0 && pair_capacity < ((int64_t)1 << 31),
                 "gs4d_bin_sort_noalloc: pair_capacity out of range");
    const size_t need = gs4d_bin_sort_workspace_size(n, n_views, pair_capacity);
    GS4D_REQUIRE(need <= GS4D_NOALLOC_SCRATCH_BYTES,
                 "gs4d_bin_sort_noalloc: this call needs %zu bytes of scratch, the library holds %zu "
                 "(use gs4d_bin_sort with a workspace)",
                 need, (size_t)GS4D_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    GS4D_TRY(scratch_for_current_device(&ws));
    return gs4d_bin_sort(rec, rect, touched, n, views, n_views, pair_capacity, keys, vals, ranges,
                         n_pairs, overflow, ws, GS4D_NOALLOC_SCRATCH_BYTES, stream);
}
