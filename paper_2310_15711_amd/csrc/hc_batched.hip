// Batched searching phase: many (pattern, text) pairs in one persistent launch.
//
// Work items are (text tile, group of patterns paired with that text). A
// workgroup stages the tile's bytes (plus the halo of the group's longest
// pattern) into LDS once and runs the searching phase of every pattern of the
// group over it; the next pattern's word vector F and bytes x are loaded into
// registers while the current one is searched. Items are dealt dynamically,
// most expensive first. Each (pair, tile) stores its count and the offset of
// its positions in a scratch buffer (reserved in large chunks, so few
// atomics); three small kernels then build the CSR offsets per pair and copy
// the positions into place, ascending per pair. The whole run is captured in a
// HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "hc_batch.h"
#include "hc_device.h"
#include "hc_internal.h"
#include "hc_runtime.h"

namespace hc {

struct BatchArgs {
    const TextView *texts;
    const BPat *pats;
    const uint8_t *xs;
    const uint8_t *Fs;             // table_bytes per pattern
    const BItem *items;
    uint32_t n_items;
    const uint32_t *glist;         // pairs of each text: pattern index << 0 in [0], pair index in [1]
    const uint64_t *pair_base;     // first (pair, tile) entry of each pair
    uint32_t *counts;              // per (pair, tile)
    uint32_t *toff;                // per (pair, tile): offset of its positions in `temp`
    int64_t *temp;
    uint64_t temp_cap;
    unsigned long long *ctl;       // [0] ticket, [1] scratch cursor, [2] overflow
    uint32_t tile, seg, table_bytes, max_m;
};

constexpr uint32_t kChunk = 8192;  // scratch positions reserved per atomic
constexpr uint64_t kMaxScratch = 0xFFFFFFFFull;   // scratch positions addressable by 32-bit offsets

template <typename WT, int Q, int K>
__device__ __forceinline__ TileResult batch_tile(const uint32_t *t32, uint32_t tb, const WT *F,
                                                 const uint32_t *x32, const PatternView &P,
                                                 uint32_t S, uint32_t seg, uint32_t *bm, Parked *park,
                                                 uint32_t *misc, uint32_t &it, uint32_t &round) {
    // ranges of `seg` starts per lane: here a long pattern's search overlaps
    // the loads of the group's next table, which it hides best when all
    // lanes take part
    return search_tile<Q, WT, K, false>(t32, tb, F, x32, P, S, seg, bm, park, misc, it, round);
}

template <typename WT, int K>
__device__ __forceinline__ TileResult batch_tile_q(uint32_t q, const uint32_t *t32, uint32_t tb,
                                                   const WT *F, const uint32_t *x32,
                                                   const PatternView &P, uint32_t S, uint32_t seg,
                                                   uint32_t *bm, Parked *park, uint32_t *misc,
                                                   uint32_t &it, uint32_t &round) {
    switch (q) {
        case 1: return batch_tile<WT, 1, K>(t32, tb, F, x32, P, S, seg, bm, park, misc, it, round);
        case 2: return batch_tile<WT, 2, K>(t32, tb, F, x32, P, S, seg, bm, park, misc, it, round);
        case 3: return batch_tile<WT, 3, K>(t32, tb, F, x32, P, S, seg, bm, park, misc, it, round);
        case 4: return batch_tile<WT, 4, K>(t32, tb, F, x32, P, S, seg, bm, park, misc, it, round);
        case 5: return batch_tile<WT, 5, K>(t32, tb, F, x32, P, S, seg, bm, park, misc, it, round);
        case 6: return batch_tile<WT, 6, K>(t32, tb, F, x32, P, S, seg, bm, park, misc, it, round);
        case 7: return batch_tile<WT, 7, K>(t32, tb, F, x32, P, S, seg, bm, park, misc, it, round);
        default: return batch_tile<WT, 8, K>(t32, tb, F, x32, P, S, seg, bm, park, misc, it, round);
    }
}

// Patterns without links (m < 2q): every window of the tile is tested at
// once (the dense schedule); the table is not read.
template <typename WT>
__device__ __forceinline__ TileResult batch_dense_q(uint32_t q, const uint32_t *t32, uint32_t tb, const WT *F,
                                                    const uint32_t *x32, const PatternView &P, uint32_t S,
                                                    uint32_t *bm, uint32_t *misc, uint32_t &it) {
    switch (q) {
        case 1: return dense_tile<1, WT, 0>(t32, tb, F, x32, P, S, bm, misc, it);
        case 2: return dense_tile<2, WT, 0>(t32, tb, F, x32, P, S, bm, misc, it);
        case 3: return dense_tile<3, WT, 0>(t32, tb, F, x32, P, S, bm, misc, it);
        case 4: return dense_tile<4, WT, 0>(t32, tb, F, x32, P, S, bm, misc, it);
        case 5: return dense_tile<5, WT, 0>(t32, tb, F, x32, P, S, bm, misc, it);
        case 6: return dense_tile<6, WT, 0>(t32, tb, F, x32, P, S, bm, misc, it);
        case 7: return dense_tile<7, WT, 0>(t32, tb, F, x32, P, S, bm, misc, it);
        default: return dense_tile<8, WT, 0>(t32, tb, F, x32, P, S, bm, misc, it);
    }
}

// Per-pattern table and bytes, staged through registers: 16 bytes per thread
// per step (patterns <= 4 KiB + padding). Only the first 8 KiB of a table
// travel in registers (more would cost the kernel a wavefront per SIMD); the
// rest of a larger table (up to 16 KiB) is copied when it is committed.
constexpr int kFStage = 2;
constexpr uint32_t kMaxBatchTable = 16384;
struct PatStage {
    u32x4 f[kFStage];
    u32x4 x[2];
};

__device__ __forceinline__ void pat_issue(const uint8_t *Fs, const uint8_t *xs, const BPat &bp,
                                          uint32_t p, uint32_t table_bytes, uint32_t x_bytes,
                                          PatStage &ps) {
    const global_u32x4 *f = (const global_u32x4 *)(Fs + uint64_t(p) * table_bytes);
    const uint32_t nf = table_bytes / 16u;
#pragma unroll
    for (int k = 0; k < kFStage; ++k) {
        const uint32_t c = k * kThreads + threadIdx.x;
        if (c < nf) ps.f[k] = f[c];
    }
    const global_u32x4 *x = (const global_u32x4 *)(xs + bp.x_off);
    const uint32_t nx = x_bytes / 16u;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const uint32_t c = k * kThreads + threadIdx.x;
        if (c < nx) ps.x[k] = x[c];
    }
}

__device__ __forceinline__ void pat_commit(const PatStage &ps, const uint8_t *Fs, uint32_t p, uint8_t *F,
                                           uint8_t *x8, uint32_t table_bytes, uint32_t x_bytes) {
    u32x4 *f = reinterpret_cast<u32x4 *>(F);
    const uint32_t nf = table_bytes / 16u;
#pragma unroll
    for (int k = 0; k < kFStage; ++k) {
        const uint32_t c = k * kThreads + threadIdx.x;
        if (c < nf) f[c] = ps.f[k];
    }
    const global_u32x4 *src = (const global_u32x4 *)(Fs + uint64_t(p) * table_bytes);
    for (uint32_t c = kFStage * kThreads + threadIdx.x; c < nf; c += kThreads) f[c] = src[c];
    u32x4 *x = reinterpret_cast<u32x4 *>(x8);
    const uint32_t nx = x_bytes / 16u;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const uint32_t c = k * kThreads + threadIdx.x;
        if (c < nx) x[c] = ps.x[k];
    }
}

template <typename WT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void hc_batch_kernel(BatchArgs A) {
    extern __shared__ __align__(16) uint8_t lds[];
    const LdsLayout L = lds_layout(A.tile, A.max_m, A.table_bytes, 0);
    uint8_t *t8 = lds + L.text_off;
    const uint32_t *t32 = reinterpret_cast<const uint32_t *>(t8);
    uint32_t *bm = reinterpret_cast<uint32_t *>(lds + L.bitmap_off);
    uint8_t *F8 = lds + L.table_off;
    const WT *F = reinterpret_cast<const WT *>(F8);
    uint8_t *x8 = lds + L.x_off;
    const uint32_t *x32 = reinterpret_cast<const uint32_t *>(x8);
    Parked *park = reinterpret_cast<Parked *>(lds + L.park_off);
    uint32_t *misc = reinterpret_cast<uint32_t *>(lds + L.misc_off);
    unsigned long long *misc64 = reinterpret_cast<unsigned long long *>(misc + 16);
    // misc: [0..3] scan, [4] first ticket, [8..11] search flags, [12..13] next
    // tickets; misc64[0] scratch cursor, [1] scratch left in the chunk, [2] offset

    const uint32_t tid = threadIdx.x;
    const uint32_t tile_words = A.tile / 32u;
    for (uint32_t i = tid; i < tile_words; i += kThreads) bm[i] = 0u;
    if (tid == 0) {
        misc[8] = misc[10] = misc[11] = 0u;
        misc64[0] = 0ull;
        misc64[1] = 0ull;
        misc[4] = uint32_t(atomicAdd(&A.ctl[0], 1ull));
    }
    __syncthreads();
    uint32_t it = 0, round = 0, k = 0;
    uint32_t item = misc[4];
    while (item < A.n_items) {
        const BItem W = A.items[item];
        // the next ticket travels while this item is searched (two slots: the
        // previous one may still be read by threads of this workgroup)
        if (tid == 0) misc[12 + (k & 1u)] = uint32_t(atomicAdd(&A.ctl[0], 1ull));
        const TextView tv = A.texts[W.text];
        const uint64_t n_t = tv.len;
        const uint64_t tile_lo = uint64_t(W.tile) * A.tile;
        // longest pattern of the group comes first
        const uint32_t span = A.pats[A.glist[2 * W.g0]].m;
        const uint64_t g1 = min<uint64_t>(tile_lo + A.tile + span - 1u, n_t);
        Stage<> st;
        const uint32_t tb = stage_issue(tv.ptr, tile_lo, g1, st);
        PatStage ps;
        {
            const uint32_t p = A.glist[2 * W.g0];
            pat_issue(A.Fs, A.xs, A.pats[p], p, A.table_bytes, L.x_bytes, ps);
        }
        lds_barrier();   // previous item finished with text, F and x
        stage_commit(st, t8);

        for (uint32_t gi = W.g0; gi < W.g1; ++gi) {
            const uint32_t p = A.glist[2 * gi], pair = A.glist[2 * gi + 1];
            const BPat bp = A.pats[p];
            pat_commit(ps, A.Fs, p, F8, x8, A.table_bytes, L.x_bytes);
            lds_barrier();
            if (gi + 1 < W.g1) {
                const uint32_t pn = A.glist[2 * (gi + 1)];
                pat_issue(A.Fs, A.xs, A.pats[pn], pn, A.table_bytes, L.x_bytes, ps);
            }
            const uint64_t starts = min<uint64_t>(n_t >= bp.m ? n_t - bp.m + 1u : 0u, tv.start_limit);
            if (tile_lo >= starts) {   // uniform: no window of this pattern starts here
                lds_barrier();
                continue;
            }
            const uint32_t S = uint32_t(min<uint64_t>(A.tile, starts - tile_lo));
            const PatternView P{bp.m, bp.q, bp.s, bp.mask, bp.hv, bp.w[0], bp.w[1], bp.w[2], bp.w[3]};
            const uint32_t shift = bp.m - bp.q + 1u;
            const TileResult R =
                bp.m < 2u * bp.q
                    ? batch_dense_q<WT>(bp.q, t32, tb, F, x32, P, S, bm, misc, it)
                    : shift <= 12u
                          ? batch_tile_q<WT, 4>(bp.q, t32, tb, F, x32, P, S, A.seg, bm, park, misc, it, round)
                          : batch_tile_q<WT, 1>(bp.q, t32, tb, F, x32, P, S, A.seg, bm, park, misc, it, round);
            const uint64_t entry = A.pair_base[pair] + W.tile;
            if (R.total == 0u) {
                if (tid == 0) A.counts[entry] = 0u;
                lds_barrier();   // F and x are replaced next
                continue;
            }
            if (tid == 0) {
                // reserve scratch for this (pair, tile) from the workgroup's chunk
                unsigned long long left = misc64[1], cur = misc64[0];
                if (left < R.total) {
                    const unsigned long long want = max<unsigned long long>(kChunk, R.total);
                    cur = atomicAdd(&A.ctl[1], want);
                    left = want;
                }
                misc64[2] = cur;
                misc64[0] = cur + R.total;
                misc64[1] = left - R.total;
                A.counts[entry] = R.total;
                if (cur + R.total > A.temp_cap) {
                    A.ctl[2] = 1ull;   // scratch too small: the host runs again with more
                    A.toff[entry] = 0xFFFFFFFFu;
                } else {
                    A.toff[entry] = uint32_t(cur);
                }
            }
            lds_barrier();
            const unsigned long long off = misc64[2];
            if (off + R.total <= A.temp_cap) {
                uint64_t idx = off + R.mine;
                for (uint32_t i = R.w0; i < R.w1; ++i) {
                    uint32_t b = bm[i];
                    while (b) {
                        const uint32_t bit = __builtin_ctz(b);
                        b &= b - 1u;
                        A.temp[idx++] = int64_t(tile_lo + i * 32u + bit);
                    }
                }
            }
            for (uint32_t i = R.w0; i < R.w1; ++i) bm[i] = 0u;
            lds_barrier();   // F and x are replaced next
        }
        item = misc[12 + (k & 1u)];
        ++k;
    }
}

// Total occurrences of each pair: one wavefront per pair.
__global__ __launch_bounds__(256) void hc_pair_totals(const uint64_t *pair_base, uint64_t n_pairs,
                                                      const uint32_t *counts, uint64_t *tot) {
    const uint64_t k = (uint64_t(blockIdx.x) * 256u + threadIdx.x) / kWave;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    if (k >= n_pairs) return;
    const uint64_t b = pair_base[k], e = pair_base[k + 1];
    uint64_t s = 0;
    for (uint64_t i = b + lane; i < e; i += kWave) s += counts[i];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += (uint64_t)__shfl_xor((long long)s, d, kWave);
    if (lane == 0) tot[k] = s;
}

// Exclusive scan of n uint64 values in three steps: per-block sums, a scan of
// the block sums by one workgroup, per-block scans with the block offsets.
constexpr uint32_t kScanItems = 16;   // values per thread and block step
constexpr uint32_t kScanBlock = 256u * kScanItems;

__device__ __forceinline__ uint64_t block_sum64(uint64_t v, uint64_t *lds8) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += (uint64_t)__shfl_xor((long long)v, d, kWave);
    const uint32_t wid = threadIdx.x / kWave;
    if ((threadIdx.x & 63u) == 0) lds8[wid] = v;
    __syncthreads();
    const uint64_t t = lds8[0] + lds8[1] + lds8[2] + lds8[3];
    __syncthreads();
    return t;
}

__device__ __forceinline__ uint64_t block_excl64(uint64_t v, uint64_t *lds8, uint64_t *total) {
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x / kWave;
    uint64_t incl = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t t = (uint64_t)__shfl_up((long long)incl, d, kWave);
        if (lane >= uint32_t(d)) incl += t;
    }
    if (lane == 63u) lds8[wid] = incl;
    __syncthreads();
    uint64_t before = 0, all = 0;
    for (uint32_t i = 0; i < 4; ++i) {
        if (i < wid) before += lds8[i];
        all += lds8[i];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

__global__ __launch_bounds__(256) void hc_scan_reduce(const uint64_t *in, uint64_t n, uint64_t *bsum) {
    __shared__ uint64_t lds8[4];
    const uint64_t base = uint64_t(blockIdx.x) * kScanBlock;
    uint64_t s = 0;
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint64_t i = base + uint64_t(k) * 256u + threadIdx.x;
        if (i < n) s += in[i];
    }
    const uint64_t t = block_sum64(s, lds8);
    if (threadIdx.x == 0) bsum[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void hc_scan_blocks(uint64_t *bsum, uint32_t nb, uint64_t *grand) {
    __shared__ uint64_t lds8[4];
    uint64_t carry = 0;
    for (uint32_t c = 0; c < nb; c += 256u) {
        const uint32_t i = c + threadIdx.x;
        const uint64_t v = i < nb ? bsum[i] : 0ull;
        uint64_t tot;
        const uint64_t ex = block_excl64(v, lds8, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *grand = carry;
}

__global__ __launch_bounds__(256) void hc_scan_apply(const uint64_t *in, uint64_t n, const uint64_t *bsum,
                                                     int64_t *out) {
    __shared__ uint64_t lds8[4];
    const uint64_t base = uint64_t(blockIdx.x) * kScanBlock;
    // each thread owns kScanItems consecutive values
    uint64_t v[kScanItems];
    uint64_t s = 0;
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint64_t i = base + uint64_t(threadIdx.x) * kScanItems + k;
        v[k] = i < n ? in[i] : 0ull;
        s += v[k];
    }
    uint64_t tot;
    uint64_t run = bsum[blockIdx.x] + block_excl64(s, lds8, &tot);
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint64_t i = base + uint64_t(threadIdx.x) * kScanItems + k;
        if (i < n) out[i] = int64_t(run);
        run += v[k];
    }
}

__global__ void hc_scan_total(const uint64_t *grand, int64_t *out_last) { *out_last = int64_t(*grand); }

// The same scan in one launch when one block holds every value (n <=
// kScanBlock): the exclusive prefix of each value and, after them, the total.
__global__ __launch_bounds__(256) void hc_scan_single(const uint64_t *in, uint64_t n, int64_t *out) {
    __shared__ uint64_t lds8[4];
    uint64_t v[kScanItems];
    uint64_t s = 0;
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint64_t i = uint64_t(threadIdx.x) * kScanItems + k;
        v[k] = i < n ? in[i] : 0ull;
        s += v[k];
    }
    uint64_t tot;
    uint64_t run = block_excl64(s, lds8, &tot);
    for (uint32_t k = 0; k < kScanItems; ++k) {
        const uint64_t i = uint64_t(threadIdx.x) * kScanItems + k;
        if (i < n) out[i] = int64_t(run);
        run += v[k];
    }
    if (threadIdx.x == 0) out[n] = int64_t(tot);
}

// Copies each pair's positions into place: one wavefront per pair walks the
// pair's tiles in order (64 at a time, prefix within the pair by a scan).
// Does nothing when the search ran out of scratch (ctl[2] set): some entries
// then have no positions stored, and the host runs the search again.
__global__ __launch_bounds__(256) void hc_pair_emit(const uint64_t *pair_base, uint64_t n_pairs,
                                                    const uint32_t *counts, const uint32_t *toff,
                                                    const int64_t *temp, const int64_t *pair_off,
                                                    int64_t *out, int64_t cap,
                                                    const unsigned long long *ctl) {
    const uint64_t k = (uint64_t(blockIdx.x) * 256u + threadIdx.x) / kWave;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    if (k >= n_pairs || ctl[2] != 0ull) return;
    const uint64_t b = pair_base[k], e = pair_base[k + 1];
    int64_t dst = pair_off[k];
    if (dst >= cap) return;
    for (uint64_t c0 = b; c0 < e; c0 += kWave) {
        const uint64_t i = c0 + lane;
        const uint32_t c = i < e ? counts[i] : 0u;
        // wavefront exclusive scan of c
        uint32_t incl = c;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)incl, d, kWave);
            if (lane >= uint32_t(d)) incl += t;
        }
        const uint32_t chunk_total = (uint32_t)__shfl((int)incl, 63, kWave);
        const int64_t mydst = dst + incl - c;
        uint64_t todo = __ballot(c != 0u);
        while (todo) {
            const int src_lane = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1ull;
            const uint32_t cc = (uint32_t)__shfl((int)c, src_lane, kWave);
            const uint32_t so = (uint32_t)__shfl((int)(i < e ? toff[min(i, e - 1)] : 0u), src_lane, kWave);
            const int64_t d0 = __shfl((long long)mydst, src_lane, kWave);
            if (so == 0xFFFFFFFFu) continue;   // no stored positions (see above)
            for (uint32_t j = lane; j < cc; j += kWave)
                if (d0 + j < cap) out[d0 + j] = temp[uint64_t(so) + j];
        }
        dst += chunk_total;
        if (dst >= cap) return;
    }
}

// Copies n staged patterns into their pool slots: entry i (stride
// table_bytes + x_stride + sizeof(BPat) bytes, all multiples of 16) holds a
// table, the padded pattern bytes and the descriptor of slot slots[i]. One
// workgroup per entry.
__global__ __launch_bounds__(256) void hc_scatter_patterns(const uint8_t *src, const uint32_t *slots, uint32_t n,
                                                           uint32_t table_bytes, uint32_t x_stride, uint8_t *Fpool,
                                                           uint8_t *xpool, BPat *pats) {
    const uint32_t i = blockIdx.x;
    if (i >= n) return;
    const uint32_t stride = table_bytes + x_stride + uint32_t(sizeof(BPat));
    const uint4 *e = reinterpret_cast<const uint4 *>(src + uint64_t(i) * stride);
    uint4 *f = reinterpret_cast<uint4 *>(Fpool + uint64_t(slots[i]) * table_bytes);
    uint4 *x = reinterpret_cast<uint4 *>(xpool + uint64_t(slots[i]) * x_stride);
    uint4 *d = reinterpret_cast<uint4 *>(pats + slots[i]);
    for (uint32_t k = threadIdx.x; k < table_bytes / 16u; k += blockDim.x) f[k] = e[k];
    for (uint32_t k = threadIdx.x; k < x_stride / 16u; k += blockDim.x) x[k] = e[table_bytes / 16u + k];
    for (uint32_t k = threadIdx.x; k < sizeof(BPat) / 16u; k += blockDim.x)
        d[k] = e[(table_bytes + x_stride) / 16u + k];
}

__global__ void hc_batch_reset(unsigned long long *ctl) {
    if (threadIdx.x < 4) ctl[threadIdx.x] = 0ull;
}


// ----------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------

DeviceBuf::~DeviceBuf() {
    if (p) (void)hipFree(p);
}

hc_status DeviceBuf::ensure(size_t b) {
    if (bytes >= b && p) return HC_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, std::max<size_t>(b, 16)) != hipSuccess) return HC_ENOMEM;
    bytes = std::max<size_t>(b, 16);
    return HC_OK;
}

hc_status DeviceBuf::upload(const void *src, size_t b, hipStream_t s) {
    if (ensure(b) != HC_OK) return HC_ENOMEM;
    if (b && hipMemcpyAsync(p, src, b, hipMemcpyHostToDevice, s) != hipSuccess) return HC_EHIP;
    return HC_OK;
}

template <typename WT>
static hc_status batch_occupancy(uint32_t lds, int *per_cu) {
    *per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, reinterpret_cast<const void *>(hc_batch_kernel<WT>),
                                                     kThreads, lds) != hipSuccess)
        return HC_EHIP;
    *per_cu = std::max(1, *per_cu);
    return HC_OK;
}

static std::mutex g_knobs_mu;
static BatchKnobs g_knobs;

BatchKnobs batch_knobs() {
    std::lock_guard<std::mutex> g(g_knobs_mu);
    return g_knobs;
}

void set_batch_knobs(const BatchKnobs *k) {
    std::lock_guard<std::mutex> g(g_knobs_mu);
    g_knobs = k ? *k : BatchKnobs{};
}

hc_status batch_shape(const hc_params *params, int &alpha, int &w, uint32_t &table_bytes, const BatchKnobs &k) {
    w = params && params->w ? params->w : k.w;
    alpha = params && params->alpha ? params->alpha : k.alpha;
    if ((w != 16 && w != 32) || alpha < 1 || alpha > alpha_max(w)) return HC_EINVAL;
    table_bytes = uint32_t((size_t(1) << alpha) * size_t(w / 8));
    table_bytes = std::max<uint32_t>(16, (table_bytes + 15u) & ~15u);
    if (table_bytes > kMaxBatchTable) return HC_EINVAL;
    return HC_OK;
}

hc_status batch_geometry(BatchDev &D, uint32_t max_m, uint32_t table_bytes, uint32_t w, const BatchKnobs &k) {
    const DeviceInfo &di = device_info();
    if (!di.ok) return HC_EHIP;
    D.max_m = std::max<uint32_t>(max_m, 1);
    D.table_bytes = table_bytes;
    D.w = w;
    D.group = std::max<uint32_t>(1, k.group);
    // tiles of the knobs' size, or as large as LDS and the staging allow
    D.seg = std::max<uint32_t>(8, std::min<uint32_t>(k.seg, 100));
    D.tile = kThreads * D.seg;
    LdsLayout L = lds_layout(D.tile, D.max_m, D.table_bytes, 0);
    while ((L.total > di.max_lds_per_block || D.tile + D.max_m - 1u > stage_limit(kThreads)) && D.seg > 8) {
        D.seg -= 4;
        D.tile = kThreads * D.seg;
        L = lds_layout(D.tile, D.max_m, D.table_bytes, 0);
    }
    if (L.total > di.max_lds_per_block) return HC_EINVAL;
    D.lds = L.total;
    int per_cu = 1;
    hc_status st = w == 16 ? batch_occupancy<uint16_t>(D.lds, &per_cu) : batch_occupancy<uint32_t>(D.lds, &per_cu);
    if (st != HC_OK) return st;
    if (k.wg_per_cu > 0) per_cu = std::min<int>(per_cu, int(k.wg_per_cu));
    D.max_grid = uint32_t(di.cus) * uint32_t(per_cu);
    return HC_OK;
}

hc_status pack_one(const uint8_t *x, int64_t m, int q_req, int alpha, int w, uint32_t table_bytes, BPat &bp,
                   uint8_t *F_out) {
    if (m < 1 || m > kMaxM) return HC_EINVAL;
    int q = q_req, a = alpha, ww = w;
    default_params(m, distinct_bytes(x, m), q, a, ww);
    q = int(std::min<int64_t>(q, m));
    if (validate_params(m, q, alpha, w) != HC_OK) return HC_EINVAL;
    PatternData pd;
    build_link_table(x, m, q, alpha, w, pd);
    std::vector<uint8_t> packed = pack_table(pd);
    if (packed.size() > table_bytes) return HC_EINVAL;
    std::memset(F_out, 0, table_bytes);
    std::memcpy(F_out, packed.data(), packed.size());
    bp = BPat{uint32_t(m), uint32_t(q), uint32_t(pd.s), pd.mask, pd.hv, 0, 0, 0, {}};
    byte_weights(bp.q, bp.s, bp.w);
    return HC_OK;
}

hc_status pack_desc(const uint8_t *x, int64_t m, int q_req, int alpha, int w, BPat &bp) {
    if (m < 1 || m > kMaxM) return HC_EINVAL;
    int q = q_req, a = alpha, ww = w;
    default_params(m, distinct_bytes(x, m), q, a, ww);
    q = int(std::min<int64_t>(q, m));
    if (validate_params(m, q, alpha, w) != HC_OK) return HC_EINVAL;
    const uint32_t s = uint32_t(alpha / q), mask = uint32_t((uint64_t(1) << alpha) - 1u);
    // H_v: hash (eq. (3)) of the q-gram at (m - q) mod q
    const uint8_t *u = x + (m - q) % q;
    uint32_t v = 0;
    for (int k = q - 1; k >= 0; --k) v = (v << s) + u[k];
    bp = BPat{uint32_t(m), uint32_t(q), s, mask, v & mask, 0, 0, 0, {}};
    byte_weights(bp.q, bp.s, bp.w);
    return HC_OK;
}

hc_status pack_patterns(const uint8_t *pat, const int64_t *pat_off, int32_t np, const hc_params *params,
                        int alpha, int w, uint32_t table_bytes, std::vector<BPat> &bp, std::vector<uint8_t> &Fh,
                        std::vector<uint8_t> &Xh, uint32_t &max_m, bool host_tables) {
    bp.assign(size_t(std::max(np, 1)), BPat{});
    Fh.assign(host_tables ? size_t(std::max(np, 1)) * table_bytes : 0, 0);
    std::vector<uint32_t> xoff(size_t(np) + 1, 0);
    int64_t mmax = 1;
    for (int32_t i = 0; i < np; ++i) {
        const int64_t m = pat_off[i + 1] - pat_off[i];
        if (m < 1 || m > kMaxM) return HC_EINVAL;
        xoff[i + 1] = xoff[i] + uint32_t(((m + 15) & ~int64_t(15)) + 32);
        mmax = std::max(mmax, m);
    }
    // every pattern's bytes are read as a block of the longest pattern's size
    Xh.assign(xoff[np] + size_t((mmax + 15) & ~int64_t(15)) + 64, 0);
    max_m = uint32_t(mmax);
    for (int32_t i = 0; i < np; ++i) {
        const uint8_t *x = pat + pat_off[i];
        const int64_t m = pat_off[i + 1] - pat_off[i];
        hc_status st = host_tables ? pack_one(x, m, params ? params->q : 0, alpha, w, table_bytes, bp[i],
                                              Fh.data() + size_t(i) * table_bytes)
                                   : pack_desc(x, m, params ? params->q : 0, alpha, w, bp[i]);
        if (st != HC_OK) return st;
        bp[i].x_off = xoff[i];
        std::memcpy(Xh.data() + xoff[i], x, size_t(m));
    }
    return HC_OK;
}

void batch_build(BatchHost &H, const std::vector<std::pair<uint32_t, uint32_t>> &pairs, uint32_t tile,
                 uint32_t group) {
    const size_t nt = H.views.size();
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> by_text(std::max<size_t>(nt, 1));
    H.pair_base.assign(pairs.size() + 1, 0);
    for (size_t k = 0; k < pairs.size(); ++k) {
        const uint32_t p = pairs[k].first, t = pairs[k].second;
        by_text[t].push_back({p, uint32_t(k)});
        const uint64_t n_t = H.views[t].len, m = H.pats[p].m;
        const uint64_t starts = std::min<uint64_t>(n_t >= m ? n_t - m + 1 : 0, H.views[t].start_limit);
        H.pair_base[k + 1] = H.pair_base[k] + (starts + tile - 1) / tile;
    }
    // pairs grouped by text, longest pattern first; items dealt most expensive first
    H.glist.clear();
    struct ItemCost {
        double cost;
        BItem it;
    };
    std::vector<ItemCost> items;
    for (size_t t = 0; t < nt; ++t) {
        auto &v = by_text[t];
        std::sort(v.begin(), v.end(),
                  [&](const std::pair<uint32_t, uint32_t> &a, const std::pair<uint32_t, uint32_t> &c) {
                      return H.pats[a.first].m > H.pats[c.first].m ||
                             (H.pats[a.first].m == H.pats[c.first].m && a.second < c.second);
                  });
        const uint64_t n_t = std::min<uint64_t>(H.views[t].len, H.views[t].start_limit);
        const uint32_t tiles = uint32_t((n_t + tile - 1) / tile);
        for (size_t g = 0; g < v.size(); g += group) {
            const uint32_t g0 = uint32_t(H.glist.size() / 2);
            double per_byte = 0;
            for (size_t j = g; j < std::min(v.size(), g + group); ++j) {
                H.glist.push_back(v[j].first);
                H.glist.push_back(v[j].second);
                const BPat &q = H.pats[v[j].first];
                per_byte += 1.0 / double(q.m - q.q + 1) + 0.02;
            }
            const uint32_t g1 = uint32_t(H.glist.size() / 2);
            for (uint32_t tl = 0; tl < tiles; ++tl) {
                const double bytes = double(std::min<uint64_t>(tile, n_t - uint64_t(tl) * tile));
                items.push_back({bytes * per_byte, BItem{uint32_t(t), tl, g0, g1}});
            }
        }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const ItemCost &a, const ItemCost &c) { return a.cost > c.cost; });
    H.items.resize(items.size());
    for (size_t i = 0; i < items.size(); ++i) H.items[i] = items[i].it;
}

hc_status batch_check(const BatchHost &H, const BatchDev &D) {
    const size_t np = H.pats.size(), nv = H.views.size(), n_pairs = H.pair_base.size() - 1;
    if (H.pair_base.empty() || H.glist.size() % 2) return HC_EINVAL;
    const uint64_t x_bytes = lds_layout(D.tile, D.max_m, D.table_bytes, 0).x_bytes;
    std::vector<uint8_t> seen(np, 0);
    for (size_t g = 0; g < H.glist.size(); g += 2) {
        const uint32_t p = H.glist[g], k = H.glist[g + 1];
        if (p >= np || k >= n_pairs) return HC_EINVAL;
        if (seen[p]) continue;
        seen[p] = 1;
        const BPat &b = H.pats[p];
        if (b.m < 1 || b.m > D.max_m || b.q < 1 || b.q > uint32_t(kMaxQ) || b.q > b.m) return HC_EINVAL;
        if ((uint64_t(p) + 1) * D.table_bytes > D.Fs_bytes) return HC_EINVAL;
        if (b.x_off % 16u || uint64_t(b.x_off) + x_bytes > D.xs_bytes) return HC_EINVAL;
    }
    for (const BItem &it : H.items) {
        if (it.text >= nv || it.g0 >= it.g1 || uint64_t(it.g1) * 2 > H.glist.size()) return HC_EINVAL;
        const TextView &v = H.views[it.text];
        if (!v.ptr || uint64_t(it.tile) * D.tile >= std::min(v.len, v.start_limit)) return HC_EINVAL;
        for (uint32_t g = it.g0; g < it.g1; ++g)
            if (H.glist[2 * g + 1] >= n_pairs) return HC_EINVAL;
        // the group's first pattern is its longest (its halo is staged)
        for (uint32_t g = it.g0 + 1; g < it.g1; ++g)
            if (H.pats[H.glist[2 * g]].m > H.pats[H.glist[2 * it.g0]].m) return HC_EINVAL;
    }
    return HC_OK;
}

hc_status batch_upload(const BatchHost &H, BatchDev &D, hipStream_t s) {
    hc_status st = batch_check(H, D);
    if (st != HC_OK) return st;
    D.n_pairs = uint32_t(H.pair_base.size() - 1);
    D.n_items = uint32_t(H.items.size());
    D.n_entries = H.pair_base.back();
    if ((st = D.views.upload(H.views.data(), H.views.size() * sizeof(TextView), s)) != HC_OK) return st;
    if (!D.pats_dev && (st = D.pats.upload(H.pats.data(), H.pats.size() * sizeof(BPat), s)) != HC_OK) return st;
    if ((st = D.items.upload(H.items.data(), H.items.size() * sizeof(BItem), s)) != HC_OK) return st;
    if ((st = D.glist.upload(H.glist.data(), H.glist.size() * 4, s)) != HC_OK) return st;
    if ((st = D.pair_base.upload(H.pair_base.data(), H.pair_base.size() * 8, s)) != HC_OK) return st;
    if (D.counts.ensure(D.n_entries * 4) != HC_OK || D.toff.ensure(D.n_entries * 4) != HC_OK ||
        D.ctl.ensure(64) != HC_OK || D.tot.ensure(size_t(D.n_pairs) * 8) != HC_OK || D.grand.ensure(8) != HC_OK)
        return HC_ENOMEM;
    D.nb = uint32_t((uint64_t(D.n_pairs) + kScanBlock - 1) / kScanBlock);
    if (D.bsum.ensure(size_t(std::max<uint32_t>(D.nb, 1)) * 8) != HC_OK) return HC_ENOMEM;
    if (D.scratch_cap == 0) D.scratch_cap = 1u << 23;   // positions; grown when a run needs more
    if (D.temp.ensure(D.scratch_cap * 8) != HC_OK) return HC_ENOMEM;
    D.grid = std::max<uint32_t>(1, std::min<uint32_t>(D.n_items, D.max_grid));
    return HC_OK;
}

hc_status batch_enqueue(BatchDev &D, int64_t *d_pos, int64_t cap, int64_t *d_pair_off, hipStream_t s) {
    // every buffer the kernels read must be in place
    const BPat *pats = D.pats_dev ? D.pats_dev : D.pats.as<BPat>();
    if (D.n_items > 0 && (!D.Fs || !D.xs || !D.views.p || !pats || !D.items.p || !D.glist.p))
        return HC_EINVAL;
    if (!D.ctl.p || !D.pair_base.p || !D.temp.p || (D.n_pairs > 0 && (!D.tot.p || !D.counts.p || !D.toff.p)))
        return HC_EINVAL;
    hipLaunchKernelGGL(hc_batch_reset, dim3(1), dim3(64), 0, s, D.ctl.as<unsigned long long>());
    BatchArgs A;
    A.texts = D.views.as<TextView>();
    A.pats = pats;
    A.xs = D.xs;
    A.Fs = D.Fs;
    A.items = D.items.as<BItem>();
    A.n_items = D.n_items;
    A.glist = D.glist.as<uint32_t>();
    A.pair_base = D.pair_base.as<uint64_t>();
    A.counts = D.counts.as<uint32_t>();
    A.toff = D.toff.as<uint32_t>();
    A.temp = D.temp.as<int64_t>();
    A.temp_cap = D.scratch_cap;
    A.ctl = D.ctl.as<unsigned long long>();
    A.tile = D.tile;
    A.seg = D.seg;
    A.table_bytes = D.table_bytes;
    A.max_m = D.max_m;
    if (D.n_items > 0) {
        if (D.w == 16)
            hipLaunchKernelGGL(hc_batch_kernel<uint16_t>, dim3(D.grid), dim3(kThreads), D.lds, s, A);
        else
            hipLaunchKernelGGL(hc_batch_kernel<uint32_t>, dim3(D.grid), dim3(kThreads), D.lds, s, A);
    }
    const uint32_t pgrid = uint32_t((uint64_t(D.n_pairs) * kWave + 255u) / 256u);
    if (D.n_pairs > 0)
        hipLaunchKernelGGL(hc_pair_totals, dim3(pgrid), dim3(256), 0, s, D.pair_base.as<uint64_t>(),
                           uint64_t(D.n_pairs), D.counts.as<uint32_t>(), D.tot.as<uint64_t>());
    if (uint64_t(D.n_pairs) <= kScanBlock) {
        // one block holds every total: one launch instead of four
        hipLaunchKernelGGL(hc_scan_single, dim3(1), dim3(256), 0, s, D.tot.as<uint64_t>(), uint64_t(D.n_pairs),
                           d_pair_off);
    } else {
        hipLaunchKernelGGL(hc_scan_reduce, dim3(D.nb), dim3(256), 0, s, D.tot.as<uint64_t>(),
                           uint64_t(D.n_pairs), D.bsum.as<uint64_t>());
        hipLaunchKernelGGL(hc_scan_blocks, dim3(1), dim3(256), 0, s, D.bsum.as<uint64_t>(), D.nb,
                           D.grand.as<uint64_t>());
        hipLaunchKernelGGL(hc_scan_apply, dim3(D.nb), dim3(256), 0, s, D.tot.as<uint64_t>(), uint64_t(D.n_pairs),
                           D.bsum.as<uint64_t>(), d_pair_off);
        hipLaunchKernelGGL(hc_scan_total, dim3(1), dim3(1), 0, s, D.grand.as<uint64_t>(), d_pair_off + D.n_pairs);
    }
    if (D.n_pairs > 0 && cap > 0)
        hipLaunchKernelGGL(hc_pair_emit, dim3(pgrid), dim3(256), 0, s, D.pair_base.as<uint64_t>(),
                           uint64_t(D.n_pairs), D.counts.as<uint32_t>(), D.toff.as<uint32_t>(),
                           D.temp.as<int64_t>(), d_pair_off, d_pos, cap, D.ctl.as<unsigned long long>());
    D.last_error = hipGetLastError();
    return D.last_error == hipSuccess ? HC_OK : HC_EHIP;
}

hc_status scatter_patterns(const uint8_t *d_src, const uint32_t *d_slots, uint32_t n, uint32_t table_bytes,
                           uint32_t x_stride, uint8_t *Fpool, uint8_t *xpool, BPat *pats, hipStream_t s) {
    if (n == 0) return HC_OK;
    if (table_bytes % 16u || x_stride % 16u || sizeof(BPat) % 16u) return HC_EINVAL;
    hipLaunchKernelGGL(hc_scatter_patterns, dim3(n), dim3(256), 0, s, d_src, d_slots, n, table_bytes, x_stride,
                       Fpool, xpool, pats);
    return hipGetLastError() == hipSuccess ? HC_OK : HC_EHIP;
}

hc_status batch_emit(BatchDev &D, int64_t *d_pos, int64_t cap, const int64_t *d_pair_off, hipStream_t s) {
    if (D.n_pairs == 0 || cap <= 0) return HC_OK;
    const uint32_t pgrid = uint32_t((uint64_t(D.n_pairs) * kWave + 255u) / 256u);
    hipLaunchKernelGGL(hc_pair_emit, dim3(pgrid), dim3(256), 0, s, D.pair_base.as<uint64_t>(),
                       uint64_t(D.n_pairs), D.counts.as<uint32_t>(), D.toff.as<uint32_t>(),
                       D.temp.as<int64_t>(), d_pair_off, d_pos, cap, D.ctl.as<unsigned long long>());
    return hipGetLastError() == hipSuccess ? HC_OK : HC_EHIP;
}

hc_status batch_grow_scratch(BatchDev &D, uint64_t reserved, uint64_t total) {
    // A workgroup reserves a new chunk of max(kChunk, c) when the c positions
    // of a (pair, tile) do not fit in what is left of its chunk; that rest
    // (< c) is abandoned. So the abandoned rests sum to at most `total`, and
    // every workgroup ends with at most one chunk partly used: a run never
    // reserves more than 2 * total + grid * kChunk.
    const uint64_t need = std::max<uint64_t>(reserved, 2 * total + uint64_t(D.grid + 16u) * kChunk);
    // scratch offsets are stored as 32-bit values (0xFFFFFFFF marks an entry
    // that did not fit): a capacity below 2^32 - 1 keeps every stored offset
    // exact
    if (need >= kMaxScratch) return HC_ENOMEM;
    if (D.temp.ensure(need * 8) != HC_OK) return HC_ENOMEM;
    D.scratch_cap = need;
    return HC_OK;
}

}  // namespace hc

using namespace hc;

struct hc_batch_plan {
    BatchDev D;
    DeviceBuf Fpool, xpool;
    // graph for (d_pos, cap, d_pair_off, stream)
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int64_t *g_pos = nullptr, *g_off = nullptr;
    int64_t g_cap = -1;
    hipStream_t g_stream = nullptr;
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~hc_batch_plan() { drop_graph(); }
};

extern "C" {

hc_status hc_batch_plan_create(const hc_batch *b, const hc_params *params, hc_batch_plan **out) {
    return hc::plan_create(b, params, hc::batch_knobs(), out);
}

}  // extern "C"

hc_status hc::plan_create(const hc_batch *b, const hc_params *params, const BatchKnobs &knobs,
                          hc_batch_plan **out) {
    if (!out) return HC_EINVAL;
    *out = nullptr;
    if (!b || b->n_pairs < 0 || b->n_texts < 0 || b->n_pats < 0) return HC_EINVAL;
    if (b->n_pairs > 0 && (!b->pair_pat || !b->pair_text || !b->text_off || !b->pat_off || !b->pat ||
                           !b->d_text))
        return HC_EINVAL;
    if (b->n_pairs > int64_t(0x7FFFFFFF)) return HC_EINVAL;
    if (!device_info().ok) return HC_EHIP;
    for (int32_t t = 0; t < b->n_texts; ++t) {
        if (b->text_off[t + 1] < b->text_off[t]) return HC_EINVAL;
        if (b->text_off[t + 1] - b->text_off[t] > int64_t(0xFFFFFFFFll)) return HC_EINVAL;
    }
    for (int64_t k = 0; k < b->n_pairs; ++k)
        if (b->pair_pat[k] < 0 || b->pair_pat[k] >= b->n_pats || b->pair_text[k] < 0 ||
            b->pair_text[k] >= b->n_texts)
            return HC_EINVAL;
    std::unique_ptr<hc_batch_plan> P(new (std::nothrow) hc_batch_plan());
    if (!P) return HC_ENOMEM;
    int alpha = 0, w = 0;
    uint32_t table_bytes = 0;
    hc_status st = batch_shape(params, alpha, w, table_bytes, knobs);
    if (st != HC_OK) return st;
    // common table shape for the batch; q per pattern
    BatchHost H;
    std::vector<uint8_t> Fh, Xh;
    uint32_t max_m = 1;
    if ((st = pack_patterns(b->pat, b->pat_off, b->n_pats, params, alpha, w, table_bytes, H.pats, Fh, Xh,
                            max_m, false)) != HC_OK)
        return st;
    if ((st = batch_geometry(P->D, max_m, table_bytes, uint32_t(w), knobs)) != HC_OK) return st;
    H.views.resize(size_t(b->n_texts));
    for (int32_t t = 0; t < b->n_texts; ++t) {
        const uint64_t len = uint64_t(b->text_off[t + 1] - b->text_off[t]);
        H.views[t] = TextView{b->d_text + b->text_off[t], len, len};
    }
    std::vector<std::pair<uint32_t, uint32_t>> pairs(size_t(b->n_pairs));
    for (int64_t k = 0; k < b->n_pairs; ++k) pairs[k] = {uint32_t(b->pair_pat[k]), uint32_t(b->pair_text[k])};
    batch_build(H, pairs, P->D.tile, P->D.group);
    hipStream_t s = nullptr;
    if ((st = P->xpool.upload(Xh.data(), Xh.size(), s)) != HC_OK) return st;
    // the word vectors are built on the device from the uploaded pattern bytes
    if (P->Fpool.ensure(size_t(std::max(b->n_pats, 1)) * table_bytes) != HC_OK) return HC_ENOMEM;
    std::vector<uint32_t> desc(size_t(b->n_pats) * 3);
    for (int32_t i = 0; i < b->n_pats; ++i) {
        desc[3 * i] = H.pats[i].x_off;
        desc[3 * i + 1] = H.pats[i].m;
        desc[3 * i + 2] = H.pats[i].q;
    }
    DeviceBuf d_desc;
    if ((st = d_desc.upload(desc.data(), desc.size() * 4, s)) != HC_OK) return st;
    if ((st = device_preprocess(P->xpool.as<uint8_t>(), d_desc.as<uint32_t>(), uint32_t(b->n_pats), alpha, w,
                                table_bytes, P->Fpool.as<uint8_t>(), nullptr, s)) != HC_OK)
        return st;
    P->D.Fs = P->Fpool.as<uint8_t>();
    P->D.xs = P->xpool.as<uint8_t>();
    P->D.Fs_bytes = P->Fpool.bytes;
    P->D.xs_bytes = P->xpool.bytes;
    if ((st = batch_upload(H, P->D, s)) != HC_OK) return st;
    // the host vectors above go out of scope: wait for the copies
    if (hipStreamSynchronize(s) != hipSuccess) return HC_EHIP;
    *out = P.release();
    return HC_OK;
}

extern "C" {

void hc_batch_plan_free(hc_batch_plan *p) { delete p; }

hc_status hc_batch_plan_run(hc_batch_plan *P, int64_t *d_pos, int64_t cap, int64_t *d_pair_off, int64_t *total,
                            void *stream) {
    if (!P || !total || !d_pair_off || cap < 0 || (cap > 0 && !d_pos)) return HC_EINVAL;
    *total = 0;
    hipStream_t s = hipStream_t(stream);
    // a second run, with the scratch grown to the bound of batch_grow_scratch
    // for the total the first run counted, always fits; a third is never
    // needed, and a second run that still falls short is reported as an error
    for (int attempt = 0; attempt < 2; ++attempt) {
        // (re)build the graph for these buffers
        if (!P->exec || P->g_pos != d_pos || P->g_off != d_pair_off || P->g_cap != cap || P->g_stream != s) {
            P->drop_graph();
            hipStream_t cs;
            if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return HC_EHIP;
            hc_status st = HC_OK;
            if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = HC_EHIP;
            if (st == HC_OK) st = batch_enqueue(P->D, d_pos, cap, d_pair_off, cs);
            hipGraph_t g = nullptr;
            if (hipStreamEndCapture(cs, &g) != hipSuccess && st == HC_OK) st = HC_EHIP;
            (void)hipStreamDestroy(cs);
            if (st != HC_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(g);
                return HC_EHIP;
            }
            P->graph = g;
            P->g_pos = d_pos;
            P->g_off = d_pair_off;
            P->g_cap = cap;
            P->g_stream = s;
        }
        if (hipGraphLaunch(P->exec, s) != hipSuccess) return HC_EHIP;
        unsigned long long ctl[4] = {0, 0, 0, 0};
        int64_t tot = 0;
        if (hipMemcpyAsync(ctl, P->D.ctl.p, sizeof(ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&tot, d_pair_off + P->D.n_pairs, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return HC_EHIP;
        *total = tot;
        if (ctl[2] == 0ull) return tot > cap ? HC_EOVERFLOW : HC_OK;
        // scratch was too small: grow it and run again
        if (batch_grow_scratch(P->D, ctl[1], uint64_t(tot)) != HC_OK) return HC_ENOMEM;
        P->drop_graph();
    }
    return HC_EHIP;
}

hc_status hc_search_batched(const hc_batch *b, const hc_params *params, int64_t *d_pos, int64_t cap,
                            int64_t *d_pair_off, int64_t *total, void *stream) {
    if (!total) return HC_EINVAL;
    *total = 0;
    if (!d_pair_off || cap < 0 || (cap > 0 && !d_pos)) return HC_EINVAL;
    hc_batch_plan *p = nullptr;
    hc_status st = hc_batch_plan_create(b, params, &p);
    if (st != HC_OK) return st;
    st = hc_batch_plan_run(p, d_pos, cap, d_pair_off, total, stream);
    hc_batch_plan_free(p);
    return st;
}

}  // extern "C"
