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

#include "hc_device.h"
#include "hc_internal.h"
#include "hc_runtime.h"

namespace hc {

struct BPat {            // one pattern of the batch, as the kernel reads it
    uint32_t m, q, s, mask, hv;
    uint32_t x_off;      // byte offset of x in the packed patterns (16-aligned)
    uint32_t pad0, pad1;
};

struct BItem {           // one work item
    uint32_t text, tile, g0, g1;   // group = glist[g0, g1), sorted by m descending
};

struct BatchArgs {
    const uint8_t *text;           // all texts
    const uint64_t *text_off;      // n_texts + 1
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

template <typename WT, int Q, int K>
__device__ __forceinline__ TileResult batch_tile(const uint32_t *t32, uint32_t tb, const WT *F,
                                                 const uint32_t *x32, const PatternView &P,
                                                 uint32_t S, uint32_t seg, uint32_t *bm, Parked *park,
                                                 uint32_t *misc, uint32_t &it, uint32_t &round) {
    return search_tile<Q, WT, K>(t32, tb, F, x32, P, S, seg, bm, park, misc, it, round);
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

// Per-pattern table and bytes, staged through registers: 16 bytes per thread
// per step (tables <= 16 KiB and patterns <= 4 KiB + padding).
constexpr int kFStage = 4;    // up to 16 KiB of F
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

__device__ __forceinline__ void pat_commit(const PatStage &ps, uint8_t *F, uint8_t *x8,
                                           uint32_t table_bytes, uint32_t x_bytes) {
    u32x4 *f = reinterpret_cast<u32x4 *>(F);
    const uint32_t nf = table_bytes / 16u;
#pragma unroll
    for (int k = 0; k < kFStage; ++k) {
        const uint32_t c = k * kThreads + threadIdx.x;
        if (c < nf) f[c] = ps.f[k];
    }
    u32x4 *x = reinterpret_cast<u32x4 *>(x8);
    const uint32_t nx = x_bytes / 16u;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const uint32_t c = k * kThreads + threadIdx.x;
        if (c < nx) x[c] = ps.x[k];
    }
}

template <typename WT>
__global__ __launch_bounds__(kThreads) void hc_batch_kernel(BatchArgs A) {
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
        const uint64_t tbase = A.text_off[W.text];
        const uint64_t n_t = A.text_off[W.text + 1] - tbase;
        const uint64_t tile_lo = uint64_t(W.tile) * A.tile;
        // longest pattern of the group comes first
        const uint32_t span = A.pats[A.glist[2 * W.g0]].m;
        const uint64_t g1 = min<uint64_t>(tile_lo + A.tile + span - 1u, n_t);
        Stage st;
        const uint32_t tb = stage_issue(A.text + tbase, tile_lo, g1, st);
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
            pat_commit(ps, F8, x8, A.table_bytes, L.x_bytes);
            lds_barrier();
            if (gi + 1 < W.g1) {
                const uint32_t pn = A.glist[2 * (gi + 1)];
                pat_issue(A.Fs, A.xs, A.pats[pn], pn, A.table_bytes, L.x_bytes, ps);
            }
            const uint64_t starts = n_t >= bp.m ? n_t - bp.m + 1u : 0u;
            if (tile_lo >= starts) {   // uniform: no window of this pattern starts here
                lds_barrier();
                continue;
            }
            const uint32_t S = uint32_t(min<uint64_t>(A.tile, starts - tile_lo));
            const PatternView P{bp.m, bp.q, bp.s, bp.mask, bp.hv};
            const uint32_t shift = bp.m - bp.q + 1u;
            const TileResult R = shift <= 12u
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

__global__ void hc_batch_reset(unsigned long long *ctl) {
    if (threadIdx.x < 4) ctl[threadIdx.x] = 0ull;
}

// ----------------------------------------------------------------------------
// host side: the plan
// ----------------------------------------------------------------------------

struct DeviceBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DeviceBuf() {
        if (p) (void)hipFree(p);
    }
    hc_status ensure(size_t b) {
        if (bytes >= b && p) return HC_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (hipMalloc(&p, std::max<size_t>(b, 16)) != hipSuccess) return HC_ENOMEM;
        bytes = std::max<size_t>(b, 16);
        return HC_OK;
    }
    template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

}  // namespace hc

using namespace hc;

struct hc_batch_plan {
    int device = -1;
    uint32_t n_pairs = 0, n_items = 0, tile = 0, seg = 100, table_bytes = 0, max_m = 1, w = 16;
    uint64_t n_entries = 0, scratch_cap = 0;
    const uint8_t *d_text = nullptr;
    DeviceBuf text_off, pats, xs, Fs, items, glist, pair_base, counts, toff, temp, ctl, tot, bsum, grand;
    uint32_t grid = 0, lds = 0, nb = 0;
    // graph for (d_pos, cap, d_pair_off, stream)
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int64_t *g_pos = nullptr, *g_off = nullptr;
    int64_t g_cap = -1;
    hipStream_t g_stream = nullptr;
    std::vector<unsigned long long> host_ctl;
    ~hc_batch_plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace hc {

template <typename WT>
static hc_status batch_occupancy(uint32_t lds, int *per_cu) {
    *per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, reinterpret_cast<const void *>(hc_batch_kernel<WT>),
                                                     kThreads, lds) != hipSuccess)
        return HC_EHIP;
    *per_cu = std::max(1, *per_cu);
    return HC_OK;
}

static hc_status enqueue_batch(hc_batch_plan *P, int64_t *d_pos, int64_t cap, int64_t *d_pair_off,
                               hipStream_t s) {
    hipLaunchKernelGGL(hc_batch_reset, dim3(1), dim3(64), 0, s, P->ctl.as<unsigned long long>());
    BatchArgs A;
    A.text = P->d_text;
    A.text_off = P->text_off.as<uint64_t>();
    A.pats = P->pats.as<BPat>();
    A.xs = P->xs.as<uint8_t>();
    A.Fs = P->Fs.as<uint8_t>();
    A.items = P->items.as<BItem>();
    A.n_items = P->n_items;
    A.glist = P->glist.as<uint32_t>();
    A.pair_base = P->pair_base.as<uint64_t>();
    A.counts = P->counts.as<uint32_t>();
    A.toff = P->toff.as<uint32_t>();
    A.temp = P->temp.as<int64_t>();
    A.temp_cap = P->scratch_cap;
    A.ctl = P->ctl.as<unsigned long long>();
    A.tile = P->tile;
    A.seg = P->seg;
    A.table_bytes = P->table_bytes;
    A.max_m = P->max_m;
    if (P->n_items > 0) {
        if (P->w == 16)
            hipLaunchKernelGGL(hc_batch_kernel<uint16_t>, dim3(P->grid), dim3(kThreads), P->lds, s, A);
        else
            hipLaunchKernelGGL(hc_batch_kernel<uint32_t>, dim3(P->grid), dim3(kThreads), P->lds, s, A);
    }
    const uint32_t pgrid = uint32_t((uint64_t(P->n_pairs) * kWave + 255u) / 256u);
    if (P->n_pairs > 0) {
        hipLaunchKernelGGL(hc_pair_totals, dim3(pgrid), dim3(256), 0, s, P->pair_base.as<uint64_t>(),
                           uint64_t(P->n_pairs), P->counts.as<uint32_t>(), P->tot.as<uint64_t>());
        hipLaunchKernelGGL(hc_scan_reduce, dim3(P->nb), dim3(256), 0, s, P->tot.as<uint64_t>(),
                           uint64_t(P->n_pairs), P->bsum.as<uint64_t>());
    }
    hipLaunchKernelGGL(hc_scan_blocks, dim3(1), dim3(256), 0, s, P->bsum.as<uint64_t>(), P->nb,
                       P->grand.as<uint64_t>());
    if (P->n_pairs > 0) {
        hipLaunchKernelGGL(hc_scan_apply, dim3(P->nb), dim3(256), 0, s, P->tot.as<uint64_t>(),
                           uint64_t(P->n_pairs), P->bsum.as<uint64_t>(), d_pair_off);
    }
    hipLaunchKernelGGL(hc_scan_total, dim3(1), dim3(1), 0, s, P->grand.as<uint64_t>(),
                       d_pair_off + P->n_pairs);
    if (P->n_pairs > 0 && cap > 0) {
        hipLaunchKernelGGL(hc_pair_emit, dim3(pgrid), dim3(256), 0, s, P->pair_base.as<uint64_t>(),
                           uint64_t(P->n_pairs), P->counts.as<uint32_t>(), P->toff.as<uint32_t>(),
                           P->temp.as<int64_t>(), d_pair_off, d_pos, cap,
                           P->ctl.as<unsigned long long>());
    }
    return hipGetLastError() == hipSuccess ? HC_OK : HC_EHIP;
}

}  // namespace hc

extern "C" {

hc_status hc_batch_plan_create(const hc_batch *b, const hc_params *params, hc_batch_plan **out) {
    if (!out) return HC_EINVAL;
    *out = nullptr;
    if (!b || b->n_pairs < 0 || b->n_texts < 0 || b->n_pats < 0) return HC_EINVAL;
    if (b->n_pairs > 0 && (!b->pair_pat || !b->pair_text || !b->text_off || !b->pat_off || !b->pat ||
                           !b->d_text))
        return HC_EINVAL;
    if (b->n_pairs > int64_t(0x7FFFFFFF)) return HC_EINVAL;
    const DeviceInfo &di = device_info();
    if (!di.ok) return HC_EHIP;
    std::unique_ptr<hc_batch_plan> P(new (std::nothrow) hc_batch_plan());
    if (!P) return HC_ENOMEM;
    P->device = di.device;
    P->d_text = b->d_text;
    P->n_pairs = uint32_t(b->n_pairs);
    for (int32_t t = 0; t < b->n_texts; ++t) {
        if (b->text_off[t + 1] < b->text_off[t]) return HC_EINVAL;
        if (b->text_off[t + 1] - b->text_off[t] > int64_t(0xFFFFFFFFll)) return HC_EINVAL;
    }
    for (int32_t i = 0; i < b->n_pats; ++i)
        if (b->pat_off[i + 1] - b->pat_off[i] < 1 || b->pat_off[i + 1] - b->pat_off[i] > kMaxM)
            return HC_EINVAL;
    for (int64_t k = 0; k < b->n_pairs; ++k)
        if (b->pair_pat[k] < 0 || b->pair_pat[k] >= b->n_pats || b->pair_text[k] < 0 ||
            b->pair_text[k] >= b->n_texts)
            return HC_EINVAL;

    // common table shape for the batch; q per pattern
    int w = params && params->w ? params->w : 16;
    int alpha = params && params->alpha ? params->alpha : 12;
    if ((w != 16 && w != 32) || alpha < 1 || alpha > alpha_max(w)) return HC_EINVAL;
    P->w = uint32_t(w);
    P->table_bytes = uint32_t((size_t(1) << alpha) * size_t(w / 8));
    P->table_bytes = std::max<uint32_t>(16, (P->table_bytes + 15u) & ~15u);
    if (P->table_bytes > uint32_t(kFStage) * kThreads * 16u) return HC_EINVAL;   // <= 16 KiB

    const int32_t np = b->n_pats;
    std::vector<BPat> bp(size_t(std::max(np, 1)));
    std::vector<uint8_t> Fh(size_t(np) * P->table_bytes, 0);
    std::vector<uint32_t> xoff(size_t(np) + 1, 0);
    for (int32_t i = 0; i < np; ++i) {
        const int64_t m = b->pat_off[i + 1] - b->pat_off[i];
        xoff[i + 1] = xoff[i] + uint32_t(((m + 15) & ~int64_t(15)) + 32);
    }
    int64_t mmax = 1;
    for (int32_t i = 0; i < np; ++i) mmax = std::max<int64_t>(mmax, b->pat_off[i + 1] - b->pat_off[i]);
    // every pattern's bytes are read as a block of the longest pattern's size
    std::vector<uint8_t> Xh(xoff[np] + size_t((mmax + 15) & ~int64_t(15)) + 64, 0);
    for (int32_t i = 0; i < np; ++i) {
        const uint8_t *x = b->pat + b->pat_off[i];
        const int64_t m = b->pat_off[i + 1] - b->pat_off[i];
        int q = params ? params->q : 0, a = alpha, ww = w;
        default_params(m, distinct_bytes(x, m), q, a, ww);
        q = int(std::min<int64_t>(q, m));
        if (validate_params(m, q, alpha, w) != HC_OK) return HC_EINVAL;
        PatternData pd;
        build_link_table(x, m, q, alpha, w, pd);
        std::vector<uint8_t> packed = pack_table(pd);
        std::memcpy(Fh.data() + size_t(i) * P->table_bytes, packed.data(), packed.size());
        std::memcpy(Xh.data() + xoff[i], x, size_t(m));
        bp[i] = BPat{uint32_t(m), uint32_t(q), uint32_t(pd.s), pd.mask, pd.hv, xoff[i], 0, 0};
        P->max_m = std::max<uint32_t>(P->max_m, uint32_t(m));
    }

    // tiles: as large as LDS allows, 4 workgroups per compute unit if possible
    P->seg = 100;
    P->tile = kThreads * P->seg;
    LdsLayout L = lds_layout(P->tile, P->max_m, P->table_bytes, 0);
    while ((L.total > di.max_lds_per_block || P->tile + P->max_m - 1u > stage_limit(kThreads)) &&
           P->seg > 8) {
        P->seg -= 4;
        P->tile = kThreads * P->seg;
        L = lds_layout(P->tile, P->max_m, P->table_bytes, 0);
    }
    if (L.total > di.max_lds_per_block) return HC_EINVAL;
    P->lds = L.total;

    // pairs grouped by text, longest pattern first, in groups of up to 128
    const int32_t nt = b->n_texts;
    std::vector<uint64_t> toff(size_t(nt) + 1, 0);
    for (int32_t t = 0; t <= nt; ++t) toff[t] = uint64_t(b->text_off[t]);
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> by_text(size_t(std::max(nt, 1)));
    std::vector<uint64_t> pair_base(size_t(P->n_pairs) + 1, 0);
    for (uint32_t k = 0; k < P->n_pairs; ++k) {
        const uint32_t p = uint32_t(b->pair_pat[k]), t = uint32_t(b->pair_text[k]);
        by_text[t].push_back({p, k});
        const uint64_t n_t = toff[t + 1] - toff[t], m = bp[p].m;
        const uint64_t starts = n_t >= m ? n_t - m + 1 : 0;
        pair_base[k + 1] = pair_base[k] + (starts + P->tile - 1) / P->tile;
    }
    P->n_entries = pair_base[P->n_pairs];
    constexpr uint32_t kGroup = 128;
    std::vector<uint32_t> glist;
    struct ItemCost {
        double cost;
        BItem it;
    };
    std::vector<ItemCost> items;
    for (int32_t t = 0; t < nt; ++t) {
        auto &v = by_text[t];
        std::sort(v.begin(), v.end(), [&](const std::pair<uint32_t, uint32_t> &a,
                                          const std::pair<uint32_t, uint32_t> &c) {
            return bp[a.first].m > bp[c.first].m || (bp[a.first].m == bp[c.first].m && a.second < c.second);
        });
        const uint64_t n_t = toff[t + 1] - toff[t];
        const uint32_t tiles = uint32_t((n_t + P->tile - 1) / P->tile);
        for (size_t g = 0; g < v.size(); g += kGroup) {
            const uint32_t g0 = uint32_t(glist.size() / 2);
            double per_byte = 0;
            for (size_t j = g; j < std::min(v.size(), g + kGroup); ++j) {
                glist.push_back(v[j].first);
                glist.push_back(v[j].second);
                const BPat &q = bp[v[j].first];
                per_byte += 1.0 / double(q.m - q.q + 1) + 0.02;
            }
            const uint32_t g1 = uint32_t(glist.size() / 2);
            for (uint32_t tl = 0; tl < tiles; ++tl) {
                const double bytes = double(std::min<uint64_t>(P->tile, n_t - uint64_t(tl) * P->tile));
                items.push_back({bytes * per_byte, BItem{uint32_t(t), tl, g0, g1}});
            }
        }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const ItemCost &a, const ItemCost &c) { return a.cost > c.cost; });
    std::vector<BItem> ih(items.size());
    for (size_t i = 0; i < items.size(); ++i) ih[i] = items[i].it;
    P->n_items = uint32_t(ih.size());

    // device buffers
    auto up = [&](DeviceBuf &d, const void *src, size_t bytes) -> hc_status {
        if (d.ensure(bytes) != HC_OK) return HC_ENOMEM;
        if (bytes && hipMemcpy(d.p, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return HC_EHIP;
        return HC_OK;
    };
    hc_status st;
    if ((st = up(P->text_off, toff.data(), toff.size() * 8)) != HC_OK) return st;
    if ((st = up(P->pats, bp.data(), bp.size() * sizeof(BPat))) != HC_OK) return st;
    if ((st = up(P->xs, Xh.data(), Xh.size())) != HC_OK) return st;
    if ((st = up(P->Fs, Fh.data(), std::max<size_t>(Fh.size(), 16))) != HC_OK) return st;
    if ((st = up(P->items, ih.data(), ih.size() * sizeof(BItem))) != HC_OK) return st;
    if ((st = up(P->glist, glist.data(), glist.size() * 4)) != HC_OK) return st;
    if ((st = up(P->pair_base, pair_base.data(), pair_base.size() * 8)) != HC_OK) return st;
    if (P->counts.ensure(P->n_entries * 4) != HC_OK || P->toff.ensure(P->n_entries * 4) != HC_OK ||
        P->ctl.ensure(64) != HC_OK || P->tot.ensure(size_t(P->n_pairs) * 8) != HC_OK ||
        P->grand.ensure(8) != HC_OK)
        return HC_ENOMEM;
    P->nb = uint32_t((uint64_t(P->n_pairs) + kScanBlock - 1) / kScanBlock);
    if (P->bsum.ensure(size_t(std::max<uint32_t>(P->nb, 1)) * 8) != HC_OK) return HC_ENOMEM;
    P->scratch_cap = 1u << 23;   // positions; grown when a run needs more
    if (P->temp.ensure(P->scratch_cap * 8) != HC_OK) return HC_ENOMEM;
    int per_cu = 1;
    st = P->w == 16 ? batch_occupancy<uint16_t>(P->lds, &per_cu) : batch_occupancy<uint32_t>(P->lds, &per_cu);
    if (st != HC_OK) return st;
    P->grid = std::max<uint32_t>(1, std::min<uint32_t>(P->n_items, uint32_t(di.cus) * uint32_t(per_cu)));
    *out = P.release();
    return HC_OK;
}

void hc_batch_plan_free(hc_batch_plan *p) { delete p; }

hc_status hc_batch_plan_run(hc_batch_plan *P, int64_t *d_pos, int64_t cap, int64_t *d_pair_off,
                            int64_t *total, void *stream) {
    if (!P || !total || !d_pair_off || cap < 0 || (cap > 0 && !d_pos)) return HC_EINVAL;
    *total = 0;
    hipStream_t s = hipStream_t(stream);
    for (int attempt = 0; attempt < 2; ++attempt) {
        // (re)build the graph for these buffers
        if (!P->exec || P->g_pos != d_pos || P->g_off != d_pair_off || P->g_cap != cap ||
            P->g_stream != s) {
            if (P->exec) (void)hipGraphExecDestroy(P->exec);
            if (P->graph) (void)hipGraphDestroy(P->graph);
            P->exec = nullptr;
            P->graph = nullptr;
            hipStream_t cs;
            if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return HC_EHIP;
            hc_status st = HC_OK;
            if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = HC_EHIP;
            if (st == HC_OK) st = enqueue_batch(P, d_pos, cap, d_pair_off, cs);
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
        if (hipMemcpyAsync(ctl, P->ctl.p, sizeof(ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&tot, d_pair_off + P->n_pairs, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return HC_EHIP;
        *total = tot;
        if (ctl[2] == 0ull) return tot > cap ? HC_EOVERFLOW : HC_OK;
        // scratch was too small: grow it to the reserved size and run again
        // every workgroup may leave at most one chunk partly unused
        const uint64_t need = std::max<uint64_t>(ctl[1], uint64_t(tot) + uint64_t(P->grid + 16u) * kChunk);
        if (P->temp.ensure(need * 8) != HC_OK) return HC_ENOMEM;
        P->scratch_cap = need;
        if (P->exec) (void)hipGraphExecDestroy(P->exec);
        if (P->graph) (void)hipGraphDestroy(P->graph);
        P->exec = nullptr;
        P->graph = nullptr;
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
