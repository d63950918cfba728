// Single-pattern searching phase of HC (Section 3.3) on gfx950.
//
// Two launches on the caller's stream:
//  1. hc_search_kernel: a persistent grid of G workgroups; workgroup b takes
//     text tiles b, b + G, ... Per tile it stages the bytes of the tile's
//     window starts plus an (m-1)-byte halo from HBM into LDS with 16-byte
//     loads (the next tile's loads are in flight while the current tile is
//     searched), runs the searching loop in every lane against F and x held
//     in LDS for the whole launch, marks candidate windows in an LDS bitmap,
//     compares them with x, and stores the tile's count and occurrences
//     (tile-relative starts, or the bitmap when there are many).
//  2. hc_emit_kernel: writes every tile's occurrences as ascending int64
//     positions at the offset given by the counts of the tiles before it.
// No workgroup ever waits for another, so any grid size is safe.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "hc_device.h"
#include "hc_internal.h"
#include "hc_runtime.h"

namespace hc {

// Internal schedule code of the SHC (sentinel) variant.
constexpr int kSchedShc = 16;

struct SearchArgs {
    const uint8_t *y;
    uint64_t n;
    const uint8_t *x;
    const void *F;
    uint32_t m, q, s, mask, hv;
    uint32_t table_bytes;
    uint32_t tile;       // window starts per tile (256 * segment, <= 65536)
    uint32_t seg;        // window starts per lane
    uint64_t starts;     // n - m + 1
    uint32_t n_tiles;
    uint32_t emit_per;   // tiles per range of the ordered output
    int64_t *out;
    int64_t cap;
    int64_t *d_count;
    uint32_t *counts;    // per tile: occurrences
    uint32_t *rsum;      // per output range: occurrences, added atomically (or null)
    uint32_t *slots;     // per tile: up to kSlot tile-relative starts
    uint32_t *spill;     // per tile: the occurrence bitmap, when denser
};

template <int Q, typename WT, int SCHED, int K>
__global__ __launch_bounds__(kBlock) void hc_search_kernel(SearchArgs A) {
    extern __shared__ __align__(16) uint8_t lds[];
    const LdsLayout L = lds_layout(A.tile, A.m, A.table_bytes, SCHED == kSchedShc ? A.m : 0u);
    uint8_t *t8 = lds + L.text_off;
    const uint32_t *t32 = reinterpret_cast<const uint32_t *>(t8);
    uint32_t *bm = reinterpret_cast<uint32_t *>(lds + L.bitmap_off);
    WT *F = reinterpret_cast<WT *>(lds + L.table_off);
    uint8_t *x8 = lds + L.x_off;
    const uint32_t *x32 = reinterpret_cast<const uint32_t *>(x8);
    Parked *park = reinterpret_cast<Parked *>(lds + L.park_off);
    uint32_t *misc = reinterpret_cast<uint32_t *>(lds + L.misc_off);
    // misc: [0..3] scan, [8..9] candidate flags by tile parity, [10..11]
    // parked-walk counts by round parity

    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const uint32_t tile_words = A.tile / 32u;

    // F and x stay in LDS for the whole launch; the bitmap starts cleared
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(A.F);
        uint4 *dst = reinterpret_cast<uint4 *>(F);
        for (uint32_t i = tid; i < (A.table_bytes + 15u) / 16u; i += kBlock) dst[i] = src[i];
        for (uint32_t i = tid; i < L.x_bytes; i += kBlock) x8[i] = i < A.m ? A.x[i] : 0;
        for (uint32_t i = tid; i < tile_words; i += kBlock) bm[i] = 0u;
    }
    const PatternView P = hash_weights(PatternView{A.m, uint32_t(Q), A.s, A.mask, A.hv});

    // ---- search phase: workgroup b takes tiles b, b + G, b + 2G, ... (at
    // any moment the grid reads one contiguous stretch of the text)
    constexpr bool kDense = SCHED >= HC_SCHED_DENSE && SCHED < kSchedShc;
    Stage<kDense ? dense_chunks(Q) : kStageMax> stage;
    const uint32_t G = gridDim.x;
    uint32_t tb = 0;
    if (blockIdx.x < A.n_tiles) {
        const uint64_t lo = uint64_t(blockIdx.x) * A.tile;
        const uint32_t S = uint32_t(min<uint64_t>(A.tile, A.starts - lo));
        tb = stage_issue(A.y, lo, lo + S + A.m - 1u, stage);
    }
    if (tid == 0) {
        misc[8] = 0u;    // candidate flags, one per tile parity
        misc[10] = 0u;   // parked-walk counts, one per round parity
        misc[11] = 0u;
    }
    __syncthreads();
    uint32_t round = 0;
    uint32_t it = 0;
    for (uint32_t t = blockIdx.x; t < A.n_tiles; t += G) {
        const uint64_t tile_lo = uint64_t(t) * A.tile;
        const uint32_t S = uint32_t(min<uint64_t>(A.tile, A.starts - tile_lo));
        stage_commit(stage, t8);
        lds_barrier();
        if constexpr (SCHED == kSchedShc) {
            // the sentinel: a copy of x right after the tile's last window
            for (uint32_t i = tid; i < A.m; i += kBlock) t8[tb + S + A.m - 1u + i] = x8[i];
            lds_barrier();
        }

        // the next tile's bytes travel while this one is searched
        const uint32_t tb_cur = tb;
        if (t + G < A.n_tiles) {
            const uint64_t lo = uint64_t(t + G) * A.tile;
            const uint32_t Sn = uint32_t(min<uint64_t>(A.tile, A.starts - lo));
            tb = stage_issue(A.y, lo, lo + Sn + A.m - 1u, stage);
        }
        uint32_t total, mine, w0, w1;
        if constexpr (SCHED == HC_SCHED_WAVE) {
            uint32_t *any = &misc[8 + (it & 1u)];
            const uint32_t per = (S + 3u) / 4u;
            const uint32_t lo = min(S, wid * per), hi = min(S, lo + per);
            hc_wave<Q, WT>(t32, tb_cur, F, P, lo, hi, bm, lane, any);
            lds_barrier();
            const bool has = *any != 0u;
            if (tid == 0) misc[8 + ((it + 1u) & 1u)] = 0u;
            ++it;
            total = mine = w0 = w1 = 0u;
            if (has) {
                const uint32_t words = (S + 31u) / 32u;
                const uint32_t wpt = (words + kBlock - 1u) / kBlock;
                w0 = min(words, tid * wpt);
                w1 = min(words, w0 + wpt);
                uint32_t c = 0;
                for (uint32_t i = w0; i < w1; ++i) {
                    uint32_t b = bm[i], keep = b;
                    while (b) {
                        const uint32_t bit = __builtin_ctz(b);
                        b &= b - 1u;
                        if (!window_equals(t32, tb_cur + i * 32u + bit, x32, A.m)) keep &= ~(1u << bit);
                    }
                    bm[i] = keep;
                    c += __popc(keep);
                }
                mine = block_exclusive_scan(c, misc, &total);
            }
        } else if constexpr (SCHED == kSchedShc) {
            const TileResult R = shc_tile<Q, WT>(t32, tb_cur, F, x32, P, S, A.seg, bm, misc, it);
            total = R.total;
            mine = R.mine;
            w0 = R.w0;
            w1 = R.w1;
        } else if constexpr (SCHED >= HC_SCHED_DENSE) {   // dense, C = SCHED - HC_SCHED_DENSE
            constexpr int C = SCHED - HC_SCHED_DENSE;
            const TileResult R = dense_tile<(C == 0 || Q <= 4 ? Q : 4), WT, C>(
                t32, tb_cur, F, x32, P, S, bm, misc, it);
            total = R.total;
            mine = R.mine;
            w0 = R.w0;
            w1 = R.w1;
        } else {
            const TileResult R = search_tile<Q, WT, K>(t32, tb_cur, F, x32, P, S, A.seg, bm, park,
                                                       misc, it, round);
            total = R.total;
            mine = R.mine;
            w0 = R.w0;
            w1 = R.w1;
        }
        if (tid == 0) {
            A.counts[t] = total;
            if (A.rsum && total != 0u) atomicAdd(&A.rsum[t / A.emit_per], total);
        }
        if (total != 0u) {
            if (total <= kSlot) {
                uint32_t j = mine;
                for (uint32_t i = w0; i < w1; ++i) {
                    uint32_t b = bm[i];
                    while (b) {
                        const uint32_t bit = __builtin_ctz(b);
                        b &= b - 1u;
                        A.slots[uint64_t(t) * kSlot + j++] = i * 32u + bit;
                    }
                }
            } else {
                for (uint32_t i = w0; i < w1; ++i) A.spill[uint64_t(t) * tile_words + i] = bm[i];
            }
            for (uint32_t i = w0; i < w1; ++i) bm[i] = 0u;
        }
    }
}

// Sparse variant for long patterns: no tile is staged. Every lane runs the
// searching loop over its block of window starts and reads each q-gram it
// hashes straight from global memory, so only the cache lines that hold
// those q-grams are fetched (with shifts of m - q + 1 most lines of the text
// are never read). The bytes of a lane's next attempt (where an empty word
// would move it) are fetched with the current one's. Candidates are marked in the LDS bitmap of the tile and compared
// with x (also read in place); counts, range totals, slots and spilled
// bitmaps are written exactly as the streaming kernel writes them, so the
// same emit kernel follows.
struct SparseLayout {
    uint32_t bm_off, table_off, x_off, misc_off, total;
};

__host__ __device__ inline SparseLayout sparse_layout(uint32_t tile, uint32_t m, uint32_t table_bytes) {
    SparseLayout L;
    L.bm_off = 0;
    L.table_off = align16(tile / 8u);
    L.x_off = L.table_off + align16(table_bytes);
    L.misc_off = L.x_off + align16(m) + 32u;
    L.total = L.misc_off + 128u;
    return L;
}

template <int Q, typename WT>
__global__ __launch_bounds__(kBlock) void hc_sparse_kernel(SearchArgs A) {
    extern __shared__ __align__(16) uint8_t lds[];
    const SparseLayout L = sparse_layout(A.tile, A.m, A.table_bytes);
    uint32_t *bm = reinterpret_cast<uint32_t *>(lds + L.bm_off);
    WT *F = reinterpret_cast<WT *>(lds + L.table_off);
    uint8_t *x8 = lds + L.x_off;
    const uint32_t *x32 = reinterpret_cast<const uint32_t *>(x8);
    uint32_t *misc = reinterpret_cast<uint32_t *>(lds + L.misc_off);
    const uint32_t tid = threadIdx.x;
    const uint32_t tile_words = A.tile / 32u;
    {
        // table, pattern bytes (zero-padded to 16 bytes on the device, plus
        // 32 zero bytes here) and a cleared bitmap, in 16-byte units
        const uint4 *src = reinterpret_cast<const uint4 *>(A.F);
        uint4 *dst = reinterpret_cast<uint4 *>(F);
        for (uint32_t i = tid; i < (A.table_bytes + 15u) / 16u; i += kBlock) dst[i] = src[i];
        const uint4 *xs = reinterpret_cast<const uint4 *>(A.x);
        uint4 *xd = reinterpret_cast<uint4 *>(x8);
        const uint32_t xw = align16(A.m) / 16u;
        for (uint32_t i = tid; i < xw + 2u; i += kBlock) xd[i] = i < xw ? xs[i] : uint4{0u, 0u, 0u, 0u};
        uint4 *bm4 = reinterpret_cast<uint4 *>(bm);
        for (uint32_t i = tid; i < tile_words / 4u; i += kBlock) bm4[i] = uint4{0u, 0u, 0u, 0u};
        if (tid == 0) misc[8] = misc[9] = 0u;
    }
    lds_barrier();
    const GlobalText T{reinterpret_cast<uintptr_t>(A.y), reinterpret_cast<uintptr_t>(A.y) + A.n};
    const uint32_t shift = A.m - uint32_t(Q) + 1u;
    const PatternView P = hash_weights(PatternView{A.m, uint32_t(Q), A.s, A.mask, A.hv});
    const uint32_t lane = tid & (kWave - 1);
    uint32_t it = 0;
    for (uint32_t t = blockIdx.x; t < A.n_tiles; t += gridDim.x) {
        const uint64_t tile_lo = uint64_t(t) * A.tile;
        const uint32_t S = uint32_t(min<uint64_t>(A.tile, A.starts - tile_lo));
        const uintptr_t base = T.lo + tile_lo;
        uint32_t *any = &misc[8 + (it & 1u)];
        const uint32_t lo = min(S, tid * A.seg), hi = min(S, lo + A.seg);
        uint32_t J = lo + A.m - 1u;
        const uint32_t Jend = hi + A.m - 1u;   // window ends of this lane: [J, Jend)
        // A chain walk longer than kSparseLocalSteps links past the span is
        // parked (state in e, v, z) and finished by the whole wavefront, 64
        // q-grams per round trip, instead of one dependent memory access per
        // link.
        bool parked = false;
        uint32_t e = 0, v = 0;
        WT z = 0;
        while (__ballot(J < Jend) != 0ull) {   // wavefront-uniform
            if (J < Jend && !parked) {
                // the 16 bytes ending at this attempt's window end and, when
                // it lies in the lane's range, at the next one (where an empty
                // word would move it), loaded together
                uint32_t w0[4], w1[4];
                const uint32_t J1 = J + shift;
                gspan16(T, base + J, w0);
                if (J1 < Jend) gspan16(T, base + J1, w1);
                uint32_t next = sparse_attempt<Q, WT>(T, base, F, P, J, w0, e, v, z, bm, any);
                if (next == J1 && J1 < Jend) {   // the next attempt's bytes are already here
                    J = J1;
                    next = sparse_attempt<Q, WT>(T, base, F, P, J, w1, e, v, z, bm, any);
                }
                if (next == kParkedJ)
                    parked = true;   // J stays the window end of the parked walk
                else
                    J = next;
            }
            // parked walks of this wavefront, one at a time, all lanes
            uint64_t pm = __ballot(parked);
            while (pm) {
                const int owner = __ffsll((unsigned long long)pm) - 1;
                pm &= pm - 1ull;
                Parked pk;
                pk.J = uint32_t(__shfl((int)J, owner, kWave));
                pk.e = uint32_t(__shfl((int)e, owner, kWave));
                pk.v = uint32_t(__shfl((int)v, owner, kWave));
                if constexpr (sizeof(WT) == 8) {
                    const uint32_t zl = uint32_t(__shfl((int)uint32_t(z), owner, kWave));
                    const uint32_t zh = uint32_t(__shfl((int)uint32_t(uint64_t(z) >> 32), owner, kWave));
                    pk.z = (uint64_t(zh) << 32) | zl;
                } else {
                    pk.z = uint32_t(__shfl((int)uint32_t(z), owner, kWave));
                }
                const uint32_t next = gchain_wave<Q, WT>(T, base, F, P, pk, lane, bm, any);
                if (lane == uint32_t(owner)) {
                    J = next;
                    parked = false;
                }
            }
        }
        lds_barrier();
        const bool has = *any != 0u;
        if (tid == 0) misc[8 + ((it + 1u) & 1u)] = 0u;
        ++it;
        uint32_t total = 0, mine = 0, w0 = 0, w1 = 0;
        if (has) {
            // verification, one candidate at a time per wavefront: the 64
            // lanes compare 256 dwords of the window per round, all their
            // loads in flight together
            const uint32_t words = (S + 31u) / 32u;
            const uint32_t wid = tid / kWave, nw = (A.m + 3u) >> 2;
            const uint32_t tail = (A.m & 3u) ? ((1u << (8u * (A.m & 3u))) - 1u) : 0xFFFFFFFFu;
            for (uint32_t i0 = wid * kWave; i0 < words; i0 += kBlock) {
                const uint32_t i = i0 + lane;
                uint32_t myw = i < words ? bm[i] : 0u;
                uint64_t nz = __ballot(myw != 0u);
                while (nz) {
                    const int src = __ffsll((unsigned long long)nz) - 1;
                    nz &= nz - 1ull;
                    uint32_t b = uint32_t(__shfl((int)myw, src, kWave)), keep = b;
                    while (b) {
                        const uint32_t bit = __builtin_ctz(b);
                        b &= b - 1u;
                        const uintptr_t wa = base + (i0 + uint32_t(src)) * 32u + bit;
                        const uint32_t sh = uint32_t(wa & 3u);
                        const uintptr_t wb = wa & ~uintptr_t(3);
                        bool diff = false;
                        constexpr int kV = 4;   // dwords per lane per round
                        for (uint32_t k0 = 0; k0 < nw; k0 += kV * kWave) {
                            uint32_t dl[kV], dh[kV];
#pragma unroll
                            for (int u = 0; u < kV; ++u) {
                                const uint32_t k = k0 + uint32_t(u) * kWave + lane;
                                dl[u] = k < nw ? gdword(T, wb + 4u * k) : 0u;
                                dh[u] = k < nw ? gdword(T, wb + 4u * (k + 1u)) : 0u;
                            }
#pragma unroll
                            for (int u = 0; u < kV; ++u) {
                                const uint32_t k = k0 + uint32_t(u) * kWave + lane;
                                uint32_t d = __builtin_amdgcn_alignbyte(dh[u], dl[u], sh) ^ (k < nw ? x32[k] : 0u);
                                if (k + 1u == nw) d &= tail;
                                diff |= k < nw && d != 0u;
                            }
                        }
                        if (__ballot(diff) != 0ull) keep &= ~(1u << bit);
                    }
                    if (lane == uint32_t(src)) myw = keep;
                }
                if (i < words) bm[i] = myw;
            }
            lds_barrier();
            const uint32_t wpt = (words + kBlock - 1u) / kBlock;
            w0 = min(words, tid * wpt);
            w1 = min(words, w0 + wpt);
            uint32_t c = 0;
            for (uint32_t i = w0; i < w1; ++i) c += __popc(bm[i]);
            mine = block_exclusive_scan(c, misc, &total);
        }
        if (tid == 0) {
            A.counts[t] = total;
            if (A.rsum && total != 0u) atomicAdd(&A.rsum[t / A.emit_per], total);
        }
        if (total != 0u) {
            if (total <= kSlot) {
                uint32_t j = mine;
                for (uint32_t i = w0; i < w1; ++i) {
                    uint32_t b = bm[i];
                    while (b) {
                        const uint32_t bit = __builtin_ctz(b);
                        b &= b - 1u;
                        A.slots[uint64_t(t) * kSlot + j++] = i * 32u + bit;
                    }
                }
            } else {
                for (uint32_t i = w0; i < w1; ++i) A.spill[uint64_t(t) * tile_words + i] = bm[i];
            }
            for (uint32_t i = w0; i < w1; ++i) bm[i] = 0u;
        }
        lds_barrier();   // the bitmap is clear before the next tile marks
    }
}

// Ordered output: workgroup b writes the occurrences of tiles
// [b * per, (b + 1) * per) in tile order. Its offset is the number of
// occurrences in all earlier tiles: with range totals (a two-level count
// scan: the search kernel adds each tile's count to its range's total), the
// totals of ranges 0..b-1, read in the same round trip as the workgroup's
// own counts; without them, the counts of all earlier tiles, read once the
// workgroup knows it has output. The search kernel has finished, so every
// count, total, slot and spilled bitmap is visible. Within the workgroup each
// wavefront takes every fourth tile, so four tiles are in progress at once.
struct EmitArgs {
    uint32_t n_tiles, tile, per;
    uint64_t starts;
    const uint32_t *counts;
    const uint32_t *rsum;   // per range: occurrences (null: sum the counts)
    uint32_t *rsum_next;    // the totals of the stream's next call, cleared here (or null)
    const uint32_t *slots;
    const uint32_t *spill;
    int64_t *out;
    int64_t cap;
    int64_t *d_count;
};

// This thread's part of v[0..r): loads issued together, eight per thread per
// pass (one pass covers 2048 values).
__device__ __forceinline__ uint64_t prefix_part(const uint32_t *v, uint32_t r) {
    constexpr int kR = 8;
    uint64_t part = 0;
    for (uint32_t base = 0; base < r; base += kR * kBlock) {
        uint32_t x[kR];
#pragma unroll
        for (int k = 0; k < kR; ++k) {
            const uint32_t i = base + uint32_t(k) * kBlock + threadIdx.x;
            x[k] = i < r ? v[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kR; ++k) part += x[k];
    }
    return part;
}

// This thread's part of counts[0..r) in 16-byte loads, twelve per thread in
// flight at once (one pass covers the 12,288 counts of a 256 MiB text at
// the default tile size).
__device__ __forceinline__ uint64_t counts_part(const uint32_t *counts, uint32_t r) {
    const uint32_t tid = threadIdx.x;
    const uint32_t nvec = r / 4u;
    constexpr int kVec = 12;
    global_u32x4 *c4 = (global_u32x4 *)counts;
    uint64_t part = 0;
    for (uint32_t base = 0; base < nvec; base += kVec * kBlock) {
        u32x4 v[kVec];
#pragma unroll
        for (int k = 0; k < kVec; ++k) {
            const uint32_t i = base + k * kBlock + tid;
            v[k] = i < nvec ? c4[i] : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int k = 0; k < kVec; ++k) part += uint64_t(v[k].x) + v[k].y + v[k].z + v[k].w;
    }
    if (tid < (r & 3u)) part += counts[nvec * 4u + tid];
    return part;
}

// Block-wide sum of one 64-bit value per thread (blockDim = 256).
__device__ __forceinline__ uint64_t block_sum64(uint64_t v, uint64_t *lds4) {
    const uint32_t lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint32_t lo = uint32_t(__shfl_xor(int(uint32_t(v)), o, kWave));
        const uint32_t hi = uint32_t(__shfl_xor(int(uint32_t(v >> 32)), o, kWave));
        v += (uint64_t(hi) << 32) | lo;
    }
    if (lane == 0) lds4[wid] = v;
    lds_barrier();
    return lds4[0] + lds4[1] + lds4[2] + lds4[3];
}

// The first kWave slots of a wavefront's first kSpecTiles tiles are loaded
// with the counts, before it is known whether they hold anything: a tile
// with at most kWave occurrences then needs no further round trip.
constexpr int kSpecTiles = 4;

// Bitmap words of a spilled tile read by one wavefront per batch: one word
// per lane per round, all rounds' loads in flight together.
constexpr int kEmitRounds = 16;

// Tiles with at most kStageTile occurrences and at most kWave * kLaneWords
// bitmap words are ordered in one pass.
constexpr uint32_t kStageTile = 1024;
constexpr int kLaneWords = 32;

// Orders LDS accesses of one wavefront (its lanes execute in lock step and
// its LDS operations complete in issue order; this only stops the compiler
// from moving them).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

__global__ __launch_bounds__(kBlock) void hc_emit_kernel(EmitArgs A) {
    __shared__ uint32_t lds_w[4];
    __shared__ uint64_t lds_s[4];
    __shared__ uint32_t cnt[kBlock];
    __shared__ uint32_t off[kBlock];
    // per wavefront, positions in ascending order before they are stored:
    // a whole tile's (tile-relative, 32 bits), or one round's of 64 bitmap
    // words (relative to the round's first window, 16 bits)
    __shared__ uint32_t stage[kBlock / kWave][kStageTile];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const uint32_t tile_words = A.tile / 32u;
    if (A.rsum_next)   // every workgroup clears its share
        for (uint32_t i = blockIdx.x + tid * gridDim.x; i < kRsumCap; i += kBlock * gridDim.x) A.rsum_next[i] = 0u;
    if (A.n_tiles == 0) {
        if (blockIdx.x == 0 && tid == 0) *A.d_count = 0;
        return;
    }
    // this workgroup's tiles (at most 256)
    const uint32_t r0 = uint32_t(min<uint64_t>(A.n_tiles, uint64_t(blockIdx.x) * A.per));
    const uint32_t r1 = uint32_t(min<uint64_t>(A.n_tiles, uint64_t(r0) + A.per));
    if (r0 >= r1) return;
    const uint32_t nc = r1 - r0;
    // one round trip: this workgroup's counts, the range totals before it (if
    // kept) and the speculative slots
    const uint32_t mycnt = tid < nc ? A.counts[r0 + tid] : 0u;
    const uint64_t part = A.rsum ? prefix_part(A.rsum, blockIdx.x) : 0u;
    uint32_t spec[kSpecTiles];
#pragma unroll
    for (int k = 0; k < kSpecTiles; ++k) {
        const uint32_t j = wv + uint32_t(k) * (kBlock / kWave);
        spec[k] = j < nc ? A.slots[uint64_t(r0 + j) * kSlot + lane] : 0u;
    }
    uint32_t range_total;
    const uint32_t myoff = block_exclusive_scan(mycnt, lds_w, &range_total);
    cnt[tid] = mycnt;
    off[tid] = myoff;
    lds_barrier();
    const bool last = r1 == A.n_tiles;
    if (range_total == 0u && !last) return;   // nothing to write, and no total to report
    const int64_t prefix = int64_t(block_sum64(A.rsum ? part : counts_part(A.counts, r0), lds_s));
    uint32_t *st32 = stage[wv];
    uint16_t *st = reinterpret_cast<uint16_t *>(st32);
    uint32_t k = 0;
    for (uint32_t j = wv; j < nc; j += kBlock / kWave, ++k) {
        const uint32_t c = cnt[j];
        if (c == 0u) continue;
        const uint32_t t = r0 + j;
        const uint64_t tile_lo = uint64_t(t) * A.tile;
        int64_t base = prefix + off[j];
        if (c <= kWave && k < uint32_t(kSpecTiles)) {
            uint32_t sv = spec[0];
#pragma unroll
            for (int u = 1; u < kSpecTiles; ++u)
                if (k == uint32_t(u)) sv = spec[u];
            if (lane < c && base + lane < A.cap) A.out[base + lane] = int64_t(tile_lo + sv);
            continue;
        }
        if (c <= kSlot) {
            for (uint32_t o = lane; o < c; o += kWave)
                if (base + o < A.cap) A.out[base + o] = int64_t(tile_lo + A.slots[uint64_t(t) * kSlot + o]);
            continue;
        }
        const uint32_t S = uint32_t(min<uint64_t>(A.tile, A.starts - tile_lo));
        const uint32_t words = (S + 31u) / 32u;   // words past these may be stale
        const uint32_t *sb = A.spill + uint64_t(t) * tile_words;
        if (c <= kStageTile && words <= kWave * kLaneWords) {
            // one pass: lane l owns the R consecutive words from l * R, so one
            // scan orders the whole tile
            const uint32_t R = (words + kWave - 1u) / kWave, w0 = lane * R;
            uint32_t v[kLaneWords], pc = 0;
#pragma unroll
            for (int k = 0; k < kLaneWords; ++k) {
                const uint32_t i = w0 + uint32_t(k);
                v[k] = uint32_t(k) < R && i < words ? sb[i] : 0u;
                pc += __popc(v[k]);
            }
            uint32_t e = wave_inclusive_sum(pc) - pc;
#pragma unroll
            for (int k = 0; k < kLaneWords; ++k) {
                uint32_t b = v[k];
                while (b) {
                    if (e < kStageTile) st32[e] = (w0 + uint32_t(k)) * 32u + uint32_t(__builtin_ctz(b));
                    ++e;
                    b &= b - 1u;
                }
            }
            wave_lds_sync();
            for (uint32_t o = lane; o < c; o += kWave)
                if (base + o < A.cap) A.out[base + o] = int64_t(tile_lo + st32[o]);
            wave_lds_sync();   // read before the next tile writes
            continue;
        }
        for (uint32_t w0 = 0; w0 < words && base < A.cap; w0 += kEmitRounds * kWave) {
            uint32_t v[kEmitRounds];
#pragma unroll
            for (int k = 0; k < kEmitRounds; ++k) {
                const uint32_t i = w0 + uint32_t(k) * kWave + lane;
                v[k] = i < words ? sb[i] : 0u;
            }
#pragma unroll
            for (int k = 0; k < kEmitRounds; ++k) {
                const uint32_t pc = __popc(v[k]);
                const uint32_t incl = wave_inclusive_sum(pc);
                const uint32_t tot = __builtin_amdgcn_readlane(incl, kWave - 1);
                if (tot == 0u) continue;
                uint32_t e = incl - pc, b = v[k];
                while (b) {
                    st[e++] = uint16_t(lane * 32u + uint32_t(__builtin_ctz(b)));
                    b &= b - 1u;
                }
                wave_lds_sync();
                const uint64_t lo = tile_lo + uint64_t(w0 + uint32_t(k) * kWave) * 32u;
                for (uint32_t o = lane; o < tot; o += kWave)
                    if (base + o < A.cap) A.out[base + o] = int64_t(lo + st[o]);
                wave_lds_sync();   // read before the next round writes
                base += tot;
            }
        }
    }
    if (last && tid == 0) *A.d_count = prefix + range_total;
}

// ----------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------

using KernelFn = void (*)(SearchArgs);

// Look-ahead of the search loop: with short shifts most attempts are cheap
// and independent, so several are fetched together.
static int lookahead_for(uint32_t shift) { return shift <= 12 ? 4 : 1; }

template <int Q, typename WT>
static KernelFn pick_sched(int sched, int K) {
    if (sched == HC_SCHED_WAVE) return hc_search_kernel<Q, WT, HC_SCHED_WAVE, 1>;
    if (sched == kSchedShc) return hc_search_kernel<Q, WT, kSchedShc, 1>;
    // dense: one instance per number of links per window (0 for any q,
    // 1..3 for q <= 4)
    if (sched == HC_SCHED_DENSE + 0) return hc_search_kernel<Q, WT, HC_SCHED_DENSE + 0, 1>;
    if constexpr (Q <= 4) {
        if (sched == HC_SCHED_DENSE + 1) return hc_search_kernel<Q, WT, HC_SCHED_DENSE + 1, 1>;
        if (sched == HC_SCHED_DENSE + 2) return hc_search_kernel<Q, WT, HC_SCHED_DENSE + 2, 1>;
        if (sched == HC_SCHED_DENSE + 3) return hc_search_kernel<Q, WT, HC_SCHED_DENSE + 3, 1>;
    }
    return K == 4 ? hc_search_kernel<Q, WT, HC_SCHED_SEGMENT, 4>
                  : hc_search_kernel<Q, WT, HC_SCHED_SEGMENT, 1>;
}

template <int Q>
static KernelFn pick_w(int w, int sched, int K) {
    switch (w) {
        case 8: return pick_sched<Q, uint8_t>(sched, K);
        case 16: return pick_sched<Q, uint16_t>(sched, K);
        case 32: return pick_sched<Q, uint32_t>(sched, K);
        default: return pick_sched<Q, uint64_t>(sched, K);
    }
}

static KernelFn pick_kernel(int q, int w, int sched, int K) {
    switch (q) {
        case 1: return pick_w<1>(w, sched, K);
        case 2: return pick_w<2>(w, sched, K);
        case 3: return pick_w<3>(w, sched, K);
        case 4: return pick_w<4>(w, sched, K);
        case 5: return pick_w<5>(w, sched, K);
        case 6: return pick_w<6>(w, sched, K);
        case 7: return pick_w<7>(w, sched, K);
        default: return pick_w<8>(w, sched, K);
    }
}

static int occupancy(KernelFn fn, uint32_t lds_bytes) {
    static std::mutex mu;
    static std::map<std::pair<void *, uint32_t>, int> cache;
    std::lock_guard<std::mutex> g(mu);
    auto key = std::make_pair(reinterpret_cast<void *>(fn), lds_bytes);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(fn), kBlock,
                                                     lds_bytes) != hipSuccess)
        nb = 1;
    nb = std::max(1, nb);
    cache[key] = nb;
    return nb;
}

template <int Q>
static KernelFn pick_sparse_w(int w) {
    switch (w) {
        case 8: return hc_sparse_kernel<Q, uint8_t>;
        case 16: return hc_sparse_kernel<Q, uint16_t>;
        case 32: return hc_sparse_kernel<Q, uint32_t>;
        default: return hc_sparse_kernel<Q, uint64_t>;
    }
}

static KernelFn pick_sparse(int q, int w) {
    switch (q) {
        case 1: return pick_sparse_w<1>(w);
        case 2: return pick_sparse_w<2>(w);
        case 3: return pick_sparse_w<3>(w);
        case 4: return pick_sparse_w<4>(w);
        case 5: return pick_sparse_w<5>(w);
        case 6: return pick_sparse_w<6>(w);
        case 7: return pick_sparse_w<7>(w);
        default: return pick_sparse_w<8>(w);
    }
}

// Grid of the ordered output and its tiles per workgroup: four workgroups
// per compute unit (measured best on dense outputs, equal on sparse ones),
// at most 256 tiles each (one count per thread), no workgroup without tiles.
static void emit_shape(uint32_t n_tiles, uint32_t *grid, uint32_t *per) {
    const DeviceInfo &di = device_info();
    const uint64_t n = std::max<uint32_t>(n_tiles, 1u);
    const uint64_t g0 = std::max<uint64_t>((n + kBlock - 1) / kBlock, std::min<uint64_t>(n, uint64_t(di.cus) * 4u));
    *per = uint32_t((n + g0 - 1) / g0);
    *grid = uint32_t((n + *per - 1) / *per);
}

static hc_status launch_emit(uint32_t n_tiles, uint32_t tile, uint64_t starts, uint32_t grid, uint32_t per,
                             const TileScratch &ts, int64_t *d_out, int64_t cap, int64_t *d_count,
                             hipStream_t stream);

// Layout of the per-tile results of one call in one region: counts, then
// the slot lists, then the spilled bitmaps, each part 256-byte aligned.
// Returns the region's size in bytes.
static uint64_t tile_scratch_layout(uint32_t n_tiles, uint32_t tile, uint64_t *slots_off, uint64_t *spill_off) {
    const uint64_t t = std::max<uint32_t>(n_tiles, 1u);
    *slots_off = (t * 4u + 255u) & ~uint64_t(255);
    *spill_off = *slots_off + ((t * kSlot * 4u + 255u) & ~uint64_t(255));
    return *spill_off + t * (tile / 32u) * 4u;
}

// Per-tile results of one call: the stream's workspace (locked in *held until
// the call's two kernels are enqueued), or, when `fixed` is set, the caller's
// region of `fixed_bytes` bytes (HC_EINVAL when the call needs more). Range
// totals come only with the workspace, for emit grids of at most kRsumCap
// workgroups: its two arrays alternate between the calls on its stream (a
// call adds into one and its emit kernel clears the other for the next
// call), which a captured and replayed call could not do, so the fixed
// region goes without them.
static hc_status tile_scratch(hipStream_t stream, uint32_t n_tiles, uint32_t tile, uint32_t emit_grid,
                              void *fixed, uint64_t fixed_bytes, TileScratch *ts,
                              std::unique_lock<std::mutex> *held) {
    if (fixed) {
        uint64_t so = 0, po = 0;
        if (tile_scratch_layout(n_tiles, tile, &so, &po) > fixed_bytes) return HC_EINVAL;
        uint8_t *b = static_cast<uint8_t *>(fixed);
        *ts = TileScratch{reinterpret_cast<uint32_t *>(b), nullptr, nullptr, reinterpret_cast<uint32_t *>(b + so),
                          reinterpret_cast<uint32_t *>(b + po), nullptr};
        return HC_OK;
    }
    Workspace *ws = nullptr;
    const hc_status st = workspace_for(stream, std::max<uint32_t>(n_tiles, 1u), tile, &ws, held);
    if (st != HC_OK) return st;
    *ts = TileScratch{ws->counts, nullptr, nullptr, ws->slots, ws->spill};
    if (n_tiles > 0 && emit_grid <= kRsumCap) {
        ts->rsum = ws->rsum + ws->parity * kRsumCap;
        ts->rsum_next = ws->rsum + (1 - ws->parity) * kRsumCap;
        ts->parity = &ws->parity;   // flipped once both kernels are enqueued
    }
    return HC_OK;
}

// Sparse variant: tiles of 256 * segment window starts (segment 0 = 1024),
// no text staging; the same emit kernel as the streaming path.
static hc_status launch_sparse(const hc_pattern *p, const DeviceCopy &dc, const uint8_t *d_y, int64_t n,
                               int64_t *d_out, int64_t cap, int64_t *d_count, const hc_launch &lc,
                               hipStream_t stream, void *fixed, uint64_t fixed_bytes) {
    const PatternData &pd = p->data;
    const DeviceInfo &di = device_info();
    const uint32_t m = uint32_t(pd.m);
    const uint32_t table_bytes = uint32_t(pd.F.size() * (pd.w / 8));
    const uint64_t starts = n >= pd.m ? uint64_t(n - pd.m + 1) : 0;
    uint32_t seg = lc.segment > 0 ? std::min<uint32_t>(uint32_t(lc.segment), 4096u) : 1024u;
    seg = std::max<uint32_t>(seg, 32u);
    // A lane tries its starts one shift (m - q + 1) apart while words are
    // empty, so a range of k whole shifts costs k attempts, as in the
    // sequential scan; any other length costs one attempt more per lane
    // (at m = 1024, a segment of 1024 starts takes two attempts where one
    // covers 1018). The segment is rounded to the nearest multiple.
    const uint32_t shift = m - uint32_t(pd.q) + 1u;
    const bool whole = shift >= 32u && shift <= 4096u;
    if (whole) seg = std::min<uint32_t>(std::max<uint32_t>(1u, (seg + shift / 2u) / shift), 4096u / shift) * shift;
    SparseLayout L = sparse_layout(kBlock * seg, m, table_bytes);
    while (L.total > di.max_lds_per_block && seg > 32) {
        seg = whole && seg >= 2u * shift ? seg - shift : seg / 2u;
        L = sparse_layout(kBlock * seg, m, table_bytes);
    }
    if (L.total > di.max_lds_per_block) return HC_EINVAL;
    const uint32_t tile = kBlock * seg;
    const uint64_t n_tiles64 = (starts + tile - 1) / tile;
    if (n_tiles64 > 0xFFFFFFFFull) return HC_EINVAL;
    const uint32_t n_tiles = uint32_t(n_tiles64);
    uint32_t emit_grid = 1, emit_per = 1;
    emit_shape(n_tiles, &emit_grid, &emit_per);
    TileScratch ts;
    std::unique_lock<std::mutex> held;   // until both kernels are enqueued
    hc_status st = tile_scratch(stream, n_tiles, tile, emit_grid, fixed, fixed_bytes, &ts, &held);
    if (st != HC_OK) return st;
    KernelFn fn = pick_sparse(pd.q, pd.w);
    // no staging to overlap across tiles: one tile per workgroup, unless the
    // caller caps workgroups per compute unit
    int64_t groups = 65535;
    if (lc.wg_per_cu > 0) groups = int64_t(di.cus) * std::min(occupancy(fn, L.total), int(lc.wg_per_cu));
    const uint32_t grid = uint32_t(std::max<int64_t>(1, std::min<int64_t>(n_tiles, groups)));
    SearchArgs A;
    A.y = d_y;
    A.n = uint64_t(n);
    A.x = dc.d_x;
    A.F = dc.d_F;
    A.m = m;
    A.q = uint32_t(pd.q);
    A.s = uint32_t(pd.s);
    A.mask = pd.mask;
    A.hv = pd.hv;
    A.table_bytes = table_bytes;
    A.tile = tile;
    A.seg = seg;
    A.starts = starts;
    A.n_tiles = n_tiles;
    A.emit_per = emit_per;
    A.out = d_out;
    A.cap = cap;
    A.d_count = d_count;
    A.counts = ts.counts;
    A.rsum = ts.rsum;
    A.slots = ts.slots;
    A.spill = ts.spill;
    if (n_tiles > 0) {
        hipLaunchKernelGGL(fn, dim3(grid), dim3(kBlock), L.total, stream, A);
        if (hipGetLastError() != hipSuccess) return HC_EHIP;
    }
    return launch_emit(n_tiles, tile, starts, emit_grid, emit_per, ts, d_out, cap, d_count, stream);
}

hc_status launch_single(const hc_pattern *p, const DeviceCopy &dc, const uint8_t *d_y, int64_t n,
                        int64_t *d_out, int64_t cap, int64_t *d_count, const hc_launch &lc,
                        hipStream_t stream, void *fixed, uint64_t fixed_bytes) {
    const PatternData &pd = p->data;
    const DeviceInfo &di = device_info();
    const uint32_t m = uint32_t(pd.m);
    const uint64_t starts = n >= pd.m ? uint64_t(n - pd.m + 1) : 0;

    if (lc.variant == HC_VARIANT_SPARSE)
        return launch_sparse(p, dc, d_y, n, d_out, cap, d_count, lc, stream, fixed, fixed_bytes);
    const bool shc = lc.variant == HC_VARIANT_SENTINEL;
    // the dense test without links never reads F (it compares the window-end
    // hash with H_v): a large table (the one-to-one hash of m = q = 2 has
    // 64 KiB) stays out of LDS; small ones are copied as everywhere else
    // (leaving them out raised occupancy and measured 2-7 % slower)
    const uint32_t full_table = uint32_t(pd.F.size() * (pd.w / 8));
    const bool no_table = !shc && lc.schedule == HC_SCHED_DENSE && int64_t(m) < 2 * int64_t(pd.q) &&
                          full_table > 16384u;
    const uint32_t table_bytes = no_table ? 0u : full_table;
    const uint32_t extra = shc ? m : 0u;   // room for the sentinel copy of x
    uint32_t seg = std::min<uint32_t>(uint32_t(lc.segment), 256u);
    LdsLayout L = lds_layout(kBlock * seg, m, table_bytes, extra);
    while (L.total > di.max_lds_per_block && seg > 8) {
        seg = std::max<uint32_t>(8, seg / 2);
        L = lds_layout(kBlock * seg, m, table_bytes, extra);
    }
    // the dense schedule is instantiated for patterns without links (any
    // q) and for q <= 4 with up to 3 links per window; other patterns run
    // the searching loop
    int sched = shc ? kSchedShc : lc.schedule;
    if (sched == HC_SCHED_DENSE) {
        const int links = int(m) / pd.q - 1;
        sched = (links == 0 || (pd.q <= 4 && links <= 3)) ? HC_SCHED_DENSE + links : HC_SCHED_SEGMENT;
    }
    const int chunks = sched >= HC_SCHED_DENSE && sched < kSchedShc ? dense_chunks(pd.q) : kStageMax;
    while (kBlock * seg + m - 1u > stage_limit(kBlock, chunks) && seg > 8) seg -= 4;
    if (L.total > di.max_lds_per_block || kBlock * seg + m - 1u > stage_limit(kBlock, chunks)) return HC_EINVAL;
    L = lds_layout(kBlock * seg, m, table_bytes, extra);
    const uint32_t tile = kBlock * seg;
    const uint64_t n_tiles64 = (starts + tile - 1) / tile;
    if (n_tiles64 > 0xFFFFFFFFull) return HC_EINVAL;
    const uint32_t n_tiles = uint32_t(n_tiles64);

    uint32_t emit_grid = 1, emit_per = 1;
    emit_shape(n_tiles, &emit_grid, &emit_per);
    TileScratch ts;
    std::unique_lock<std::mutex> held;   // until both kernels are enqueued
    hc_status st = tile_scratch(stream, n_tiles, tile, emit_grid, fixed, fixed_bytes, &ts, &held);
    if (st != HC_OK) return st;

    KernelFn fn = pick_kernel(pd.q, pd.w, sched, lookahead_for(m - uint32_t(pd.q) + 1u));
    int per_cu = occupancy(fn, L.total);
    if (lc.wg_per_cu > 0) per_cu = std::min(per_cu, int(lc.wg_per_cu));
    const uint32_t grid = uint32_t(std::max<int64_t>(1, std::min<int64_t>(n_tiles, int64_t(di.cus) * per_cu)));

    SearchArgs A;
    A.y = d_y;
    A.n = uint64_t(n);
    A.x = dc.d_x;
    A.F = dc.d_F;
    A.m = m;
    A.q = uint32_t(pd.q);
    A.s = uint32_t(pd.s);
    A.mask = pd.mask;
    A.hv = pd.hv;
    A.table_bytes = table_bytes;
    A.tile = tile;
    A.seg = seg;
    A.starts = starts;
    A.n_tiles = n_tiles;
    A.emit_per = emit_per;
    A.out = d_out;
    A.cap = cap;
    A.d_count = d_count;
    A.counts = ts.counts;
    A.rsum = ts.rsum;
    A.slots = ts.slots;
    A.spill = ts.spill;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kBlock), L.total, stream, A);
    if (hipGetLastError() != hipSuccess) return HC_EHIP;

    return launch_emit(n_tiles, tile, starts, emit_grid, emit_per, ts, d_out, cap, d_count, stream);
}

static hc_status launch_emit(uint32_t n_tiles, uint32_t tile, uint64_t starts, uint32_t grid, uint32_t per,
                             const TileScratch &ts, int64_t *d_out, int64_t cap, int64_t *d_count,
                             hipStream_t stream) {
    EmitArgs E;
    E.n_tiles = n_tiles;
    E.tile = tile;
    E.per = per;
    const uint32_t emit_grid = grid;
    E.starts = starts;
    E.counts = ts.counts;
    E.rsum = ts.rsum;
    E.rsum_next = ts.rsum_next;
    E.slots = ts.slots;
    E.spill = ts.spill;
    E.out = d_out;
    E.cap = cap;
    E.d_count = d_count;
    hipLaunchKernelGGL(hc_emit_kernel, dim3(emit_grid), dim3(kBlock), 0, stream, E);
    if (hipGetLastError() != hipSuccess) return HC_EHIP;
    if (ts.parity) *ts.parity = 1 - *ts.parity;   // still under the workspace's lock
    return HC_OK;
}

}  // namespace hc

// ----------------------------------------------------------------------------
// hc_search_async_noalloc: the same two kernels with their per-tile results
// in a fixed device array instead of the per-stream workspace.
// ----------------------------------------------------------------------------

namespace hc {

// Bytes of the fixed array: per-tile results of texts up to about 420 MiB at
// the default tile shapes ((4 + 4 * kSlot + tile / 8) bytes per tile).
constexpr uint64_t kNoallocScratchBytes = uint64_t(64) << 20;

// One copy per device, held until the process ends. Host code never passes
// this name to a kernel: it stands for a host-side symbol, not the device
// address; the address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current device (looked up on the first
// call per device, with that device current).
static hc_status noalloc_scratch(void **out) {
    static std::mutex mu;
    static void *ptrs[kMaxDevices] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HC_EHIP;
    std::lock_guard<std::mutex> g(mu);
    if (!ptrs[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HC_EHIP;
        ptrs[dev] = p;
    }
    *out = ptrs[dev];
    return HC_OK;
}

}  // namespace hc

extern "C" hc_status hc_search_async_noalloc(const hc_pattern *pc, const uint8_t *d_y, int64_t n,
                                             int64_t *d_out, int64_t cap, int64_t *d_count,
                                             const hc_launch *launch, void *stream) {
    using namespace hc;
    if (!pc || !d_count || n < 0 || cap < 0 || (cap > 0 && !d_out)) return HC_EINVAL;
    if (n > 0 && !d_y) return HC_EINVAL;
    if (n > int64_t(0xFFFFFFFFll)) return HC_EINVAL;
    if (launch && (launch->segment < 0 || launch->segment > 4096 || launch->schedule < 0 ||
                   launch->schedule > HC_SCHED_DENSE || launch->variant < 0 ||
                   launch->variant > HC_VARIANT_SPARSE || launch->wg_per_cu < 0 || launch->wg_per_cu > 8))
        return HC_EINVAL;
    if (!device_info().ok) return HC_EHIP;
    hc_pattern *p = const_cast<hc_pattern *>(pc);
    const DeviceCopy *dc = pattern_resident(p);
    if (!dc) return HC_EINVAL;   // not uploaded to this device yet (that would allocate)
    void *fixed = nullptr;
    const hc_status st = noalloc_scratch(&fixed);
    if (st != HC_OK) return st;
    const hc_launch lc = choose_launch(p->data, n, launch);
    return launch_single(p, *dc, d_y, n, d_out, cap, d_count, lc, hipStream_t(stream), fixed,
                         kNoallocScratchBytes);
}
