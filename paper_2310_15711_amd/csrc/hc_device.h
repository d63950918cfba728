// Device-side building blocks of the HC searching phase on gfx950.
//
// Text is staged per tile into LDS; the word vector F and the pattern x sit in
// LDS for the whole launch. Each lane runs the searching loop of Section 3.3
// over its share of window starts and marks occurrences in an LDS bitmap; the
// bitmap is then compacted into ascending int64 positions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hc {

constexpr int kWave = 64;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------------------
// LDS layout of one workgroup (bytes, every region 16-byte aligned)
// ----------------------------------------------------------------------------
struct LdsLayout {
    uint32_t text_off, text_bytes;   // 16 pad + chunks + 16 pad (+ sentinel copy)
    uint32_t bitmap_off, bitmap_bytes;
    uint32_t table_off, table_bytes;
    uint32_t x_off, x_bytes;
    uint32_t misc_off, misc_bytes;
    uint32_t total;
};

__host__ __device__ inline uint32_t align16(uint32_t v) { return (v + 15u) & ~15u; }

// Chunks of 16 bytes needed to stage `span` bytes that start at any alignment.
__host__ __device__ inline uint32_t chunks_for(uint32_t span) { return (span + 15u) / 16u + 1u; }

// tile: window starts per tile; halo: m - 1; extra: bytes appended after the
// staged text (a sentinel copy of x, or 0).
__host__ __device__ inline LdsLayout lds_layout(uint32_t tile, uint32_t m, uint32_t table_bytes,
                                                uint32_t extra) {
    LdsLayout L;
    L.text_off = 0;
    L.text_bytes = 16u + 16u * chunks_for(tile + m - 1u) + align16(extra) + 16u;
    L.bitmap_off = L.text_off + L.text_bytes;
    L.bitmap_bytes = align16(tile / 8u);
    L.table_off = L.bitmap_off + L.bitmap_bytes;
    L.table_bytes = align16(table_bytes);
    L.x_off = L.table_off + L.table_bytes;
    L.x_bytes = align16(m) + 16u;
    L.misc_off = L.x_off + L.x_bytes;
    L.misc_bytes = 128u;
    L.total = L.misc_off + L.misc_bytes;
    return L;
}

// ----------------------------------------------------------------------------
// Hash of the q-gram that ends at LDS byte position e (equation (3)):
// h = sum_k u[k] * 2^(s*k) mod 2^alpha, u[0] the leftmost character.
// The q <= 8 bytes are fetched as aligned dwords and funnel-shifted.
// ----------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ uint32_t qgram_hash(const uint32_t *__restrict__ t32, uint32_t e,
                                               uint32_t s, uint32_t mask) {
    uint32_t v = 0;
    if constexpr (Q <= 4) {
        const uint32_t p = e - 3u;
        const uint32_t a = p >> 2, sh = p & 3u;
        const uint32_t w = __builtin_amdgcn_alignbyte(t32[a + 1], t32[a], sh);  // bytes p..p+3
#pragma unroll
        for (int k = Q - 1; k >= 0; --k)
            v = (v << s) + __builtin_amdgcn_ubfe(w, 8 * (4 - Q + k), 8);
    } else {
        const uint32_t p = e - 7u;
        const uint32_t a = p >> 2, sh = p & 3u;
        const uint32_t d0 = t32[a], d1 = t32[a + 1], d2 = t32[a + 2];
        const uint32_t lo = __builtin_amdgcn_alignbyte(d1, d0, sh);   // bytes p..p+3
        const uint32_t hi = __builtin_amdgcn_alignbyte(d2, d1, sh);   // bytes p+4..p+7
#pragma unroll
        for (int k = Q - 1; k >= 0; --k) {
            const int b = 8 - Q + k;   // byte index within p..p+7
            const uint32_t c = b < 4 ? __builtin_amdgcn_ubfe(lo, 8 * b, 8)
                                     : __builtin_amdgcn_ubfe(hi, 8 * (b - 4), 8);
            v = (v << s) + c;
        }
    }
    return v & mask;
}

// Link test of equation (5): bit (v mod w) of word z.
template <typename WT>
__device__ __forceinline__ bool linked(WT z, uint32_t v) {
    constexpr uint32_t wbits = sizeof(WT) * 8u;
    return (z >> (v & (wbits - 1u))) & 1u;
}

// Compare the m bytes at LDS byte position a of the text with x (LDS).
__device__ __forceinline__ bool window_equals(const uint8_t *__restrict__ t8, uint32_t a,
                                              const uint8_t *__restrict__ x8, uint32_t m) {
    for (uint32_t k = 0; k < m; ++k)
        if (t8[a + k] != x8[k]) return false;
    return true;
}

// Parameters of one pattern as seen by a kernel.
struct PatternView {
    uint32_t m, q, s, mask, hv;
};

// One attempt of the searching phase at window end J (LDS byte position of
// the window's last character is tb + J). Returns the next window end. When
// every q-gram of the window links and the last hash equals H_v, the window
// is compared with x and, if equal, *hit is set.
template <int Q, typename WT>
__device__ __forceinline__ uint32_t hc_attempt(const uint32_t *__restrict__ t32,
                                               const uint8_t *__restrict__ t8, uint32_t tb,
                                               const WT *__restrict__ F,
                                               const uint8_t *__restrict__ x8,
                                               const PatternView &P, uint32_t J, bool *hit) {
    uint32_t v = qgram_hash<Q>(t32, tb + J, P.s, P.mask);
    WT z = F[v];
    const uint32_t shift = P.m - Q + 1u;
    if (z == 0) return J + shift;            // no q-gram of x hashes here
    int32_t e = int32_t(J);
    const int32_t lo = int32_t(J) - int32_t(P.m) + 2 * Q;
    while (e >= lo) {                        // a whole q-gram still fits before e
        e -= Q;
        v = qgram_hash<Q>(t32, tb + uint32_t(e), P.s, P.mask);
        if (!linked(z, v)) return uint32_t(e) + shift;   // u_p u is not a factor
        z = F[v];
    }
    // every q-gram of the window is linked: candidate
    if (v == P.hv && window_equals(t8, tb + J + 1u - P.m, x8, P.m)) *hit = true;
    return J + 1u;
}

// Searching loop over window ends [jlo, jhi) (tile-relative), one lane.
// Marks the start of each occurrence in the tile bitmap.
template <int Q, typename WT>
__device__ __forceinline__ void hc_segment(const uint32_t *__restrict__ t32,
                                           const uint8_t *__restrict__ t8, uint32_t tb,
                                           const WT *__restrict__ F,
                                           const uint8_t *__restrict__ x8, const PatternView &P,
                                           uint32_t jlo, uint32_t jhi, uint32_t *bitmap) {
    uint32_t J = jlo;
    const uint32_t shift = P.m - Q + 1u;
    while (J < jhi) {
        // fast path: empty word, shift by m - q + 1
        const uint32_t v = qgram_hash<Q>(t32, tb + J, P.s, P.mask);
        if (F[v] == 0) {
            J += shift;
            continue;
        }
        bool hit = false;
        const uint32_t next = hc_attempt<Q, WT>(t32, t8, tb, F, x8, P, J, &hit);
        if (hit) {
            const uint32_t st = J + 1u - P.m;
            atomicOr(&bitmap[st >> 5], 1u << (st & 31u));
        }
        J = next;
    }
}

// Wavefront schedule over window starts [slo, shi) (tile-relative): the 64
// lanes try 64 consecutive windows; each attempt proves that no occurrence
// starts strictly between its own start and the start of its next window,
// so the wavefront may continue from the furthest such start (or 64 on).
template <int Q, typename WT>
__device__ __forceinline__ void hc_wave(const uint32_t *__restrict__ t32,
                                        const uint8_t *__restrict__ t8, uint32_t tb,
                                        const WT *__restrict__ F, const uint8_t *__restrict__ x8,
                                        const PatternView &P, uint32_t slo, uint32_t shi,
                                        uint32_t *bitmap, uint32_t lane) {
    uint32_t base = slo;
    while (base < shi) {
        const uint32_t st = base + lane;
        uint32_t next_start = 0;
        if (st < shi) {
            bool hit = false;
            const uint32_t J = st + P.m - 1u;
            const uint32_t nJ = hc_attempt<Q, WT>(t32, t8, tb, F, x8, P, J, &hit);
            if (hit) atomicOr(&bitmap[st >> 5], 1u << (st & 31u));
            next_start = nJ + 1u - P.m;
        }
        uint32_t far = next_start;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) far = max(far, (uint32_t)__shfl_xor((int)far, d, kWave));
        base = max(base + uint32_t(kWave), far);
    }
}

// ----------------------------------------------------------------------------
// Tile status words for the single-pass ordered compaction (decoupled
// look-back): [63:62] flag (1 = tile count, 2 = inclusive prefix),
// [61:32] launch generation, [31:0] value.
// ----------------------------------------------------------------------------
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPre = 2ull << 62;
constexpr uint32_t kGenMask = 0x3FFFFFFFu;

__device__ __forceinline__ uint64_t status_word(uint64_t flag, uint32_t gen, uint32_t value) {
    return flag | (uint64_t(gen & kGenMask) << 32) | value;
}

__device__ __forceinline__ uint64_t load_agent(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Polls of a predecessor's status before a look-back gives up (about a
// minute): every wait then ends, and the launch reports an error instead of
// hanging.
constexpr uint32_t kSpinLimit = 1u << 26;

// Exclusive prefix of tile `t` given its own count; run by one whole
// wavefront. Publishes the tile's count, then its inclusive prefix. Sets
// *err when a predecessor never published.
__device__ inline uint32_t lookback(uint64_t *status, uint32_t t, uint32_t gen, uint32_t count,
                                    uint32_t lane, uint32_t *err) {
    if (t == 0) {
        if (lane == 0) store_agent(&status[0], status_word(kFlagPre, gen, count));
        return 0;
    }
    if (lane == 0) store_agent(&status[t], status_word(kFlagAgg, gen, count));
    uint32_t excl = 0;
    int64_t k = int64_t(t) - 1;
    uint32_t spins = 0;
    while (true) {
        const int64_t idx = k - int64_t(lane);
        const uint64_t e = idx >= 0 ? load_agent(&status[idx]) : 0ull;
        const uint32_t fl = uint32_t(e >> 62);
        const bool valid = fl != 0 && uint32_t((e >> 32) & kGenMask) == (gen & kGenMask);
        const uint64_t bpre = __ballot(valid && fl == 2);
        const uint64_t binv = __ballot(!valid && idx >= 0);
        const int p = bpre ? __ffsll((unsigned long long)bpre) - 1 : 64;
        const uint64_t need = p >= 63 ? ~0ull : ((2ull << p) - 1ull);
        if (binv & need) {
            if (++spins > kSpinLimit) {
                if (lane == 0) __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint32_t val = (int(lane) <= p && idx >= 0) ? uint32_t(e) : 0u;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) val += (uint32_t)__shfl_xor((int)val, d, kWave);
        excl += val;
        if (p < 64) break;
        k -= kWave;
    }
    if (lane == 0) store_agent(&status[t], status_word(kFlagPre, gen, excl + count));
    return excl;
}

// Control block of one launch workspace (device memory, zero-initialised).
struct Ctl {
    uint32_t ticket;   // next tile ticket
    uint32_t done;     // workgroups finished
    uint32_t gen;      // launch generation
    uint32_t err;      // a look-back gave up during this launch
};

// Called by every workgroup (all threads) after its last tile: the last one to
// finish resets the counters and advances the generation; on wrap-around the
// status words are cleared so that no stale generation can match. A launch
// whose look-back gave up reports a total of -1.
__device__ inline void finish_launch(Ctl *ctl, uint64_t *status, uint32_t status_cap,
                                     uint32_t gen, uint32_t *lds_flag, int64_t *d_total) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t d = __hip_atomic_fetch_add(&ctl->done, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        *lds_flag = (d == gridDim.x - 1u) ? 1u : 0u;
    }
    __syncthreads();
    if (*lds_flag == 0u) return;
    const uint32_t ng = (gen + 1u) & kGenMask;
    if (ng == 0u) {
        for (uint32_t i = threadIdx.x; i < status_cap; i += blockDim.x) store_agent(&status[i], 0ull);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (__hip_atomic_exchange(&ctl->err, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u &&
            d_total)
            *d_total = -1;
        __hip_atomic_store(&ctl->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->gen, ng, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Stage bytes [g0, g1) of a text into LDS as aligned 16-byte chunks. Byte g0
// lands at LDS text position 16 + ((uintptr)(y + g0) & 15); returns that
// position. Every chunk read holds at least one byte of [g0, g1), so no read
// leaves the pages that hold the text.
__device__ __forceinline__ uint32_t stage_text(const uint8_t *y, uint64_t g0, uint64_t g1,
                                               uint8_t *lds_text) {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(y + g0);
    const uintptr_t p0 = a0 & ~uintptr_t(15);
    const uint32_t nch = uint32_t((reinterpret_cast<uintptr_t>(y + g1) - p0 + 15u) >> 4);
    const u32x4 *src = reinterpret_cast<const u32x4 *>(p0);
    u32x4 *dst = reinterpret_cast<u32x4 *>(lds_text + 16);
    constexpr int kUnroll = 8;
    for (uint32_t base = 0; base < nch; base += kUnroll * blockDim.x) {
        u32x4 r[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const uint32_t c = base + k * blockDim.x + threadIdx.x;
            if (c < nch) r[k] = __builtin_nontemporal_load(src + c);
        }
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const uint32_t c = base + k * blockDim.x + threadIdx.x;
            if (c < nch) dst[c] = r[k];
        }
    }
    return 16u + uint32_t(a0 - p0);
}

// Block-wide exclusive scan of one value per thread (blockDim = 256).
// Returns the thread's exclusive prefix; *total receives the block sum.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t c, uint32_t *lds_w,
                                                         uint32_t *total) {
    const uint32_t lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    uint32_t incl = c;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)incl, d, kWave);
        if (lane >= uint32_t(d)) incl += t;
    }
    if (lane == kWave - 1) lds_w[wid] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    const uint32_t nw = blockDim.x / kWave;
    for (uint32_t i = 0; i < nw; ++i) {
        const uint32_t v = lds_w[i];
        if (i < wid) before += v;
        all += v;
    }
    *total = all;
    return before + incl - c;
}

}  // namespace hc
