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
constexpr uint32_t kThreads = 256;   // threads per workgroup of the search kernels

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Workgroup barrier that orders LDS only. A plain __syncthreads() also waits
// for every outstanding global load (vmcnt(0) on gfx9), which would drain the
// prefetch of the next tile at each barrier; all cross-wave data here goes
// through LDS, so the LDS-scoped fences are sufficient.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ----------------------------------------------------------------------------
// LDS layout of one workgroup (bytes, every region 16-byte aligned)
// ----------------------------------------------------------------------------
struct LdsLayout {
    uint32_t text_off, text_bytes;   // 16 pad + chunks + 16 pad (+ sentinel copy)
    uint32_t bitmap_off, bitmap_bytes;
    uint32_t table_off, table_bytes;
    uint32_t x_off, x_bytes;
    uint32_t park_off, park_bytes;
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
    L.text_bytes = 16u + 16u * chunks_for(tile + m - 1u) + align16(extra) + 32u;
    L.bitmap_off = L.text_off + L.text_bytes;
    L.bitmap_bytes = align16(tile / 8u);
    L.table_off = L.bitmap_off + L.bitmap_bytes;
    L.table_bytes = align16(table_bytes);
    L.x_off = L.table_off + L.table_bytes;
    L.x_bytes = align16(m) + 32u;
    L.park_off = L.x_off + L.x_bytes;
    L.park_bytes = 32u * 24u;   // parked chain walks
    L.misc_off = L.park_off + L.park_bytes;
    L.misc_bytes = 128u;
    L.total = L.misc_off + L.misc_bytes;
    return L;
}

// Parameters of one pattern as seen by a kernel; wl0..wh1 are the byte
// weights of its hash (set by hash_weights).
struct PatternView {
    uint32_t m, q, s, mask, hv;
    uint32_t wl0 = 0, wl1 = 0, wh0 = 0, wh1 = 0;
};

// Byte weights of the hash of equation (3) for 4 x 8-bit dot products. The
// q-gram's character j (0 = leftmost) counts 2^(s j); qgram_hash reads the
// q-gram from the one (q <= 4) or two dwords that end with it, where
// character j sits at byte b = (q <= 4 ? 4 - q : 8 - q) + j. Weights below
// 2^8 go to wl (byte b of dword b / 4), the others divided by 2^8 to wh:
// s j <= alpha - s < 16 because alpha <= 16 (tables of at most 64 KiB).
// w = {wl0, wl1, wh0, wh1}.
__host__ __device__ inline void byte_weights(uint32_t q, uint32_t s, uint32_t w[4]) {
    w[0] = w[1] = w[2] = w[3] = 0u;
    const uint32_t base = q <= 4u ? 4u - q : 8u - q;
    for (uint32_t j = 0; j < q; ++j) {
        const uint32_t b = base + j, e = s * j, sh = 8u * (b & 3u);
        if (e < 8u)
            w[b >> 2] |= (1u << e) << sh;
        else
            w[2u + (b >> 2)] |= (1u << (e - 8u)) << sh;
    }
}

__device__ __forceinline__ PatternView hash_weights(PatternView P) {
    uint32_t w[4];
    byte_weights(P.q, P.s, w);
    P.wl0 = w[0];
    P.wl1 = w[1];
    P.wh0 = w[2];
    P.wh1 = w[3];
    return P;
}

// ----------------------------------------------------------------------------
// Hash of the q-gram that ends at LDS byte position e (equation (3)):
// h = sum_j u[j] * 2^(s*j) mod 2^alpha, u[0] the leftmost character. The
// q <= 8 bytes are fetched as aligned dwords and funnel-shifted; the sum is
// two dot products per dword (weights below and above 2^8).
// ----------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ uint32_t qgram_hash(const uint32_t *__restrict__ t32, uint32_t e,
                                               const PatternView &P) {
    if constexpr (Q == 1) {
        const uint32_t w = t32[e >> 2];
        return __builtin_amdgcn_ubfe(w, 8u * (e & 3u), 8) & P.mask;
    } else if constexpr (Q <= 4) {
        const uint32_t p = e - 3u;
        const uint32_t a = p >> 2, sh = p & 3u;
        const uint32_t w = __builtin_amdgcn_alignbyte(t32[a + 1], t32[a], sh);  // bytes p..p+3
        const uint32_t hi = __builtin_amdgcn_udot4(w, P.wh0, 0u, false);
        return __builtin_amdgcn_udot4(w, P.wl0, hi << 8, false) & P.mask;
    } else {
        const uint32_t p = e - 7u;
        const uint32_t a = p >> 2, sh = p & 3u;
        const uint32_t d0 = t32[a], d1 = t32[a + 1], d2 = t32[a + 2];
        const uint32_t lo = __builtin_amdgcn_alignbyte(d1, d0, sh);   // bytes p..p+3
        const uint32_t hi = __builtin_amdgcn_alignbyte(d2, d1, sh);   // bytes p+4..p+7
        const uint32_t t = __builtin_amdgcn_udot4(hi, P.wh1, __builtin_amdgcn_udot4(lo, P.wh0, 0u, false), false);
        return __builtin_amdgcn_udot4(hi, P.wl1, __builtin_amdgcn_udot4(lo, P.wl0, t << 8, false), false) & P.mask;
    }
}

// Link test of equation (5): bit (v mod w) of word z.
template <typename WT>
__device__ __forceinline__ bool linked(WT z, uint32_t v) {
    constexpr uint32_t wbits = sizeof(WT) * 8u;
    return (z >> (v & (wbits - 1u))) & 1u;
}

// Compare the m bytes at LDS byte position a of the text with x (LDS, 16-byte
// aligned and padded). Four bytes per step with sixteen bytes of each side
// in flight; bytes read past either end (within the LDS padding) are masked.
__device__ __forceinline__ bool window_equals(const uint32_t *__restrict__ t32, uint32_t a,
                                              const uint32_t *__restrict__ x32, uint32_t m) {
    const uint32_t sh = a & 3u, base = a >> 2;
    const uint32_t nw = (m + 3u) >> 2;
    const uint32_t tail = (m & 3u) ? ((1u << (8u * (m & 3u))) - 1u) : 0xFFFFFFFFu;
    uint32_t lo = t32[base];
    for (uint32_t i = 0; i < nw; i += 4) {
        uint32_t d[4], xw[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            d[j] = t32[base + i + j + 1];
            xw[j] = x32[i + j];
        }
        uint32_t diff = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t w = __builtin_amdgcn_alignbyte(d[j], j == 0 ? lo : d[j - 1], sh);
            uint32_t dj = w ^ xw[j];
            if (i + j + 1 == nw) dj &= tail;
            if (i + j < nw) diff |= dj;
        }
        if (diff) return false;
        lo = d[3];
    }
    return true;
}

// A chain walk that a lane has parked for its wavefront to finish: window end
// J, the end e of the last q-gram checked so far, its hash v and its word z.
struct Parked {
    uint32_t J, e, v, owner;   // owner: thread id * 2 + stream
    uint64_t z;
};
constexpr uint32_t kParkCap = 32;   // parked walks per workgroup and round
constexpr int kLocalSteps = 8;      // chain steps a lane takes before parking
// The same for walks read in place (sparse variant): each step there is a
// dependent global load, so the walk is handed to the wavefront (64 q-grams
// per load round) after one; the walk of a true occurrence crosses m / q
// links and sets the time of its tile.
constexpr int kSparseLocalSteps = 1;

// Outcome of an attempt: the next window end, or "parked".
constexpr uint32_t kParkedJ = 0xFFFFFFFFu;

// Chain walk of the searching phase for the window ending at J, from the
// q-gram ending at e (hash v, word z = F[v] != 0) towards the window start:
// the q-grams ending at e - q, e - 2q, ... are hashed while they stay inside
// the window; each must carry its link bit in the word of the q-gram after
// it. A broken link at the q-gram ending at e' moves the window end to
// e' + m - q + 1 (u_p u is not a factor of x). When every q-gram links and the
// last hash equals H_v the window is a candidate (*hit), compared with x in a
// later pass, and the window end moves by one. After `steps` links the walk is
// handed back (kParkedJ) with its position in (e, v, z).
template <int Q, typename WT>
__device__ __forceinline__ uint32_t hc_chain(const uint32_t *__restrict__ t32, uint32_t tb,
                                             const WT *__restrict__ F, const PatternView &P,
                                             uint32_t J, uint32_t &e, uint32_t &v, WT &z,
                                             int steps, bool *hit) {
    const uint32_t shift = P.m - Q + 1u;
    const int32_t lo = int32_t(J) - int32_t(P.m) + 2 * Q;
    while (int32_t(e) >= lo) {               // a whole q-gram still fits before e
        if (steps-- == 0) return kParkedJ;
        const uint32_t ep = e - Q;
        const uint32_t vp = qgram_hash<Q>(t32, tb + ep, P);
        if (!linked(z, vp)) return ep + shift;
        e = ep;
        v = vp;
        z = F[vp];
    }
    if (v == P.hv) *hit = true;              // every q-gram of the window links
    return J + 1u;
}

template <int Q, typename WT>
__device__ __forceinline__ uint32_t hc_attempt(const uint32_t *__restrict__ t32, uint32_t tb,
                                               const WT *__restrict__ F, const PatternView &P,
                                               uint32_t J, bool *hit) {
    uint32_t v = qgram_hash<Q>(t32, tb + J, P);
    WT z = F[v];
    if (z == 0) return J + P.m - Q + 1u;     // no q-gram of x hashes here
    uint32_t e = J;
    return hc_chain<Q, WT>(t32, tb, F, P, J, e, v, z, 1 << 30, hit);
}

__device__ __forceinline__ void mark(uint32_t *bitmap, uint32_t st, uint32_t *any) {
    atomicOr(&bitmap[st >> 5], 1u << (st & 31u));
    *any = 1u;
}

// Searching loop of one lane over window ends [J0, jmid) and [J1, jhi)
// (tile-relative), the two halves of its range searched side by side. Each
// half also looks K attempts ahead: the words of the q-grams ending at J,
// J + s, ..., J + (K-1) s (s = m - q + 1, the shift after an empty word) are
// fetched together, and the first non-empty one continues the search there
// (the attempts before it would each have shifted by s). Up to 2K LDS round
// trips are thus in flight per lane. Marks candidate window starts in the
// tile bitmap and sets *any. A chain walk longer than kLocalSteps is parked
// in `park` (capacity kParkCap, count *npark, slot *myslot) and the lane
// stops; it resumes after its wavefront has finished the walk. Returns false
// when the lane parked a walk.
template <int Q, typename WT, int K>
__device__ __forceinline__ bool hc_segment(const uint32_t *__restrict__ t32, uint32_t tb,
                                           const WT *__restrict__ F, const PatternView &P,
                                           uint32_t &J0, uint32_t jmid, uint32_t &J1, uint32_t jhi,
                                           uint32_t *bitmap, uint32_t *any, Parked *park,
                                           uint32_t *npark, uint32_t *myslot) {
    const uint32_t shift = P.m - Q + 1u;
    const uint32_t jsafe = J0 < jmid ? J0 : J1;   // a window end of this lane's range
    while (J0 < jmid || J1 < jhi) {
        uint32_t vv[2][K];
        WT zz[2][K];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t J = h == 0 ? J0 : J1, Jend = h == 0 ? jmid : jhi;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                // positions past the half's end read a window of the lane instead (unused)
                const uint32_t Jn = J + uint32_t(i) * shift;
                const uint32_t Ji = Jn < Jend ? Jn : jsafe;
                vv[h][i] = qgram_hash<Q>(t32, tb + Ji, P);
                zz[h][i] = F[vv[h][i]];
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint32_t &J = h == 0 ? J0 : J1;
            const uint32_t Jend = h == 0 ? jmid : jhi;
            if (J >= Jend) continue;
            int first = K;
#pragma unroll
            for (int i = K - 1; i >= 0; --i)
                if (zz[h][i] != 0 && J + uint32_t(i) * shift < Jend) first = i;
            if (first == K) {
                J += uint32_t(K) * shift;        // K empty words in a row
                continue;
            }
            uint32_t v = vv[h][0];
            WT z = zz[h][0];
#pragma unroll
            for (int i = 1; i < K; ++i)
                if (first == i) {
                    v = vv[h][i];
                    z = zz[h][i];
                }
            J += uint32_t(first) * shift;
            bool hit = false;
            uint32_t e = J;
            const uint32_t next = hc_chain<Q, WT>(t32, tb, F, P, J, e, v, z, kLocalSteps, &hit);
            if (next == kParkedJ) {
                const uint32_t slot = atomicAdd(npark, 1u);
                if (slot < kParkCap) {
                    park[slot] = Parked{J, e, v, threadIdx.x * 2u + uint32_t(h), uint64_t(z)};
                    *myslot = slot;
                    return false;
                }
                // no room: finish the walk here
                const uint32_t n2 = hc_chain<Q, WT>(t32, tb, F, P, J, e, v, z, 1 << 30, &hit);
                if (hit) mark(bitmap, J + 1u - P.m, any);
                J = n2;
                continue;
            }
            if (hit) mark(bitmap, J + 1u - P.m, any);
            J = next;
        }
    }
    return true;
}

// A whole wavefront finishes a parked chain walk: lane i hashes the q-gram
// that ends i + 1 steps further back and looks up its word, so 64 links are
// checked per round; a ballot finds the first broken one. Returns the next
// window end of the walk's window and marks it when it is a candidate.
// The walk itself, with the q-gram hash at a tile-relative end supplied by
// `hash` (text in LDS, or read in place from global memory).
template <int Q, typename WT, typename H>
__device__ __forceinline__ uint32_t chain_wave_impl(H hash, const WT *__restrict__ F, const PatternView &P,
                                                    const Parked &pk, uint32_t lane, uint32_t *bitmap,
                                                    uint32_t *any) {
    const uint32_t shift = P.m - Q + 1u;
    const int32_t lo = int32_t(pk.J) - int32_t(P.m) + 2 * Q;
    int32_t e = int32_t(pk.e);
    WT z = WT(pk.z);
    uint32_t v = pk.v;
    while (true) {
        // step i (1-based) checks the q-gram ending at e - i q; it exists when
        // the previous end e - (i - 1) q is still >= lo
        const int32_t step = int32_t(lane) + 1;
        const int32_t ei = e - step * Q;
        const bool valid = e - (step - 1) * Q >= lo;
        uint32_t vi = 0;
        WT zi = 0;
        if (valid) {
            vi = hash(uint32_t(ei));
            zi = F[vi];
        }
        // word of the q-gram after step i: step i - 1's word, or z for step 1
        WT zprev;
        if constexpr (sizeof(WT) == 8) {
            const uint32_t lo32 = (uint32_t)__shfl_up((int)uint32_t(zi), 1, kWave);
            const uint32_t hi32 = (uint32_t)__shfl_up((int)uint32_t(uint64_t(zi) >> 32), 1, kWave);
            zprev = WT((uint64_t(hi32) << 32) | lo32);
        } else {
            zprev = WT((uint32_t)__shfl_up((int)uint32_t(zi), 1, kWave));
        }
        if (lane == 0) zprev = z;
        const uint64_t broken = __ballot(valid && !linked(zprev, vi));
        if (broken) {
            const int f = __ffsll((unsigned long long)broken) - 1;
            return uint32_t(e - (f + 1) * Q) + shift;
        }
        const uint64_t vmask = __ballot(valid);
        if (vmask != ~0ull) {
            // the walk reached the window start inside this round
            const int last = vmask ? 63 - __clzll((long long)vmask) : -1;
            const uint32_t vl = last >= 0 ? (uint32_t)__shfl((int)vi, last, kWave) : v;
            if (vl == P.hv && lane == 0) mark(bitmap, pk.J + 1u - P.m, any);
            return pk.J + 1u;
        }
        // all 64 steps linked: continue from the last one
        v = (uint32_t)__shfl((int)vi, 63, kWave);
        if constexpr (sizeof(WT) == 8) {
            const uint32_t lo32 = (uint32_t)__shfl((int)uint32_t(zi), 63, kWave);
            const uint32_t hi32 = (uint32_t)__shfl((int)uint32_t(uint64_t(zi) >> 32), 63, kWave);
            z = WT((uint64_t(hi32) << 32) | lo32);
        } else {
            z = WT((uint32_t)__shfl((int)uint32_t(zi), 63, kWave));
        }
        e -= 64 * Q;
    }
}

template <int Q, typename WT>
__device__ __forceinline__ uint32_t hc_chain_wave(const uint32_t *__restrict__ t32, uint32_t tb,
                                                  const WT *__restrict__ F, const PatternView &P,
                                                  const Parked &pk, uint32_t lane,
                                                  uint32_t *bitmap, uint32_t *any) {
    return chain_wave_impl<Q, WT>([&](uint32_t e) { return qgram_hash<Q>(t32, tb + e, P); }, F, P, pk,
                                  lane, bitmap, any);
}

// Wavefront schedule over window starts [slo, shi) (tile-relative): the 64
// lanes try 64 consecutive windows; each attempt proves that no occurrence
// starts strictly between its own start and the start of its next window,
// so the wavefront may continue from the furthest such start (or 64 on).
template <int Q, typename WT>
__device__ __forceinline__ void hc_wave(const uint32_t *__restrict__ t32, uint32_t tb,
                                        const WT *__restrict__ F, const PatternView &P,
                                        uint32_t slo, uint32_t shi, uint32_t *bitmap,
                                        uint32_t lane, uint32_t *any) {
    uint32_t base = slo;
    while (base < shi) {
        const uint32_t st = base + lane;
        uint32_t next_start = 0;
        if (st < shi) {
            bool hit = false;
            const uint32_t J = st + P.m - 1u;
            const uint32_t nJ = hc_attempt<Q, WT>(t32, tb, F, P, J, &hit);
            if (hit) mark(bitmap, st, any);
            next_start = nJ + 1u - P.m;
        }
        uint32_t far = next_start;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) far = max(far, (uint32_t)__shfl_xor((int)far, d, kWave));
        base = max(base + uint32_t(kWave), far);
    }
}

// Staging of text bytes [g0, g1) into LDS as aligned 16-byte chunks, in two
// halves so that the loads of the next tile are in flight while the current
// tile is searched: stage_issue() loads into registers, stage_commit() stores
// them to LDS. Byte g0 lands at LDS text position 16 + ((uintptr)(y + g0) & 15)
// (returned by stage_issue). Every chunk read holds at least one byte of
// [g0, g1), so no read leaves the pages that hold the text.
// 16-byte chunks per thread held in registers while they travel: (tile +
// m - 1) <= 16 * 256 * kStageMax - 32. Seven (tiles up to 27.6 K starts for
// m = 1024) keep the kernels at 4-6 wavefronts per SIMD; ten cost each of
// them a wavefront per SIMD, worth more than larger tiles.
constexpr int kStageMax = 7;

// Dense-schedule kernels with q >= 3 hold five (tiles up to 20 K starts):
// they are the most VALU-bound and gain most from the extra wavefronts; with
// q <= 2 their loop is short enough that seven (larger tiles) measured 5-10 %
// faster, and 1 % slower at q = 3.
constexpr int kStageDense = 5;
__host__ __device__ constexpr int dense_chunks(int q) { return q <= 2 ? kStageMax : kStageDense; }

template <int N = kStageMax>
struct Stage {
    u32x4 r[N];
    uint32_t nch;
};

__host__ __device__ inline uint32_t stage_limit(uint32_t threads, int chunks = kStageMax) {
    return 16u * threads * uint32_t(chunks) - 32u;
}

typedef const __attribute__((address_space(1))) u32x4 global_u32x4;

template <int N>
__device__ __forceinline__ uint32_t stage_issue(const uint8_t *y, uint64_t g0, uint64_t g1, Stage<N> &st) {
    const uint8_t *a = y + g0;
    const uint32_t mis = uint32_t(reinterpret_cast<uintptr_t>(a) & 15u);
    st.nch = (mis + uint32_t(g1 - g0) + 15u) >> 4;
    // global address space: flat loads would also count against the LDS
    // counter and make every LDS barrier wait for this prefetch
    global_u32x4 *src = (global_u32x4 *)(a - mis);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const uint32_t c = k * 256u + threadIdx.x;   // 256 threads per workgroup
        if (c < st.nch) st.r[k] = __builtin_nontemporal_load(src + c);
    }
    return 16u + mis;
}

template <int N>
__device__ __forceinline__ void stage_commit(const Stage<N> &st, uint8_t *lds_text) {
    u32x4 *dst = reinterpret_cast<u32x4 *>(lds_text + 16);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const uint32_t c = k * 256u + threadIdx.x;   // 256 threads per workgroup
        if (c < st.nch) dst[c] = st.r[k];
    }
}

// ----------------------------------------------------------------------------
// Text read in place from global memory (the sparse variant): only the
// aligned dwords that hold bytes of a hashed q-gram or of a verified window
// are loaded. A dword that holds no byte of the text reads as 0 without a
// load, so nothing outside the text's pages is touched.
// ----------------------------------------------------------------------------
typedef const __attribute__((address_space(1))) uint32_t global_u32;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef u32x2 u32x2_a4 __attribute__((aligned(4)));
typedef u32x3 u32x3_a4 __attribute__((aligned(4)));
typedef const __attribute__((address_space(1))) u32x2_a4 global_u32x2_a4;
typedef const __attribute__((address_space(1))) u32x3_a4 global_u32x3_a4;

struct GlobalText {
    uintptr_t lo, hi;   // the text's bytes are [lo, hi) (absolute addresses)
};

__device__ __forceinline__ uint32_t gdword(const GlobalText &T, uintptr_t d) {
    return (d + 4u > T.lo && d < T.hi) ? *(global_u32 *)d : 0u;
}

// Hash (eq. (3)) of the q-gram that ends at absolute address e. The aligned
// dwords holding it are read with one load when each of them holds a text
// byte (everywhere but at the text's two ends), else one by one.
template <int Q>
__device__ __forceinline__ uint32_t ghash(const GlobalText &T, uintptr_t e, uint32_t s, uint32_t mask) {
    uint32_t v = 0;
    if constexpr (Q <= 4) {
        const uintptr_t p = e - 3u, a = p & ~uintptr_t(3);
        uint32_t d0, d1;
        if (a + 4u > T.lo && a + 4u < T.hi) {
            const u32x2 d = *(global_u32x2_a4 *)a;
            d0 = d.x;
            d1 = d.y;
        } else {
            d0 = gdword(T, a);
            d1 = gdword(T, a + 4u);
        }
        const uint32_t w = __builtin_amdgcn_alignbyte(d1, d0, uint32_t(p & 3u));
#pragma unroll
        for (int k = Q - 1; k >= 0; --k) v = (v << s) + __builtin_amdgcn_ubfe(w, 8 * (4 - Q + k), 8);
    } else {
        const uintptr_t p = e - 7u, a = p & ~uintptr_t(3);
        const uint32_t sh = uint32_t(p & 3u);
        uint32_t d0, d1, d2;
        if (a + 4u > T.lo && a + 8u < T.hi) {
            const u32x3 d = *(global_u32x3_a4 *)a;
            d0 = d.x;
            d1 = d.y;
            d2 = d.z;
        } else {
            d0 = gdword(T, a);
            d1 = gdword(T, a + 4u);
            d2 = gdword(T, a + 8u);
        }
        const uint32_t lo = __builtin_amdgcn_alignbyte(d1, d0, sh);
        const uint32_t hi = __builtin_amdgcn_alignbyte(d2, d1, sh);
#pragma unroll
        for (int k = Q - 1; k >= 0; --k) {
            const int b = 8 - Q + k;
            const uint32_t c = b < 4 ? __builtin_amdgcn_ubfe(lo, 8 * b, 8) : __builtin_amdgcn_ubfe(hi, 8 * (b - 4), 8);
            v = (v << s) + c;
        }
    }
    return v & mask;
}

typedef uint32_t u32x4_v __attribute__((ext_vector_type(4)));
typedef u32x4_v u32x4_a4 __attribute__((aligned(4)));
typedef const __attribute__((address_space(1))) u32x4_a4 global_u32x4_a4;

// The 16 text bytes ending at absolute address e, as four dwords (w[0]'s
// lowest byte is e - 15, w[3]'s highest is e), read with one 16-byte and one
// 4-byte load where every dword read holds a text byte, else dword by dword
// (dwords with no text byte read as 0).
__device__ __forceinline__ void gspan16(const GlobalText &T, uintptr_t e, uint32_t (&w)[4]) {
    const uintptr_t p = e - 15u, a = p & ~uintptr_t(3);
    uint32_t d[5];
    if (a + 4u > T.lo && a + 16u < T.hi) {
        const u32x4_v v = *(global_u32x4_a4 *)a;
        d[0] = v.x;
        d[1] = v.y;
        d[2] = v.z;
        d[3] = v.w;
        d[4] = *(global_u32 *)(a + 16u);
    } else {
#pragma unroll
        for (int i = 0; i < 5; ++i) d[i] = gdword(T, a + 4u * uint32_t(i));
    }
    const uint32_t sh = uint32_t(p & 3u);
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sh);
}

// Hash (eq. (3)) of the q-gram that ends I * Q bytes before the end of a
// 16-byte span (I * Q + Q <= 16).
template <int Q, int I>
__device__ __forceinline__ uint32_t span_hash(const uint32_t (&w)[4], uint32_t s, uint32_t mask) {
    static_assert(I * Q + Q <= 16, "q-gram inside the span");
    uint32_t v = 0;
#pragma unroll
    for (int k = Q - 1; k >= 0; --k) {
        constexpr int kEnd = 15 - I * Q;
        const int b = kEnd - (Q - 1) + k;   // span position of byte k of the q-gram
        v = (v << s) + __builtin_amdgcn_ubfe(w[b >> 2], 8 * (b & 3), 8);
    }
    return v & mask;
}

// Chain steps I..KS of an attempt whose q-grams lie in the span w (the
// q-gram of step i ends i * Q bytes before the span's end). Returns true with
// `next` set when a link is missing; false when the steps in the span are
// used up or the walk reached the window start (then e < lo).
template <int Q, int I, int KS, typename WT>
__device__ __forceinline__ bool span_chain(const uint32_t (&w)[4], const PatternView &P, const WT *__restrict__ F,
                                           int32_t lo, uint32_t &e, uint32_t &v, WT &z, uint32_t &next) {
    if constexpr (I > KS) {
        return false;
    } else {
        if (int32_t(e) < lo) return false;
        const uint32_t vp = span_hash<Q, I>(w, P.s, P.mask);
        const uint32_t ep = e - Q;
        if (!linked(z, vp)) {
            next = ep + P.m - Q + 1u;
            return true;
        }
        e = ep;
        v = vp;
        z = F[vp];
        return span_chain<Q, I + 1, KS, WT>(w, P, F, lo, e, v, z, next);
    }
}

// One attempt of the searching loop at window end J (tile-relative; base =
// absolute address of tile position 0) with the 16 bytes ending at J already
// in w: the first word, then the chain of links towards the window start,
// its first 16 / Q - 1 steps from w and the rest read in place. Returns the
// next window end; after kSparseLocalSteps links read in place the walk is
// handed back (kParkedJ) with its position in (e, v, z). Marks candidates.
template <int Q, typename WT>
__device__ __forceinline__ uint32_t sparse_attempt(const GlobalText &T, uintptr_t base, const WT *__restrict__ F,
                                                   const PatternView &P, uint32_t J, const uint32_t (&w)[4],
                                                   uint32_t &e, uint32_t &v, WT &z, uint32_t *bitmap,
                                                   uint32_t *any) {
    constexpr int KS = 16 / Q - 1;   // chain steps inside the span
    const uint32_t shift = P.m - Q + 1u;
    v = span_hash<Q, 0>(w, P.s, P.mask);
    z = F[v];
    if (z == 0) return J + shift;   // no q-gram of x hashes here
    const int32_t lo = int32_t(J) - int32_t(P.m) + 2 * Q;
    e = J;
    uint32_t next = 0;
    if (span_chain<Q, 1, KS, WT>(w, P, F, lo, e, v, z, next)) return next;
    int steps = kSparseLocalSteps;
    while (int32_t(e) >= lo) {
        if (steps-- == 0) return kParkedJ;
        const uint32_t ep = e - Q;
        const uint32_t vp = ghash<Q>(T, base + ep, P.s, P.mask);
        if (!linked(z, vp)) return ep + shift;
        e = ep;
        v = vp;
        z = F[vp];
    }
    if (v == P.hv) mark(bitmap, J + 1u - P.m, any);
    return J + 1u;
}

// A parked chain walk finished by the whole wavefront with the q-grams read
// in place; `base` is the absolute address of tile position 0.
template <int Q, typename WT>
__device__ __forceinline__ uint32_t gchain_wave(const GlobalText &T, uintptr_t base, const WT *__restrict__ F,
                                                const PatternView &P, const Parked &pk, uint32_t lane,
                                                uint32_t *bitmap, uint32_t *any) {
    return chain_wave_impl<Q, WT>([&](uint32_t e) { return ghash<Q>(T, base + e, P.s, P.mask); }, F, P, pk, lane,
                                  bitmap, any);
}

// Inclusive prefix sum across a wavefront with DPP row shifts and row
// broadcasts (no LDS round trips).
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    // row_shr:1,2,4,8 within rows of 16 lanes (bound_ctrl: shifted-in lanes read 0)
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);
    // row_bcast:15 adds the last lane of each row to the next row (rows 1, 3)
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
    // row_bcast:31 adds lane 31 to rows 2 and 3
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
    return v;
}

// Block-wide exclusive scan of one value per thread (blockDim = 256).
// Returns the thread's exclusive prefix; *total receives the block sum.
// lds_w holds four words; callers separate successive scans by a barrier.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t c, uint32_t *lds_w,
                                                         uint32_t *total) {
    const uint32_t lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const uint32_t incl = wave_inclusive_sum(c);
    if (lane == kWave - 1) lds_w[wid] = incl;
    lds_barrier();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
        const uint32_t v = lds_w[i];
        if (i < wid) before += v;
        all += v;
    }
    *total = all;
    return before + incl - c;
}

// ----------------------------------------------------------------------------
// One tile searched for one pattern: the searching loop of every lane over
// its block of window starts (rounds separated by LDS barriers while lanes
// have parked chain walks), then the comparison of the candidate windows with
// x. Leaves the occurrences in the bitmap `bm` (tile-relative starts) and
// returns the tile's count, this thread's exclusive prefix and its bitmap
// word range. Every thread of the workgroup calls it. `it` and `round` are
// per-workgroup counters that select double-buffered LDS flags; misc[8..11]
// hold those flags and misc[0..3] the scan.
// ----------------------------------------------------------------------------
struct TileResult {
    uint32_t total, mine, w0, w1;
};

// After the marking phase and a barrier: compares the tile's marked windows
// with x, keeps the occurrences in the bitmap and counts them (this thread's
// words [w0, w1), its exclusive offset and the tile total). Reads and resets
// the candidate flags, which alternate between two LDS words per call.
__device__ __forceinline__ TileResult verify_tile(const uint32_t *__restrict__ t32, uint32_t tb,
                                                  const uint32_t *__restrict__ x32, const PatternView &P,
                                                  uint32_t S, uint32_t *bm, uint32_t *misc, uint32_t &it,
                                                  bool exact = false) {
    const uint32_t tid = threadIdx.x;
    const bool has = misc[8 + (it & 1u)] != 0u;
    if (tid == 0) misc[8 + ((it + 1u) & 1u)] = 0u;   // flag of the next call
    ++it;
    TileResult R{0u, 0u, 0u, 0u};
    if (!has) return R;                           // most tiles: no candidate at all
    // compare candidates with x; count this thread's share of the tile
    const uint32_t words = (S + 31u) / 32u;
    const uint32_t wpt = (words + kThreads - 1u) / kThreads;
    R.w0 = min(words, tid * wpt);
    R.w1 = min(words, R.w0 + wpt);
    uint32_t c = 0;
    for (uint32_t i = R.w0; i < R.w1; ++i) {
        uint32_t b = bm[i], keep = b;
        while (b && !exact) {   // exact: the marks were compared with x already
            const uint32_t bit = __builtin_ctz(b);
            b &= b - 1u;
            if (!window_equals(t32, tb + i * 32u + bit, x32, P.m)) keep &= ~(1u << bit);
        }
        bm[i] = keep;
        c += __popc(keep);
    }
    R.mine = block_exclusive_scan(c, misc, &R.total);
    return R;
}

template <int Q, typename WT, int K, bool WIDE = true>
__device__ __forceinline__ TileResult search_tile(const uint32_t *__restrict__ t32, uint32_t tb,
                                                  const WT *__restrict__ F,
                                                  const uint32_t *__restrict__ x32,
                                                  const PatternView &P, uint32_t S, uint32_t seg,
                                                  uint32_t *bm, Parked *park, uint32_t *misc,
                                                  uint32_t &it, uint32_t &round) {
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    uint32_t *any = &misc[8 + (it & 1u)];
    {
        // WIDE: a lane's range holds at least two shifts (one per half): a
        // first attempt whose word is empty already rules out a shift's
        // worth of window ends, so narrower ranges would only repeat
        // attempts. With long patterns only the first ranges hold windows;
        // range r goes to lane r / 4 of wavefront r % 4, so those are spread
        // over the workgroup's four wavefronts (and SIMDs).
        const uint32_t span = WIDE ? max(seg, 2u * (P.m - Q + 1u)) : seg;
        const uint32_t r = (lane << 2) | wid;
        const uint32_t lo = min(S, r * span), hi = min(S, lo + span);
        const uint32_t jlo = lo + P.m - 1u, jhi = hi + P.m - 1u;
        const uint32_t jmid = jlo + ((jhi - jlo) >> 1);
        uint32_t J0 = jlo, J1 = jmid, myslot = kParkCap;
        bool running = lo < hi;
        while (true) {
            uint32_t *npark = &misc[10 + (round & 1u)];
            if (running)   // afterwards: true when the lane parked a walk
                running = !hc_segment<Q, WT, K>(t32, tb, F, P, J0, jmid, J1, jhi, bm, any, park,
                                                npark, &myslot);
            lds_barrier();
            const uint32_t np = min(*npark, kParkCap);
            if (tid == 0) misc[10 + ((round + 1u) & 1u)] = 0u;
            ++round;
            if (np == 0u) break;
            // long chain walks, finished by whole wavefronts
            for (uint32_t i = wid; i < np; i += kThreads / kWave) {
                const Parked pk = park[i];
                const uint32_t next = hc_chain_wave<Q, WT>(t32, tb, F, P, pk, lane, bm, any);
                if (lane == 0) park[i].J = next;
            }
            lds_barrier();
            if (running) {
                const Parked &pk = park[myslot];
                if ((pk.owner & 1u) == 0u) J0 = pk.J; else J1 = pk.J;
                myslot = kParkCap;
            }
            // slots are numbered from 0 again in the next round: every wave
            // must have read its walk's result before any wave parks again
            lds_barrier();
        }
    }
    return verify_tile(t32, tb, x32, P, S, bm, misc, it);
}

// SHC (Section 3.4, third optimisation) on a tile: a copy of x sits right
// after the tile's staged bytes (the sentinel), so the loop over empty words
// needs no position test: it always stops at a non-empty word, at the latest
// inside the copy of x, whose q-grams all have non-empty words and which is
// longer than one shift. A lane's loop may thus run past its own range; the
// window it stops at is then simply not searched by this lane.
template <int Q, typename WT>
__device__ __forceinline__ void shc_lane(const uint32_t *__restrict__ t32, uint32_t tb, const WT *__restrict__ F,
                                         const PatternView &P, uint32_t J, uint32_t Jend, uint32_t *bitmap,
                                         uint32_t *any) {
    const uint32_t shift = P.m - Q + 1u;
    while (J < Jend) {
        uint32_t v = qgram_hash<Q>(t32, tb + J, P);
        WT z = F[v];
        while (z == 0) {   // no bounds test: the sentinel ends this loop
            J += shift;
            v = qgram_hash<Q>(t32, tb + J, P);
            z = F[v];
        }
        if (J >= Jend) break;
        uint32_t e = J;
        bool hit = false;
        const uint32_t next = hc_chain<Q, WT>(t32, tb, F, P, J, e, v, z, 1 << 30, &hit);
        if (hit) mark(bitmap, J + 1u - P.m, any);
        J = next;
    }
}

template <int Q, typename WT>
__device__ __forceinline__ TileResult shc_tile(const uint32_t *__restrict__ t32, uint32_t tb,
                                               const WT *__restrict__ F, const uint32_t *__restrict__ x32,
                                               const PatternView &P, uint32_t S, uint32_t seg, uint32_t *bm,
                                               uint32_t *misc, uint32_t &it) {
    const uint32_t lo = min(S, threadIdx.x * seg), hi = min(S, lo + seg);
    shc_lane<Q, WT>(t32, tb, F, P, lo + P.m - 1u, hi + P.m - 1u, bm, &misc[8 + (it & 1u)]);
    lds_barrier();
    return verify_tile(t32, tb, x32, P, S, bm, misc, it);
}

// Dense schedule: the test of the searching loop (first word nonzero, each
// q-gram of the chain linked to the next, last hash equal to H_v), applied to
// every window of the tile rather than only to the windows the shifts land
// on. A shift only skips windows that fail this test, and verification
// removes every non-occurrence, so the result is the same. Each lane takes 8
// consecutive window starts at a time: it loads the text around them once,
// hashes the 8 window-end q-grams and the C * q q-gram ends behind them
// (C = m / q - 1 links per window), looks up their words, and writes the 8
// outcomes as one bitmap byte. Everything is branch-free, so no lane waits
// for another's shift: this pays when shifts (m - q + 1) are short.
// With no links (m < 2q) the test is H(window-end q-gram) = H_v alone: the
// word F[H_v] is never empty (H_v hashes one of the first q q-grams of x,
// which is linked or marked). The windows that pass are compared with x by
// the lane that tested them, one candidate at a time after its last step (a
// wavefront tests 1024 windows per step, so a comparison inside each step
// with a candidate would run for the whole wavefront on almost every step);
// when q = m and s >= 8 the hash is one-to-one on windows and the test
// itself is exact.
// Marks the tile's windows that pass the test; returns whether any did.
// The bitmap is all zero on entry (every tile leaves it cleared), so only
// nonzero bytes are written.
//
// No links (m < 2q): 16 windows per lane and step. The 16 window-end hashes
// are formed two at a time in 16-bit lanes: column k holds byte k of every
// window's q-gram, zero-extended in pairs, and is added times 2^(s k); sums
// wrap mod 2^16, which 2^alpha divides (alpha <= 16). S8: q = 2 and s = 8
// (alpha = 16), where the hash is the window's own 16-bit value, gathered
// by one permute per pair. t = (H xor H_v) mod 2^alpha per half; the 16
// halves are folded by packed 16-bit minimums, so one test per step tells
// whether any window passed, and only such steps take the bits one by one.
// SAD4: m = 4 (q = 3 or 4). Without links the test reads the window-end
// q-gram and verification then reads the whole window, so together they
// decide exactly whether the window equals x; with a window of one dword the
// kernel compares it with x directly: t = the sum of absolute byte
// differences, zero exactly for an occurrence. One quad-SAD instruction
// gives it for four consecutive windows (the four byte offsets of an 8-byte
// source) as four 16-bit halves. SAD8: 5 <= m <= 8, the same with two quad
// SADs per four windows, over the window's first and last 4 bytes (which
// overlap when m < 8), the second accumulating onto the first.
// The marks left are occurrences (every candidate has been compared with x).
constexpr int kNolinkHash = 0, kNolinkS8 = 1, kNolinkSad4 = 2, kNolinkSad8 = 3;

template <int Q, int MODE>
__device__ __forceinline__ bool dense_mark_nolink(const uint32_t *__restrict__ t32, uint32_t tb,
                                                  const uint32_t *__restrict__ x32, const PatternView &P,
                                                  uint32_t S, uint32_t *bm) {
    static_assert(Q >= 1 && Q <= 8, "q-grams of at most 8 bytes");
    typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
    // the words loaded start PRE bytes before the first window end
    constexpr int PRE = (Q <= 4 && MODE != kNolinkSad8) ? 3 : 7;
    constexpr int NWW = (PRE + 15) / 4 + 1;   // aligned words covering the 16 q-grams
    uint16_t *bm16 = reinterpret_cast<uint16_t *>(bm);
    const uint32_t steps = (S + 15u) / 16u;
    const uint32_t mask2 = P.mask | (P.mask << 16), hv2 = P.hv | (P.hv << 16);
    // q = m and s >= 8: the hash is one-to-one on windows (each byte in its
    // own 8 bits), so a window passes the test exactly when it equals x
    const bool exact = MODE == kNolinkSad4 || MODE == kNolinkSad8 || (P.m == uint32_t(Q) && P.s >= 8u);
    // SAD4 / SAD8: the pattern's first 4 bytes, and its last 4 (SAD8)
    const uint32_t x4 = x32[0];
    const uint32_t x4last = uint32_t(((uint64_t(x32[1]) << 32) | x32[0]) >> (8u * ((P.m - 4u) & 7u)));
    uint32_t cmask = 0;   // this lane's steps with candidates
    uint32_t ks = 0;
    for (uint32_t g = threadIdx.x; g < steps; g += kThreads, ++ks) {
        const uint32_t st0 = 16u * g;
        // window st0 + j ends at LDS byte a0 + j; w[i] = bytes p0 + 4i .. p0 + 4i + 3
        const uint32_t a0 = tb + st0 + P.m - 1u;
        const uint32_t p0 = a0 - uint32_t(PRE), base = p0 >> 2, sh = p0 & 3u;
        uint32_t d[NWW + 1], w[NWW];
#pragma unroll
        for (int i = 0; i <= NWW; ++i) d[i] = t32[base + i];
#pragma unroll
        for (int i = 0; i < NWW; ++i) w[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sh);
        // pair i = windows 2i (low half) and 2i + 1 (high half); per half
        // t = 0 exactly when the window passes
        uint32_t t[8];
        if constexpr (MODE == kNolinkSad4) {
            static_assert(Q >= 3 && Q <= 4, "m = 4 without links");
            // window 4h + k starts at byte 4h + k of the words (p0 is the
            // first window's start)
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const uint64_t src = (uint64_t(w[h + 1]) << 32) | w[h];
                const uint64_t sad = __builtin_amdgcn_qsad_pk_u16_u8(src, x4, 0ull);
                t[2 * h] = uint32_t(sad);
                t[2 * h + 1] = uint32_t(sad >> 32);
            }
        } else if constexpr (MODE == kNolinkSad8) {
            // p0 = the first window's start - (8 - m): window 4h + k has its
            // last 4 bytes at byte 4 + 4h + k of the words and its first 4 at
            // byte (8 - m) + 4h + k, i.e. byte 4h + k of the words f
            const uint32_t o = 8u - P.m;   // 0..3
            uint32_t f[NWW - 1];
#pragma unroll
            for (int i = 0; i < NWW - 1; ++i) f[i] = __builtin_amdgcn_alignbyte(w[i + 1], w[i], o);
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const uint64_t first = (uint64_t(f[h + 1]) << 32) | f[h];
                const uint64_t last = (uint64_t(w[h + 2]) << 32) | w[h + 1];
                const uint64_t sad = __builtin_amdgcn_qsad_pk_u16_u8(
                    last, x4last, __builtin_amdgcn_qsad_pk_u16_u8(first, x4, 0ull));
                t[2 * h] = uint32_t(sad);
                t[2 * h + 1] = uint32_t(sad >> 32);
            }
        } else {
            // byte k of the pair's q-grams sits at p0 + c and p0 + c + 1,
            // c = PRE + 1 - Q + k + 2i
            u16x2 acc[8];
            if constexpr (MODE == kNolinkS8) {
                static_assert(Q == 2, "one-to-one 16-bit windows");
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    // bytes c, c + 1 (low half) and c + 1, c + 2 (high half)
                    const int c = PRE - 1 + 2 * i;
                    const int h = (c >> 2) < NWW - 2 ? (c >> 2) : NWW - 2;
                    const uint32_t o = uint32_t(c - 4 * h);
                    acc[i] = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(w[h + 1], w[h],
                                                                             o | ((o + 1u) << 8) | ((o + 1u) << 16) |
                                                                                 ((o + 2u) << 24)));
                }
            } else {
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    const uint32_t mk = 1u << (P.s * uint32_t(k));   // s k <= alpha - s < 16
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        // v_perm numbers the bytes of {src0, src1} from src1's
                        // lowest; selector 0x0C yields a zero byte
                        const int c = PRE + 1 - Q + k + 2 * i;
                        const int h = (c >> 2) < NWW - 2 ? (c >> 2) : NWW - 2;
                        const uint32_t o = uint32_t(c - 4 * h);
                        const uint32_t pr = __builtin_amdgcn_perm(w[h + 1], w[h], 0x0C000C00u | o | ((o + 1u) << 16));
                        const u16x2 r = __builtin_bit_cast(u16x2, pr);
                        acc[i] = k == 0 ? r : acc[i] + r * u16x2{uint16_t(mk), uint16_t(mk)};
                    }
                }
            }
            // t = (H ^ H_v) mod 2^alpha
#pragma unroll
            for (int i = 0; i < 8; ++i) t[i] = (__builtin_bit_cast(uint32_t, acc[i]) ^ hv2) & mask2;
        }
        u16x2 mn = __builtin_bit_cast(u16x2, t[0]);
#pragma unroll
        for (int i = 1; i < 8; ++i) mn = __builtin_elementwise_min(mn, __builtin_bit_cast(u16x2, t[i]));
        const uint32_t mv = __builtin_bit_cast(uint32_t, mn);
        // a zero half: some window passed (exact for 16-bit halves)
        const bool hit = ((mv - 0x00010001u) & ~mv & 0x80008000u) != 0u;
        uint32_t bits = 0;
        if (__builtin_amdgcn_ballot_w64(hit) != 0ull) {   // uniform: rare unless windows match often
            // nz: 1 in a half iff that half of t is non-zero (a packed
            // minimum with 1, written out so that it stays one instruction
            // and is not computed above the branch); the bytes 0 and 2 of
            // two pairs are gathered into one dword and weighted 1, 2, 4, 8
            uint32_t nz[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)   // both halves of the second operand: 0x0001 0x0001
                asm volatile("v_pk_min_u16 %0, %1, %2" : "=v"(nz[i]) : "v"(t[i]), "s"(0x00010001u));
            uint32_t nb = 0;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const uint32_t four = __builtin_amdgcn_perm(nz[2 * p + 1], nz[2 * p], 0x06040200u);
                nb |= __builtin_amdgcn_udot4(four, 0x08040201u, 0u, false) << (4 * p);
            }
            bits = nb ^ 0xFFFFu;                                  // window j passed: bit j
            if (st0 + 16u > S) bits &= (1u << (S - st0)) - 1u;   // windows past the tile
        }
        if (bits) {
            bm16[g] = uint16_t(bits);
            cmask |= 1u << ks;
        }
    }
    if (exact) return cmask != 0u;
    // the candidates, one at a time
    uint32_t any = 0;
    ks = 0;
    for (uint32_t g = threadIdx.x; g < steps; g += kThreads, ++ks) {
        if (!((cmask >> ks) & 1u)) continue;
        uint32_t b = bm16[g], keep = b;
        while (b) {
            const uint32_t bit = __builtin_ctz(b);
            b &= b - 1u;
            if (!window_equals(t32, tb + 16u * g + bit, x32, P.m)) keep &= ~(1u << bit);
        }
        bm16[g] = uint16_t(keep);
        any |= keep;
    }
    return any != 0u;
}

// With links (C = m / q - 1 >= 1): 8 windows per lane and step; the 8
// window-end q-grams and the C * q q-gram ends behind them are hashed one by
// one (dot products with the pattern's byte weights, as in qgram_hash) and
// their words looked up.
template <int Q, typename WT, int C>
__device__ __forceinline__ bool dense_mark(const uint32_t *__restrict__ t32, uint32_t tb, const WT *__restrict__ F,
                                           const uint32_t *__restrict__ x32, const PatternView &P, uint32_t S,
                                           uint32_t *bm) {
    static_assert(Q >= 1 && Q <= 4 && C >= 1, "dense schedule hashes 4-byte words");
    constexpr int E = 8 + C * Q;                  // q-gram ends per group of 8 windows
    constexpr int NW = ((E - 1) >> 2) + 2;        // aligned words covering them
    uint8_t *bm8 = reinterpret_cast<uint8_t *>(bm);
    const uint32_t groups = (S + 7u) / 8u;
    uint32_t any = 0;
    for (uint32_t g = threadIdx.x; g < groups; g += kThreads) {
        const uint32_t st0 = 8u * g;
        // LDS position of the earliest q-gram end needed, and the first byte
        // of the 4-byte word that ends there
        const uint32_t a0 = tb + st0 + P.m - 1u - uint32_t(C * Q);
        const uint32_t p0 = a0 - 3u, base = p0 >> 2, sh = p0 & 3u;
        uint32_t d[NW + 1];
#pragma unroll
        for (int i = 0; i <= NW; ++i) d[i] = t32[base + i];
        uint32_t w[NW];
#pragma unroll
        for (int i = 0; i < NW; ++i) w[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sh);
        uint32_t h[E];
#pragma unroll
        for (int j = 0; j < E; ++j) {
            // bytes a0 + j - 3 .. a0 + j
            const uint32_t word = (j & 3) ? __builtin_amdgcn_alignbyte(w[(j >> 2) + 1], w[j >> 2], j & 3)
                                          : w[j >> 2];
            const uint32_t hi = __builtin_amdgcn_udot4(word, P.wh0, 0u, false);
            h[j] = __builtin_amdgcn_udot4(word, P.wl0, hi << 8, false) & P.mask;
        }
        WT z[E - Q];
#pragma unroll
        for (int j = Q; j < E; ++j) z[j - Q] = F[h[j]];
        uint32_t bits = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = j + C * Q;          // index of the window-end q-gram
            bool alive = z[e - Q] != 0;
#pragma unroll
            for (int k = 1; k <= C; ++k) alive = alive && linked(z[e - (k - 1) * Q - Q], h[e - k * Q]);
            alive = alive && h[e - C * Q] == P.hv;
            bits |= uint32_t(alive) << j;
        }
        if (st0 + 8u > S) bits &= (1u << (S - st0)) - 1u;   // windows past the tile
        if (bits) bm8[g] = uint8_t(bits);
        any |= bits;
    }
    return any != 0u;
}

template <int Q, typename WT, int C>
__device__ __forceinline__ TileResult dense_tile(const uint32_t *__restrict__ t32, uint32_t tb,
                                                 const WT *__restrict__ F, const uint32_t *__restrict__ x32,
                                                 const PatternView &P, uint32_t S, uint32_t *bm, uint32_t *misc,
                                                 uint32_t &it) {
    bool found;
    if constexpr (C == 0)
    {
        // windows of 4 to 8 bytes are compared with x directly (SAD4, SAD8)
        if constexpr (Q == 2)
            found = P.s == 8u ? dense_mark_nolink<2, kNolinkS8>(t32, tb, x32, P, S, bm)
                              : dense_mark_nolink<2, kNolinkHash>(t32, tb, x32, P, S, bm);
        else if constexpr (Q == 3 || Q == 4)
            found = P.m == 4u  ? dense_mark_nolink<Q, kNolinkSad4>(t32, tb, x32, P, S, bm)
                    : P.m >= 5u ? dense_mark_nolink<Q, kNolinkSad8>(t32, tb, x32, P, S, bm)   // m < 2q <= 8
                                : dense_mark_nolink<Q, kNolinkHash>(t32, tb, x32, P, S, bm);
        else if constexpr (Q >= 5)   // m >= q >= 5
            found = P.m <= 8u ? dense_mark_nolink<Q, kNolinkSad8>(t32, tb, x32, P, S, bm)
                              : dense_mark_nolink<Q, kNolinkHash>(t32, tb, x32, P, S, bm);
        else
            found = dense_mark_nolink<Q, kNolinkHash>(t32, tb, x32, P, S, bm);
    }
    else
        found = dense_mark<Q, WT, C>(t32, tb, F, x32, P, S, bm);
    if (found) misc[8 + (it & 1u)] = 1u;
    lds_barrier();
    // without links the marks are occurrences already: the pass only counts
    return verify_tile(t32, tb, x32, P, S, bm, misc, it, C == 0);
}

}  // namespace hc
