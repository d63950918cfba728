// Single-pattern searching phase of HC (Section 3.3) on gfx950.
//
// One persistent workgroup per slot on the chip takes text tiles in ticket
// order. Per tile it stages the window starts' bytes (tile plus an (m-1)-byte
// halo) from HBM into LDS with 16-byte loads, runs the searching loop in every
// lane against F and x held in LDS for the whole launch, marks occurrences in
// an LDS bitmap, and writes them as ascending int64 positions at an offset
// found by decoupled look-back over the preceding tiles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "hc_device.h"
#include "hc_internal.h"
#include "hc_runtime.h"

namespace hc {

struct SearchArgs {
    const uint8_t *y;
    uint64_t n;
    const uint8_t *x;
    const void *F;
    uint32_t m, q, s, mask, hv;
    uint32_t table_bytes;
    uint32_t tile;       // window starts per tile (256 * segment)
    uint32_t seg;        // window starts per lane
    uint64_t starts;     // n - m + 1
    uint32_t n_tiles;
    uint32_t status_cap;
    int64_t *out;
    int64_t cap;
    int64_t *d_count;
    uint64_t *status;
    Ctl *ctl;
};

template <int Q, typename WT, int SCHED>
__global__ __launch_bounds__(kBlock) void hc_search_kernel(SearchArgs A) {
    extern __shared__ __align__(16) uint8_t lds[];
    const LdsLayout L = lds_layout(A.tile, A.m, A.table_bytes, 0);
    uint8_t *t8 = lds + L.text_off;
    const uint32_t *t32 = reinterpret_cast<const uint32_t *>(t8);
    uint32_t *bitmap = reinterpret_cast<uint32_t *>(lds + L.bitmap_off);
    WT *F = reinterpret_cast<WT *>(lds + L.table_off);
    uint8_t *x8 = lds + L.x_off;
    uint32_t *misc = reinterpret_cast<uint32_t *>(lds + L.misc_off);
    // misc[0..3] wavefront sums, [4] next ticket, [5] generation, [6] tile offset, [7] flag

    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;

    // F and x stay in LDS for the whole launch
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(A.F);
        uint4 *dst = reinterpret_cast<uint4 *>(F);
        for (uint32_t i = tid; i < (A.table_bytes + 15u) / 16u; i += kBlock) dst[i] = src[i];
        for (uint32_t i = tid; i < A.m; i += kBlock) x8[i] = A.x[i];
    }
    if (tid == 0) {
        misc[5] = __hip_atomic_load(&A.ctl->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        misc[4] = __hip_atomic_fetch_add(&A.ctl->ticket, 1u, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
        if (blockIdx.x == 0 && A.n_tiles == 0) *A.d_count = 0;
    }
    __syncthreads();
    const uint32_t gen = misc[5];
    uint32_t t = misc[4];
    const PatternView P{A.m, uint32_t(Q), A.s, A.mask, A.hv};

    while (t < A.n_tiles) {
        const uint64_t tile_lo = uint64_t(t) * A.tile;
        const uint32_t S = uint32_t(min<uint64_t>(A.tile, A.starts - tile_lo));
        const uint32_t tb = stage_text(A.y, tile_lo, tile_lo + S + A.m - 1u, t8);
        for (uint32_t i = tid; i < A.tile / 32u; i += kBlock) bitmap[i] = 0u;
        if (tid == 0)
            misc[4] = __hip_atomic_fetch_add(&A.ctl->ticket, 1u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();

        if constexpr (SCHED == HC_SCHED_WAVE) {
            const uint32_t per = (S + 3u) / 4u;
            const uint32_t lo = min(S, wid * per), hi = min(S, lo + per);
            hc_wave<Q, WT>(t32, t8, tb, F, x8, P, lo, hi, bitmap, lane);
        } else {
            const uint32_t lo = min(S, tid * A.seg), hi = min(S, lo + A.seg);
            if (lo < hi) hc_segment<Q, WT>(t32, t8, tb, F, x8, P, lo + A.m - 1u, hi + A.m - 1u, bitmap);
        }
        __syncthreads();

        // ordered compaction of the tile's bitmap
        const uint32_t words = (S + 31u) / 32u;
        const uint32_t wpt = (words + kBlock - 1u) / kBlock;
        const uint32_t w0 = min(words, tid * wpt), w1 = min(words, w0 + wpt);
        uint32_t c = 0;
        for (uint32_t i = w0; i < w1; ++i) c += __popc(bitmap[i]);
        uint32_t total;
        const uint32_t mine = block_exclusive_scan(c, misc, &total);
        if (wid == 0) {
            const uint32_t excl = lookback(A.status, t, gen, total, lane, &A.ctl->err);
            if (lane == 0) {
                misc[6] = excl;
                if (t == A.n_tiles - 1u) *A.d_count = int64_t(excl) + total;
            }
        }
        __syncthreads();
        int64_t idx = int64_t(misc[6]) + mine;
        for (uint32_t i = w0; i < w1 && idx < A.cap; ++i) {
            uint32_t b = bitmap[i];
            while (b && idx < A.cap) {
                const uint32_t bit = __builtin_ctz(b);
                b &= b - 1u;
                A.out[idx++] = int64_t(tile_lo + i * 32u + bit);
            }
        }
        t = misc[4];
        __syncthreads();
    }
    finish_launch(A.ctl, A.status, A.status_cap, gen, &misc[7], A.d_count);
}

// ----------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------

using KernelFn = void (*)(SearchArgs);

template <int Q, typename WT>
static KernelFn pick_sched(int sched) {
    return sched == HC_SCHED_WAVE ? hc_search_kernel<Q, WT, HC_SCHED_WAVE>
                                  : hc_search_kernel<Q, WT, HC_SCHED_SEGMENT>;
}

template <int Q>
static KernelFn pick_w(int w, int sched) {
    switch (w) {
        case 8: return pick_sched<Q, uint8_t>(sched);
        case 16: return pick_sched<Q, uint16_t>(sched);
        case 32: return pick_sched<Q, uint32_t>(sched);
        default: return pick_sched<Q, uint64_t>(sched);
    }
}

static KernelFn pick_kernel(int q, int w, int sched) {
    switch (q) {
        case 1: return pick_w<1>(w, sched);
        case 2: return pick_w<2>(w, sched);
        case 3: return pick_w<3>(w, sched);
        case 4: return pick_w<4>(w, sched);
        case 5: return pick_w<5>(w, sched);
        case 6: return pick_w<6>(w, sched);
        case 7: return pick_w<7>(w, sched);
        default: return pick_w<8>(w, sched);
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

hc_status launch_single(const hc_pattern *p, const DeviceCopy &dc, const uint8_t *d_y, int64_t n,
                        int64_t *d_out, int64_t cap, int64_t *d_count, const hc_launch &lc,
                        hipStream_t stream) {
    const PatternData &pd = p->data;
    const DeviceInfo &di = device_info();
    const uint32_t m = uint32_t(pd.m);
    const uint32_t table_bytes = uint32_t(pd.F.size() * (pd.w / 8));
    const uint64_t starts = n >= pd.m ? uint64_t(n - pd.m + 1) : 0;

    uint32_t seg = uint32_t(lc.segment);
    LdsLayout L = lds_layout(kBlock * seg, m, table_bytes, 0);
    while (L.total > di.max_lds_per_block && seg > 8) {
        seg = std::max<uint32_t>(8, seg / 2);
        L = lds_layout(kBlock * seg, m, table_bytes, 0);
    }
    if (L.total > di.max_lds_per_block) return HC_EINVAL;
    const uint32_t tile = kBlock * seg;
    const uint64_t n_tiles64 = (starts + tile - 1) / tile;
    if (n_tiles64 > 0xFFFFFFFFull) return HC_EINVAL;
    const uint32_t n_tiles = uint32_t(n_tiles64);

    Workspace *ws = nullptr;
    hc_status st = workspace_for(stream, std::max<uint32_t>(n_tiles, 1), &ws);
    if (st != HC_OK) return st;

    KernelFn fn = pick_kernel(pd.q, pd.w, lc.schedule);
    int per_cu = occupancy(fn, L.total);
    if (lc.wg_per_cu > 0) per_cu = std::min(per_cu, int(lc.wg_per_cu));
    uint32_t grid = uint32_t(std::max<int64_t>(1, std::min<int64_t>(n_tiles, int64_t(di.cus) * per_cu)));

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
    A.status_cap = ws->status_cap;
    A.out = d_out;
    A.cap = cap;
    A.d_count = d_count;
    A.status = ws->status;
    A.ctl = reinterpret_cast<Ctl *>(ws->ctl);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kBlock), L.total, stream, A);
    return hipGetLastError() == hipSuccess ? HC_OK : HC_EHIP;
}

}  // namespace hc
