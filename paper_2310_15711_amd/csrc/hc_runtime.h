// Host runtime of libhc: device checks, per-stream launch workspaces, lazy
// upload of pattern tables, and the launchers behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "hc_internal.h"

namespace hc {

struct DeviceInfo {
    int device = -1;
    int cus = 0;
    uint32_t max_lds_per_block = 0;
    uint32_t lds_per_cu = 0;
    bool ok = false;   // gfx950
};

// Info for the current device (cached per device id).
const DeviceInfo &device_info();

// Launch workspace of one (device, stream): per-tile results of the search
// phase (counts, short position slots, spilled bitmaps), written by the
// search kernel and read by the emit kernel that follows it on the stream.
// Work on one stream runs in order, so the pair of one call finishes before
// the next call's search kernel starts; host threads that enqueue on the same
// stream hold the workspace's lock from the lookup until both kernels of their
// call are enqueued, so the pairs of two calls never interleave and a
// regrowth never frees buffers that a call has already taken.
// Occurrences a tile keeps as a list of tile-relative starts; denser tiles
// keep their bitmap.
constexpr uint32_t kSlot = 128;

// Range totals of the ordered output per call (its emit grid is at most this
// many workgroups when they are used).
constexpr uint32_t kRsumCap = 2048;

struct Workspace {
    std::mutex mu;                // held by the call that enqueues on this stream
    uint32_t *counts = nullptr;   // tiles_cap entries
    uint32_t *slots = nullptr;    // tiles_cap * kSlot entries
    uint32_t *spill = nullptr;    // spill_words_cap entries
    uint32_t tiles_cap = 0;
    uint64_t spill_words_cap = 0;
    // two arrays of kRsumCap range totals of the ordered output, used by
    // turns: the current call adds into array `parity` and its emit kernel
    // clears the other one for the next call (allocated cleared)
    uint32_t *rsum = nullptr;
    int parity = 0;
};

// Workspace of (current device, stream) with room for `tiles` tiles of `tile`
// window starts; returns with *lock holding the workspace's mutex.
hc_status workspace_for(hipStream_t stream, uint32_t tiles, uint32_t tile, Workspace **out,
                        std::unique_lock<std::mutex> *lock);

// Per-tile results of one search call (counts, range totals of the ordered
// output and the ones the emit kernel clears for the next call, or null,
// slot lists, spilled bitmaps).
struct TileScratch {
    uint32_t *counts = nullptr;
    uint32_t *rsum = nullptr;
    uint32_t *rsum_next = nullptr;
    uint32_t *slots = nullptr;
    uint32_t *spill = nullptr;
    int *parity = nullptr;   // the workspace's turn, flipped once the call is enqueued
};

// Device copies of a pattern's F (packed w-bit words) and x on the current
// device, uploaded on first use.
hc_status pattern_on_device(hc_pattern *p, const DeviceCopy **out);
// The same without uploading: null when the pattern has no copy on the
// current device yet.
const DeviceCopy *pattern_resident(hc_pattern *p);

// Enqueues one search call (search kernel + emit kernel) on `stream`. The
// per-tile results go to the stream's workspace, or, when `fixed` is set, to
// that device region of `fixed_bytes` bytes (HC_EINVAL when the call needs
// more; nothing is allocated then).
hc_status launch_single(const hc_pattern *p, const DeviceCopy &dc, const uint8_t *d_y, int64_t n,
                        int64_t *d_out, int64_t cap, int64_t *d_count, const hc_launch &lc,
                        hipStream_t stream, void *fixed = nullptr, uint64_t fixed_bytes = 0);

// Launch shape chosen for a pattern when the caller leaves fields at 0.
hc_launch choose_launch(const PatternData &p, int64_t n, const hc_launch *req);

#define HC_CHECK_HIP(expr)                       \
    do {                                         \
        if ((expr) != hipSuccess) return HC_EHIP; \
    } while (0)

}  // namespace hc
