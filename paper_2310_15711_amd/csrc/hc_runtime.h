// Host runtime of libhc: device checks, per-stream launch workspaces, lazy
// upload of pattern tables, and the launchers behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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

// Launch workspace of one (device, stream): the grid-barrier control block and
// per-tile results of the search phase (counts, short position slots, spilled
// bitmaps). Calls on one stream serialise, so one workspace per stream is never
// used by two launches at once.
// Occurrences a tile keeps as a list of tile-relative starts; denser tiles
// keep their bitmap.
constexpr uint32_t kSlot = 128;

struct Workspace {
    void *ctl = nullptr;          // control words (work tickets), zero-initialised
    uint32_t *counts = nullptr;   // tiles_cap entries
    uint32_t *slots = nullptr;    // tiles_cap * kSlot entries
    uint32_t *spill = nullptr;    // spill_words_cap entries
    uint32_t tiles_cap = 0;
    uint64_t spill_words_cap = 0;
};

hc_status workspace_for(hipStream_t stream, uint32_t tiles, uint32_t tile, Workspace **out);

// Device copies of a pattern's F (packed w-bit words) and x on the current device.
hc_status pattern_on_device(hc_pattern *p, const DeviceCopy **out);

hc_status launch_single(const hc_pattern *p, const DeviceCopy &dc, const uint8_t *d_y, int64_t n,
                        int64_t *d_out, int64_t cap, int64_t *d_count, const hc_launch &lc,
                        hipStream_t stream);

// Launch shape chosen for a pattern when the caller leaves fields at 0.
hc_launch choose_launch(const PatternData &p, int64_t n, const hc_launch *req);

#define HC_CHECK_HIP(expr)                       \
    do {                                         \
        if ((expr) != hipSuccess) return HC_EHIP; \
    } while (0)

}  // namespace hc
