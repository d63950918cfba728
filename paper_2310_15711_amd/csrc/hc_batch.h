// Host interface of the batched searching kernel, shared by the batch plans
// of the C ABI and the serving loop. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>
#include <vector>

#include "hc_internal.h"

namespace hc {

struct BPat {            // one pattern of the batch, as the kernel reads it
    uint32_t m, q, s, mask, hv;
    uint32_t x_off;      // byte offset of x in the packed patterns (16-aligned)
    uint32_t pad0, pad1;
    uint32_t w[4];       // byte weights of the hash (byte_weights: wl0, wl1, wh0, wh1)
};

struct BItem {           // one work item
    uint32_t text, tile, g0, g1;   // group = glist[g0, g1), sorted by m descending
};

struct TextView {        // one text as a batch sees it
    const uint8_t *ptr;
    uint64_t len;          // bytes readable from ptr
    uint64_t start_limit;  // only window starts below this are searched
};

// Owned device allocation that only grows.
struct DeviceBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DeviceBuf() = default;
    DeviceBuf(const DeviceBuf &) = delete;
    DeviceBuf &operator=(const DeviceBuf &) = delete;
    ~DeviceBuf();
    hc_status ensure(size_t b);
    hc_status upload(const void *src, size_t b, hipStream_t s);   // async on s
    template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

// What the host decides for one batch: texts, patterns, pairs and work items.
struct BatchHost {
    std::vector<TextView> views;
    std::vector<BPat> pats;
    std::vector<uint32_t> glist;      // (pattern, pair) per group member
    std::vector<uint64_t> pair_base;  // n_pairs + 1
    std::vector<BItem> items;
};

// Device side of a batch: geometry, uploaded descriptors and result buffers.
struct BatchDev {
    uint32_t tile = 0, seg = 100, table_bytes = 0, max_m = 1, w = 16, lds = 0, max_grid = 0, group = 128;
    uint32_t n_pairs = 0, n_items = 0, grid = 0, nb = 0;
    uint64_t n_entries = 0, scratch_cap = 0;
    const uint8_t *Fs = nullptr;   // table_bytes per pattern index
    const uint8_t *xs = nullptr;   // pattern bytes at BPat::x_off
    size_t Fs_bytes = 0, xs_bytes = 0;
    hipError_t last_error = hipSuccess;   // of the last batch_enqueue
    const BPat *pats_dev = nullptr;       // resident descriptors (then `pats` is not uploaded)
    DeviceBuf views, pats, items, glist, pair_base, counts, toff, temp, ctl, tot, bsum, grand;
};

// Launch shape of the batched kernel: table shape for fields the caller
// leaves at 0, window starts per lane (tile = 256 * seg, reduced to fit
// LDS and the staging registers), patterns per staged tile, and a cap on
// resident workgroups per compute unit (0 = as many as fit).
struct BatchKnobs {
    int alpha = 12, w = 16;
    uint32_t seg = 100, group = 128, wg_per_cu = 0;
};

// The library's current choice (hc_batch_autotune's winner, else the
// defaults above); process-wide.
BatchKnobs batch_knobs();
void set_batch_knobs(const BatchKnobs *k);   // null = back to the defaults

// Common table shape of a batch (w in {16, 32}; tables up to 16 KiB); fields
// of params left at 0 come from the knobs.
hc_status batch_shape(const hc_params *params, int &alpha, int &w, uint32_t &table_bytes,
                      const BatchKnobs &k = batch_knobs());

// hc_batch_plan_create with explicit knobs.
hc_status plan_create(const hc_batch *b, const hc_params *params, const BatchKnobs &knobs,
                      hc_batch_plan **out);

// Tile size, LDS and grid bound for patterns up to max_m bytes.
hc_status batch_geometry(BatchDev &D, uint32_t max_m, uint32_t table_bytes, uint32_t w,
                         const BatchKnobs &k = batch_knobs());

// Preprocesses np patterns (CSR pat/pat_off) into packed tables and bytes.
hc_status pack_patterns(const uint8_t *pat, const int64_t *pat_off, int32_t np, const hc_params *params,
                        int alpha, int w, uint32_t table_bytes, std::vector<BPat> &bp,
                        std::vector<uint8_t> &Fh, std::vector<uint8_t> &Xh, uint32_t &max_m, bool host_tables);

// A pattern's descriptor (m, q, s, mask, H_v) without its table.
hc_status pack_desc(const uint8_t *x, int64_t m, int q_req, int alpha, int w, BPat &bp);

// Builds the word vectors of n patterns on the device (one workgroup each):
// pattern i's bytes at d_x + desc[3i], length desc[3i+1], q desc[3i+2]; its
// table at d_F + i * table_bytes; s, mask, H_v into d_info (may be null).
hc_status device_preprocess(const uint8_t *d_x, const uint32_t *d_desc, uint32_t n, int alpha, int w,
                            uint32_t table_bytes, uint8_t *d_F, uint32_t *d_info, hipStream_t s);

// One pattern's descriptor, table and bytes (for pools that place x themselves).
hc_status pack_one(const uint8_t *x, int64_t m, int q_req, int alpha, int w, uint32_t table_bytes,
                   BPat &bp, uint8_t *F_out);

// Groups the (pattern, text) pairs into work items (views and pats already set).
void batch_build(BatchHost &H, const std::vector<std::pair<uint32_t, uint32_t>> &pairs, uint32_t tile,
                 uint32_t group);

// Checks that every index the kernel derives from H stays inside the views,
// pattern tables, pattern bytes and per-pair entries (HC_EINVAL otherwise).
hc_status batch_check(const BatchHost &H, const BatchDev &D);

// Checks H (batch_check), uploads descriptors on stream s and sizes the
// result buffers.
hc_status batch_upload(const BatchHost &H, BatchDev &D, hipStream_t s);

// Enqueues the search, the CSR offsets (d_pair_off, n_pairs + 1 entries) and
// the copy of at most cap positions into d_pos, all on stream s.
hc_status batch_enqueue(BatchDev &D, int64_t *d_pos, int64_t cap, int64_t *d_pair_off, hipStream_t s);

// After a run reported scratch overflow: room for `total` positions.
hc_status batch_grow_scratch(BatchDev &D, uint64_t reserved, uint64_t total);

// Copies n staged (table, padded bytes, descriptor) entries into pool slots
// d_slots[i] of the tables, the pattern bytes and the descriptors.
hc_status scatter_patterns(const uint8_t *d_src, const uint32_t *d_slots, uint32_t n, uint32_t table_bytes,
                           uint32_t x_stride, uint8_t *Fpool, uint8_t *xpool, BPat *pats, hipStream_t s);

// Only the copy of the positions into d_pos (after a run whose scratch held
// every position but whose output capacity was too small).
hc_status batch_emit(BatchDev &D, int64_t *d_pos, int64_t cap, const int64_t *d_pair_off, hipStream_t s);


}  // namespace hc
