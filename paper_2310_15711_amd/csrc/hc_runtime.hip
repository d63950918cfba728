// Host runtime and single-pattern entry points of the libhc C ABI.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>

#include "hc_device.h"
#include "hc_internal.h"
#include "hc_runtime.h"

namespace hc {

const DeviceInfo &device_info() {
    static std::mutex mu;
    static std::map<int, DeviceInfo> cache;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    DeviceInfo di;
    di.device = dev;
    hipDeviceProp_t prop;
    if (dev >= 0 && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        di.cus = prop.multiProcessorCount;
        di.max_lds_per_block = uint32_t(prop.sharedMemPerBlock);
        di.lds_per_cu = uint32_t(prop.maxSharedMemoryPerMultiProcessor);
        di.ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 && di.cus > 0;
    }
    return cache.emplace(dev, di).first->second;
}

hc_status workspace_for(hipStream_t stream, uint32_t tiles, uint32_t tile, Workspace **out,
                        std::unique_lock<std::mutex> *lock) {
    static std::mutex mu;
    static std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> spaces;
    const DeviceInfo &di = device_info();
    if (!di.ok) return HC_EHIP;
    Workspace *ws = nullptr;
    {
        std::lock_guard<std::mutex> g(mu);
        auto &slot = spaces[std::make_pair(di.device, stream)];
        if (!slot) {
            slot.reset(new (std::nothrow) Workspace());
            if (!slot) return HC_ENOMEM;
        }
        ws = slot.get();   // entries are never removed: the address stays valid
    }
    std::unique_lock<std::mutex> held(ws->mu);
    if (!ws->rsum) {
        if (hipMalloc(reinterpret_cast<void **>(&ws->rsum), sizeof(uint32_t) * 2u * kRsumCap) != hipSuccess) {
            ws->rsum = nullptr;
            return HC_ENOMEM;
        }
        if (hipMemset(ws->rsum, 0, sizeof(uint32_t) * 2u * kRsumCap) != hipSuccess) {
            (void)hipFree(ws->rsum);
            ws->rsum = nullptr;
            return HC_EHIP;
        }
        ws->parity = 0;
    }
    const uint64_t spill_words = uint64_t(tiles) * (tile / 32u);
    if (ws->tiles_cap < tiles || ws->spill_words_cap < spill_words) {
        // earlier launches on this stream may still use the old buffers
        HC_CHECK_HIP(hipStreamSynchronize(stream));
        if (ws->tiles_cap < tiles) {
            (void)hipFree(ws->counts);
            (void)hipFree(ws->slots);
            ws->counts = nullptr;
            ws->slots = nullptr;
            ws->tiles_cap = 0;
            const uint32_t cap = std::max<uint32_t>(tiles, 4096);
            if (hipMalloc(reinterpret_cast<void **>(&ws->counts), sizeof(uint32_t) * cap) != hipSuccess ||
                hipMalloc(reinterpret_cast<void **>(&ws->slots), sizeof(uint32_t) * kSlot * cap) != hipSuccess)
                return HC_ENOMEM;
            ws->tiles_cap = cap;
        }
        if (ws->spill_words_cap < spill_words) {
            (void)hipFree(ws->spill);
            ws->spill = nullptr;
            ws->spill_words_cap = 0;
            const uint64_t cap = std::max<uint64_t>(spill_words, 1u << 20);
            if (hipMalloc(reinterpret_cast<void **>(&ws->spill), sizeof(uint32_t) * cap) != hipSuccess)
                return HC_ENOMEM;
            ws->spill_words_cap = cap;
        }
    }
    *out = ws;
    *lock = std::move(held);
    return HC_OK;
}

hc_status pattern_on_device(hc_pattern *p, const DeviceCopy **out) {
    const DeviceInfo &di = device_info();
    if (!di.ok) return HC_EHIP;
    std::lock_guard<std::mutex> g(p->mu);
    for (const DeviceCopy &dc : p->dev)
        if (dc.device == di.device) {
            *out = &dc;
            return HC_OK;
        }
    DeviceCopy dc;
    dc.device = di.device;
    std::vector<uint8_t> packed = pack_table(p->data);
    packed.resize((packed.size() + 15) & ~size_t(15), 0);   // kernels copy 16-byte chunks
    if (hipMalloc(&dc.d_F, packed.size()) != hipSuccess) return HC_ENOMEM;
    const size_t xb = (size_t(p->data.m) + 15) & ~size_t(15);
    if (hipMalloc(reinterpret_cast<void **>(&dc.d_x), xb) != hipSuccess) {
        (void)hipFree(dc.d_F);
        return HC_ENOMEM;
    }
    std::vector<uint8_t> xpad(xb, 0);
    std::memcpy(xpad.data(), p->data.x.data(), size_t(p->data.m));
    if (hipMemcpy(dc.d_F, packed.data(), packed.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dc.d_x, xpad.data(), xb, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dc.d_F);
        (void)hipFree(dc.d_x);
        return HC_EHIP;
    }
    p->dev.push_back(dc);
    *out = &p->dev.back();
    return HC_OK;
}

const DeviceCopy *pattern_resident(hc_pattern *p) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> g(p->mu);
    for (const DeviceCopy &dc : p->dev)
        if (dc.device == dev) return &dc;
    return nullptr;
}

hc_launch choose_launch(const PatternData &p, int64_t n, const hc_launch *req) {
    hc_launch lc{0, 0, 0, 0};
    if (req) lc = *req;
    const Tuned t = get_tuned(p.m);
    // untuned: patterns without links (m < 2q) take the dense schedule on
    // tiles of 16384 starts, the others the searching loop on tiles of 25600
    const bool nolink = p.m < 2 * int64_t(p.q);
    const bool dense = lc.schedule == HC_SCHED_DENSE ||
                       (lc.schedule == HC_SCHED_AUTO && (t.set ? t.schedule == HC_SCHED_DENSE : nolink));
    if (lc.segment <= 0) lc.segment = t.set ? t.segment : (dense ? 64 : 100);
    if (lc.schedule == HC_SCHED_AUTO) lc.schedule = t.set ? t.schedule : (nolink ? HC_SCHED_DENSE : HC_SCHED_SEGMENT);
    if (lc.variant == HC_VARIANT_AUTO) lc.variant = t.set && t.variant ? t.variant : HC_VARIANT_HC;
    (void)n;
    return lc;
}

}  // namespace hc

using namespace hc;

extern "C" {

const char *hc_strerror(hc_status st) {
    switch (st) {
        case HC_OK: return "ok";
        case HC_EINVAL: return "invalid argument";
        case HC_ENOMEM: return "out of memory";
        case HC_EOVERFLOW: return "more results than the output capacity";
        case HC_EAGAIN: return "request not finished";
        case HC_EHIP: return "HIP runtime error or no gfx950 device";
    }
    return "unknown status";
}

hc_status hc_preprocess(const uint8_t *x, int64_t m, const hc_params *params, hc_pattern **out) {
    if (!out) return HC_EINVAL;
    *out = nullptr;
    if (!x || m < 1 || m > kMaxM) return HC_EINVAL;
    int q = params ? params->q : 0, alpha = params ? params->alpha : 0, w = params ? params->w : 0;
    if (q < 0 || alpha < 0 || w < 0) return HC_EINVAL;
    default_params(m, distinct_bytes(x, m), q, alpha, w);
    hc_status st = validate_params(m, q, alpha, w);
    if (st != HC_OK) return st;
    hc_pattern *p = new (std::nothrow) hc_pattern();
    if (!p) return HC_ENOMEM;
    try {
        build_link_table(x, m, q, alpha, w, p->data);
    } catch (...) {
        delete p;
        return HC_ENOMEM;
    }
    *out = p;
    return HC_OK;
}

hc_status hc_pattern_info(const hc_pattern *p, hc_params *used, int32_t *s, uint32_t *mask,
                          uint32_t *hv, const uint64_t **F_host, int64_t *F_words, int64_t *m) {
    if (!p) return HC_EINVAL;
    const PatternData &d = p->data;
    if (used) *used = hc_params{d.q, d.alpha, d.w};
    if (s) *s = d.s;
    if (mask) *mask = d.mask;
    if (hv) *hv = d.hv;
    if (F_host) *F_host = d.F.data();
    if (F_words) *F_words = int64_t(d.F.size());
    if (m) *m = d.m;
    return HC_OK;
}

void hc_pattern_free(hc_pattern *p) {
    if (!p) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (DeviceCopy &dc : p->dev) {
        if (hipSetDevice(dc.device) == hipSuccess) {
            (void)hipFree(dc.d_F);
            (void)hipFree(dc.d_x);
        }
    }
    if (cur >= 0 && !p->dev.empty()) (void)hipSetDevice(cur);
    delete p;
}

hc_status hc_search_async(const hc_pattern *pc, const uint8_t *d_y, int64_t n, int64_t *d_out,
                          int64_t cap, int64_t *d_count, const hc_launch *launch, void *stream) {
    if (!pc || !d_count || n < 0 || cap < 0 || (cap > 0 && !d_out)) return HC_EINVAL;
    if (n > 0 && !d_y) return HC_EINVAL;
    if (n > int64_t(0xFFFFFFFFll)) return HC_EINVAL;
    if (launch && (launch->segment < 0 || launch->segment > 4096 || launch->schedule < 0 ||
                   launch->schedule > HC_SCHED_DENSE || launch->variant < 0 ||
                   launch->variant > HC_VARIANT_SPARSE || launch->wg_per_cu < 0 ||
                   launch->wg_per_cu > 8))
        return HC_EINVAL;
    hc_pattern *p = const_cast<hc_pattern *>(pc);
    const DeviceCopy *dc = nullptr;
    hc_status st = pattern_on_device(p, &dc);
    if (st != HC_OK) return st;
    hc_launch lc = choose_launch(p->data, n, launch);
    return launch_single(p, *dc, d_y, n, d_out, cap, d_count, lc, hipStream_t(stream));
}

hc_status hc_search(const hc_pattern *p, const uint8_t *d_y, int64_t n, int64_t *d_out,
                    int64_t cap, int64_t *count, void *stream) {
    if (!p || !count) return HC_EINVAL;
    *count = 0;
    if (n >= 0 && n < p->data.m) return (cap < 0 || (cap > 0 && !d_out)) ? HC_EINVAL : HC_OK;
    // the total goes through a small per-thread pinned + device pair
    struct CountSlot {
        int64_t *d = nullptr;
        int64_t *h = nullptr;
        int device = -1;
    };
    thread_local std::map<int, CountSlot> slots;
    int dev = -1;
    HC_CHECK_HIP(hipGetDevice(&dev));
    CountSlot &cs = slots[dev];
    if (!cs.d) {
        if (hipMalloc(reinterpret_cast<void **>(&cs.d), sizeof(int64_t)) != hipSuccess) return HC_ENOMEM;
        if (hipHostMalloc(reinterpret_cast<void **>(&cs.h), sizeof(int64_t)) != hipSuccess) return HC_ENOMEM;
        cs.device = dev;
    }
    hc_status st = hc_search_async(p, d_y, n, d_out, cap, cs.d, nullptr, stream);
    if (st != HC_OK) return st;
    HC_CHECK_HIP(hipMemcpyAsync(cs.h, cs.d, sizeof(int64_t), hipMemcpyDeviceToHost,
                                hipStream_t(stream)));
    HC_CHECK_HIP(hipStreamSynchronize(hipStream_t(stream)));
    *count = *cs.h;
    return *count > cap ? HC_EOVERFLOW : HC_OK;
}

}  // extern "C"
