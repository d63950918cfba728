// Batched searching phase: many (pattern, text) pairs per call.
#include <hip/hip_runtime.h>

#include <memory>
#include <new>
#include <vector>

#include "hc_internal.h"
#include "hc_runtime.h"

using namespace hc;

extern "C" hc_status hc_search_batched(const hc_batch *b, const hc_params *params, int64_t *d_pos,
                                       int64_t cap, int64_t *d_pair_off, int64_t *total,
                                       void *stream) {
    if (!b || !total || !d_pair_off || cap < 0 || (cap > 0 && !d_pos)) return HC_EINVAL;
    *total = 0;
    if (b->n_pairs < 0 || b->n_texts < 0 || b->n_pats < 0) return HC_EINVAL;
    if (b->n_pairs > 0 && (!b->pair_pat || !b->pair_text || !b->text_off || !b->pat_off || !b->pat))
        return HC_EINVAL;
    hipStream_t s = hipStream_t(stream);
    const int64_t np = b->n_pairs;
    std::vector<std::unique_ptr<hc_pattern, void (*)(hc_pattern *)>> pats;
    pats.reserve(size_t(b->n_pats));
    for (int32_t i = 0; i < b->n_pats; ++i) {
        hc_pattern *p = nullptr;
        const int64_t m = b->pat_off[i + 1] - b->pat_off[i];
        hc_status st = hc_preprocess(b->pat + b->pat_off[i], m, params, &p);
        if (st != HC_OK) return st;
        pats.emplace_back(p, hc_pattern_free);
    }
    for (int64_t k = 0; k < np; ++k) {
        const int32_t pi = b->pair_pat[k], ti = b->pair_text[k];
        if (pi < 0 || pi >= b->n_pats || ti < 0 || ti >= b->n_texts) return HC_EINVAL;
        if (b->text_off[ti + 1] < b->text_off[ti]) return HC_EINVAL;
    }
    int64_t *d_counts = nullptr;
    HC_CHECK_HIP(hipMallocAsync(reinterpret_cast<void **>(&d_counts), sizeof(int64_t) * (np + 1), s));
    hc_status st = HC_OK;
    // pass 1: counts only
    for (int64_t k = 0; k < np && st == HC_OK; ++k) {
        const int32_t pi = b->pair_pat[k], ti = b->pair_text[k];
        st = hc_search_async(pats[pi].get(), b->d_text + b->text_off[ti],
                             b->text_off[ti + 1] - b->text_off[ti], nullptr, 0, d_counts + k,
                             nullptr, stream);
    }
    std::vector<int64_t> counts(size_t(np) + 1, 0), off(size_t(np) + 1, 0);
    if (st == HC_OK && np > 0) {
        if (hipMemcpyAsync(counts.data(), d_counts, sizeof(int64_t) * np, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = HC_EHIP;
    }
    for (int64_t k = 0; k < np; ++k) off[k + 1] = off[k] + counts[k];
    // pass 2: positions at their CSR offsets
    for (int64_t k = 0; k < np && st == HC_OK; ++k) {
        const int32_t pi = b->pair_pat[k], ti = b->pair_text[k];
        const int64_t room = std::max<int64_t>(0, std::min(cap, off[k + 1]) - off[k]);
        if (room == 0) continue;
        st = hc_search_async(pats[pi].get(), b->d_text + b->text_off[ti],
                             b->text_off[ti + 1] - b->text_off[ti], d_pos + off[k], room,
                             d_counts + k, nullptr, stream);
    }
    if (st == HC_OK && hipMemcpyAsync(d_pair_off, off.data(), sizeof(int64_t) * (np + 1),
                                      hipMemcpyHostToDevice, s) != hipSuccess)
        st = HC_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess && st == HC_OK) st = HC_EHIP;
    (void)hipFreeAsync(d_counts, s);
    (void)hipStreamSynchronize(s);
    if (st != HC_OK) return st;
    *total = off[np];
    return *total > cap ? HC_EOVERFLOW : HC_OK;
}
