// Autotuner: measures, on the caller's device text, which parameters (q,
// alpha, w) and launch shape (schedule, segment) make the searching phase
// fastest for each requested pattern length, and installs the winners as the
// library's defaults for that length bucket.
//
// For each length m, sample patterns are copied out of the text at fixed
// pseudo-random offsets (so they occur at least once, like the paper's
// randomly extracted patterns, Section 4). Phase 1 times every (q, alpha, w,
// schedule, variant) candidate on two patterns at the default segment; phase
// 2 times the four best with several segments on all sample patterns. A
// 512 MiB buffer is overwritten before each timed launch so the text comes
// from HBM. The median time per launch decides. Results never depend on the
// choice, only speed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "hc_batch.h"
#include "hc_internal.h"
#include "hc_runtime.h"

namespace hc {
namespace {

struct Cand {
    int q, alpha, w, schedule, segment, variant = HC_VARIANT_HC;
    double ms = 0;
};

uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Buffer overwritten before each timed launch, so that the text is read
// from HBM as in a run over many texts, not from the 256 MB last-level cache.
struct Flush {
    void *p = nullptr;
    size_t bytes = 0;
    ~Flush() {
        if (p) (void)hipFree(p);
    }
};

// Median milliseconds per launch of one candidate over `pats`.
hc_status time_candidate(const Cand &c, const std::vector<std::vector<uint8_t>> &pats, size_t np,
                         const uint8_t *d_y, int64_t n, int64_t *d_out, int64_t cap, int64_t *d_count,
                         const Flush &fl, hipStream_t s, double *ms) {
    std::vector<hc_pattern *> hs;
    hc_status st = HC_OK;
    for (size_t i = 0; i < np && st == HC_OK; ++i) {
        hc_params prm{c.q, c.alpha, c.w};
        hc_pattern *p = nullptr;
        st = hc_preprocess(pats[i].data(), int64_t(pats[i].size()), &prm, &p);
        if (st == HC_OK) hs.push_back(p);
    }
    const hc_launch lc{c.segment, c.schedule, c.variant, 0};
    std::vector<Timer> ev(hs.size());
    if (st == HC_OK && !hs.empty())   // warm-up: uploads the table, loads the kernel
        st = hc_search_async(hs[0], d_y, n, d_out, cap, d_count, &lc, s);
    for (size_t i = 0; i < hs.size() && st == HC_OK; ++i) {
        if (fl.p && hipMemsetAsync(fl.p, int(i & 0xFF), fl.bytes, s) != hipSuccess) {
            st = HC_EHIP;
            break;
        }
        if (hipEventCreate(&ev[i].a) != hipSuccess || hipEventCreate(&ev[i].b) != hipSuccess ||
            hipEventRecord(ev[i].a, s) != hipSuccess) {
            st = HC_EHIP;
            break;
        }
        st = hc_search_async(hs[i], d_y, n, d_out, cap, d_count, &lc, s);
        if (st == HC_OK && hipEventRecord(ev[i].b, s) != hipSuccess) st = HC_EHIP;
    }
    if (st == HC_OK && hipStreamSynchronize(s) != hipSuccess) st = HC_EHIP;
    std::vector<double> t;
    for (size_t i = 0; i < hs.size() && st == HC_OK; ++i) {
        float f = 0;
        if (hipEventElapsedTime(&f, ev[i].a, ev[i].b) != hipSuccess) st = HC_EHIP;
        t.push_back(f);
    }
    for (hc_pattern *p : hs) hc_pattern_free(p);
    if (st != HC_OK) return st;
    std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
    *ms = t[t.size() / 2];
    return HC_OK;
}

// Lane segment of the sparse variant: k shifts of m - q + 1 starts, at most
// 4096 starts.
int sparse_segment(int64_t m, int q, int k) {
    return int(std::min<int64_t>(int64_t(k) * (m - q + 1), 4096));
}

std::vector<Cand> candidates(int64_t m) {
    static const int shapes[][2] = {{8, 8}, {10, 16}, {11, 16}, {12, 16}, {12, 32}};
    std::vector<Cand> out;
    for (int q = 1; q <= std::min<int64_t>(kMaxQ, m); ++q)
        for (const auto &aw : shapes) {
            if (aw[0] > alpha_max(aw[1])) continue;
            out.push_back(Cand{q, aw[0], aw[1], HC_SCHED_SEGMENT, 100});
            if (m < 2 * q || (q <= 4 && m / q - 1 <= 3))
                out.push_back(Cand{q, aw[0], aw[1], HC_SCHED_DENSE, 100});
            // long patterns: text read in place (most cache lines never fetched)
            if (m >= 256 && q >= 3)
                out.push_back(Cand{q, aw[0], aw[1], HC_SCHED_SEGMENT, sparse_segment(m, q, 1), HC_VARIANT_SPARSE});
        }
    // m = q = 2 with alpha = 16: the hash is one-to-one on windows (the dense
    // test needs no comparison with x, and no table in LDS)
    if (m == 2) out.push_back(Cand{2, 16, 8, HC_SCHED_DENSE, 100});
    return out;
}

}  // namespace
}  // namespace hc

using namespace hc;

extern "C" hc_status hc_autotune(const uint8_t *d_y, int64_t n, const int64_t *ms, int32_t n_ms,
                                 int32_t patterns, hc_tuning *out, void *stream) {
    if (!d_y || !ms || n_ms < 1 || patterns < 1 || patterns > 64) return HC_EINVAL;
    if (n < 1 || n > int64_t(0xFFFFFFFFll)) return HC_EINVAL;
    for (int32_t i = 0; i < n_ms; ++i)
        if (ms[i] < 1 || ms[i] > kMaxM || ms[i] > n) return HC_EINVAL;
    if (!device_info().ok) return HC_EHIP;
    hipStream_t s = hipStream_t(stream);
    const int64_t cap = std::min<int64_t>(n, int64_t(1) << 25);
    int64_t *d_out = nullptr, *d_count = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&d_out), size_t(cap) * 8) != hipSuccess) return HC_ENOMEM;
    if (hipMalloc(reinterpret_cast<void **>(&d_count), 8) != hipSuccess) {
        (void)hipFree(d_out);
        return HC_ENOMEM;
    }
    Flush fl;   // best effort: without it the timings are cache-warm
    fl.bytes = size_t(512) << 20;
    if (hipMalloc(&fl.p, fl.bytes) != hipSuccess) {
        fl.p = nullptr;
        (void)hipGetLastError();
    }
    hc_status st = HC_OK;
    uint64_t seed = 0x2310157110ull;
    const size_t np = size_t(std::max(patterns, 2));
    for (int32_t i = 0; i < n_ms && st == HC_OK; ++i) {
        const int64_t m = ms[i];
        std::vector<std::vector<uint8_t>> pats(np, std::vector<uint8_t>(size_t(m)));
        for (auto &x : pats) {
            const int64_t off = int64_t(splitmix(seed) % uint64_t(n - m + 1));
            if (hipMemcpy(x.data(), d_y + off, size_t(m), hipMemcpyDeviceToHost) != hipSuccess) st = HC_EHIP;
        }
        if (st != HC_OK) break;
        // phase 1: every (q, alpha, w, schedule), two patterns
        std::vector<Cand> cs = candidates(m);
        for (Cand &c : cs) {
            st = time_candidate(c, pats, 2, d_y, n, d_out, cap, d_count, fl, s, &c.ms);
            if (st != HC_OK) break;
        }
        if (st != HC_OK) break;
        std::sort(cs.begin(), cs.end(), [](const Cand &a, const Cand &b) { return a.ms < b.ms; });
        // phase 2: the best four with several segments, all sample patterns
        Cand best{0, 0, 0, 0, 0, HC_VARIANT_HC};
        best.ms = 1e30;
        static const int hc_segs[4] = {48, 64, 80, 100};   // larger tiles do not fit the staging
        for (size_t k = 0; k < std::min<size_t>(4, cs.size()) && st == HC_OK; ++k)
            for (int j = 0; j < 4; ++j) {
                Cand c = cs[k];
                // sparse lanes take 1, 2, 4 or 8 whole shifts (at most 4096 starts)
                c.segment = c.variant == HC_VARIANT_SPARSE ? sparse_segment(m, c.q, 1 << j) : hc_segs[j];
                st = time_candidate(c, pats, np, d_y, n, d_out, cap, d_count, fl, s, &c.ms);
                if (st != HC_OK) break;
                if (c.ms < best.ms) best = c;
            }
        if (st != HC_OK) break;
        Tuned t;
        t.set = true;
        t.q = best.q;
        t.alpha = best.alpha;
        t.w = best.w;
        t.schedule = best.schedule;
        t.segment = best.segment;
        t.variant = best.variant;
        set_tuned(m, t);
        if (out) {
            out[i].m = m;
            out[i].params = hc_params{best.q, best.alpha, best.w};
            out[i].launch = hc_launch{best.segment, best.schedule, best.variant, 0};
            out[i].gbps = double(n) / (best.ms * 1e-3) / 1e9;
        }
    }
    (void)hipFree(d_out);
    (void)hipFree(d_count);
    return st;
}

extern "C" void hc_autotune_reset(void) {
    for (int b = 0; b < kBuckets; ++b) set_tuned(int64_t(1) << b, Tuned{});
    set_batch_knobs(nullptr);
}

// ----------------------------------------------------------------------------
// Batched kernel: table shape (alpha, w), tile segment, patterns per staged
// tile and resident workgroups per compute unit, timed on the caller's own
// batch (or an evenly spaced sample of its pairs).
// ----------------------------------------------------------------------------

namespace hc {
namespace {

struct BatchCand {
    BatchKnobs k;
    double ms = 1e30;
};

// Median-free minimum of two timed runs of a plan built with knobs k.
hc_status time_batch(const hc_batch &b, const BatchKnobs &k, hipStream_t s, double *ms) {
    hc_batch_plan *plan = nullptr;
    hc_status st = plan_create(&b, nullptr, k, &plan);
    if (st != HC_OK) return st;
    int64_t *d_off = nullptr, *d_pos = nullptr;
    int64_t total = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&d_off), size_t(b.n_pairs + 1) * 8) != hipSuccess) st = HC_ENOMEM;
    if (st == HC_OK) {
        st = hc_batch_plan_run(plan, nullptr, 0, d_off, &total, s);   // counts only
        if (st == HC_EOVERFLOW) st = HC_OK;
    }
    if (st == HC_OK && hipMalloc(reinterpret_cast<void **>(&d_pos), size_t(std::max<int64_t>(total, 1)) * 8) != hipSuccess)
        st = HC_ENOMEM;
    if (st == HC_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = HC_EHIP;
    double best = 1e30;
    for (int r = 0; r < 3 && st == HC_OK; ++r) {   // the first run builds the graph
        int64_t t2 = 0;
        if (hipEventRecord(e0, s) != hipSuccess) st = HC_EHIP;
        if (st == HC_OK) st = hc_batch_plan_run(plan, d_pos, total, d_off, &t2, s);
        if (st == HC_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
            st = HC_EHIP;
        float f = 0;
        if (st == HC_OK && hipEventElapsedTime(&f, e0, e1) != hipSuccess) st = HC_EHIP;
        if (st == HC_OK && r > 0) best = std::min(best, double(f));
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(d_pos);
    (void)hipFree(d_off);
    hc_batch_plan_free(plan);
    *ms = best;
    return st;
}

}  // namespace
}  // namespace hc

extern "C" hc_status hc_batch_autotune(const hc_batch *b, int64_t max_pairs, hc_batch_tuning *out, void *stream) {
    if (!b || max_pairs < 1 || b->n_pairs < 1) return HC_EINVAL;
    if (!device_info().ok) return HC_EHIP;
    hipStream_t s = hipStream_t(stream);
    // an evenly spaced sample of the pairs (every pair when there are few)
    std::vector<int32_t> pp, pt;
    const int64_t step = (b->n_pairs + max_pairs - 1) / max_pairs;
    for (int64_t k = 0; k < b->n_pairs; k += step) {
        pp.push_back(b->pair_pat[k]);
        pt.push_back(b->pair_text[k]);
    }
    hc_batch sub = *b;
    sub.pair_pat = pp.data();
    sub.pair_text = pt.data();
    sub.n_pairs = int64_t(pp.size());
    // phase 1: table shape x segment; phase 2: the best two with other
    // group sizes and workgroup caps
    static const int shapes[][2] = {{10, 16}, {11, 16}, {12, 16}, {13, 16}, {12, 32}};
    static const uint32_t segs[] = {64, 80, 100};
    std::vector<BatchCand> cs;
    hc_status st = HC_OK;
    for (const auto &aw : shapes)
        for (uint32_t seg : segs) {
            BatchCand c;
            c.k.alpha = aw[0];
            c.k.w = aw[1];
            c.k.seg = seg;
            st = time_batch(sub, c.k, s, &c.ms);
            if (st == HC_EINVAL) {   // shape does not fit (LDS): skip it
                st = HC_OK;
                continue;
            }
            if (st != HC_OK) return st;
            cs.push_back(c);
        }
    if (cs.empty()) return HC_EINVAL;
    std::sort(cs.begin(), cs.end(), [](const BatchCand &x, const BatchCand &y) { return x.ms < y.ms; });
    BatchCand best = cs[0];
    for (size_t i = 0; i < std::min<size_t>(2, cs.size()); ++i)
        for (uint32_t group : {32u, 64u, 128u})
            for (uint32_t wg : {0u, 2u}) {
                BatchCand c = cs[i];
                c.k.group = group;
                c.k.wg_per_cu = wg;
                if (group == 128u && wg == 0u) continue;   // timed in phase 1
                st = time_batch(sub, c.k, s, &c.ms);
                if (st != HC_OK) return st;
                if (c.ms < best.ms) best = c;
            }
    set_batch_knobs(&best.k);
    if (out) {
        double bytes = 0;
        for (size_t k = 0; k < pp.size(); ++k)
            bytes += double(b->text_off[pt[k] + 1] - b->text_off[pt[k]]);
        out->params = hc_params{0, best.k.alpha, best.k.w};
        out->segment = int32_t(best.k.seg);
        out->group = int32_t(best.k.group);
        out->wg_per_cu = int32_t(best.k.wg_per_cu);
        out->gbps = bytes / (best.ms * 1e-3) / 1e9;
    }
    return HC_OK;
}
