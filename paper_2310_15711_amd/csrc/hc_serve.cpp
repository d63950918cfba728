// Serving: continuous batching of search requests against resident texts.
//
// Every text is cut into chunks. A scheduler thread runs steps; one step
// searches the current chunk of every text that has active requests, for all
// of that text's active requests at once, with the batched kernel (one launch
// for all texts and requests of the step). A text's chunk cursor moves on by
// one chunk per step and wraps around, so a request admitted at any step
// starts at the cursor and is complete after one full cycle over its text;
// its positions come in two ascending runs (from its first chunk to the end
// of the text, then from the start) that are rotated into order at the end.
// New requests are admitted between steps while a pattern slot and the
// device-memory budget allow; the others wait in FIFO order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hc_batch.h"
#include "hc_runtime.h"

namespace hc {

namespace {

using Clock = std::chrono::steady_clock;

// Text bytes per request per step. Each step costs a fixed host round trip
// (build, upload, launch, read back), so larger chunks mean fewer steps per
// request: measured at 8 x 128 MiB texts, 10 K req/s, p50/p99 went from
// 4.4/7.0 ms (8 MiB) to 1.4/3.2 ms (64 MiB), 1.3/3.7 ms (128 MiB).
constexpr uint64_t kServeChunk = 64ull << 20;
constexpr uint32_t kXStride = uint32_t(kMaxM) + 32;  // pattern bytes per slot
constexpr uint64_t kResultReserve = 4096;           // positions per request per step
constexpr uint32_t kMaxSlots = 8192;

struct Request {
    uint64_t id = 0;
    int32_t text = 0;
    std::vector<uint8_t> x;
    BPat bp{};
    std::vector<uint8_t> F;        // packed table
    Clock::time_point t_submit;
    // running state
    int32_t slot = -1;
    uint64_t chunks_left = 0;
    size_t wrap_at = 0;            // positions gathered before the cursor wrapped
    bool wrapped = false;
    std::vector<int64_t> pos;
    bool done = false;
    hc_status status = HC_OK;
};

struct Text {
    const uint8_t *d = nullptr;
    uint64_t n = 0;
    uint64_t chunks = 0;
    uint64_t cursor = 0;           // next chunk to search
};

}  // namespace

}  // namespace hc

using namespace hc;

struct hc_server {
    int device = -1;
    std::vector<Text> texts;
    int alpha = 12, w = 16, q_req = 0;
    uint32_t table_bytes = 0;
    uint64_t budget = 0, per_request = 0;
    uint32_t slots = 0;

    // device state (scheduler thread only, after creation)
    hipStream_t stream = nullptr;
    BatchDev D;
    DeviceBuf Fpool, xpool, d_pos, d_off;
    int64_t *h_pos = nullptr;   // pinned
    size_t h_pos_cap = 0;
    int64_t *h_off = nullptr;   // pinned
    size_t h_off_cap = 0;
    unsigned long long *h_ctl = nullptr;   // pinned, 4 words

    // shared state
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_id = 1;
    std::deque<std::shared_ptr<Request>> pending;
    std::vector<std::shared_ptr<Request>> active;   // by slot (null = free)
    std::unordered_map<uint64_t, std::shared_ptr<Request>> by_id;
    std::deque<uint64_t> done_q;   // completed ids not yet taken by hc_serve_next_done
    uint64_t used_bytes = 0;
    std::vector<double> lat_us;
    double busy_s = 0, bytes_searched = 0;
    hc_status fatal = HC_OK;

    std::thread worker;

    ~hc_server() {
        if (h_up) (void)hipHostFree(h_up);
        if (h_pos) (void)hipHostFree(h_pos);
        if (h_off) (void)hipHostFree(h_off);
        if (h_ctl) (void)hipHostFree(h_ctl);
        if (stream) (void)hipStreamDestroy(stream);
    }

    hc_status pinned(int64_t *&p, size_t &cap, size_t need) {
        if (cap >= need && p) return HC_OK;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        const size_t n = std::max<size_t>(need, 1024);
        if (hipHostMalloc(reinterpret_cast<void **>(&p), n * 8, hipHostMallocDefault) != hipSuccess)
            return HC_ENOMEM;
        cap = n;
        return HC_OK;
    }

    // Admits pending requests while slots and budget allow (lock held).
    void admit(std::vector<std::shared_ptr<Request>> &uploads) {
        while (!pending.empty()) {
            auto r = pending.front();
            const Text &t = texts[r->text];
            if (t.n < r->x.size()) {   // no window fits: complete at once
                pending.pop_front();
                r->done = true;
                done_q.push_back(r->id);
                lat_us.push_back(std::chrono::duration<double, std::micro>(Clock::now() - r->t_submit).count());
                continue;
            }
            if (used_bytes + per_request > budget) break;
            int32_t slot = -1;
            for (uint32_t i = 0; i < slots; ++i)
                if (!active[i]) {
                    slot = int32_t(i);
                    break;
                }
            if (slot < 0) break;
            pending.pop_front();
            r->slot = slot;
            r->chunks_left = t.chunks;
            r->bp.x_off = uint32_t(slot) * kXStride;
            active[slot] = r;
            used_bytes += per_request;
            uploads.push_back(r);
        }
    }

    hc_status step(std::vector<std::shared_ptr<Request>> &members, uint64_t &bytes);
    hc_status upload(const std::vector<std::shared_ptr<Request>> &reqs);

    // staging of newly admitted patterns: one copy and one scatter per step
    uint8_t *h_up = nullptr;   // pinned
    size_t h_up_cap = 0;
    DeviceBuf d_up, d_up_slots;
    void run();
};

// Tables and bytes of newly admitted requests into their slots: packed in
// pinned memory, copied once, scattered by one kernel. The step that follows
// synchronises the stream before the staging buffer is reused.
hc_status hc_server::upload(const std::vector<std::shared_ptr<Request>> &reqs) {
    const size_t entry = size_t(table_bytes) + kXStride, need = entry * reqs.size();
    if (h_up_cap < need) {
        if (h_up) (void)hipHostFree(h_up);
        h_up = nullptr;
        h_up_cap = 0;
        if (hipHostMalloc(reinterpret_cast<void **>(&h_up), need, hipHostMallocDefault) != hipSuccess)
            return HC_ENOMEM;
        h_up_cap = need;
    }
    std::vector<uint32_t> slot(reqs.size());
    for (size_t i = 0; i < reqs.size(); ++i) {
        uint8_t *e = h_up + i * entry;
        std::memcpy(e, reqs[i]->F.data(), table_bytes);
        std::memset(e + table_bytes, 0, kXStride);
        std::memcpy(e + table_bytes, reqs[i]->x.data(), reqs[i]->x.size());
        slot[i] = uint32_t(reqs[i]->slot);
    }
    if (d_up.ensure(need) != HC_OK) return HC_ENOMEM;
    if (hipMemcpyAsync(d_up.p, h_up, need, hipMemcpyHostToDevice, stream) != hipSuccess) return HC_EHIP;
    hc_status st = d_up_slots.upload(slot.data(), slot.size() * 4, stream);
    if (st != HC_OK) return st;
    // the slot list is pageable: wait for its copy before the vector goes
    if (hipStreamSynchronize(stream) != hipSuccess) return HC_EHIP;
    return scatter_patterns(d_up.as<uint8_t>(), d_up_slots.as<uint32_t>(), uint32_t(reqs.size()), table_bytes,
                            kXStride, Fpool.as<uint8_t>(), xpool.as<uint8_t>(), stream);
}

// One step: the current chunk of every text with active requests, for all
// of them (`members`, in pair order); their positions are appended.
hc_status hc_server::step(std::vector<std::shared_ptr<Request>> &members, uint64_t &bytes) {
    auto fail = [&](const char *where, hc_status st) {
        const hipError_t e = hipGetLastError();
        std::fprintf(stderr, "hc_serve: step failed in %s: %s (HIP: %s; launch: %s)\n", where, hc_strerror(st),
                     hipGetErrorString(e), hipGetErrorString(D.last_error));
        return st;
    };
    BatchHost H;
    std::vector<std::pair<uint32_t, uint32_t>> pairs;
    std::vector<int32_t> text_of_view;
    std::vector<uint64_t> base_of_view;
    uint32_t max_m = 1;
    {
        std::vector<int32_t> view_of_text(texts.size(), -1);
        H.pats.assign(slots, BPat{});
        for (auto &r : members) {
            int32_t &v = view_of_text[r->text];
            if (v < 0) {
                const Text &t = texts[r->text];
                v = int32_t(H.views.size());
                const uint64_t base = t.cursor * kServeChunk;
                H.views.push_back(TextView{t.d + base, t.n - base, std::min<uint64_t>(kServeChunk, t.n - base)});
                text_of_view.push_back(r->text);
                base_of_view.push_back(base);
            }
            H.pats[r->slot] = r->bp;
            pairs.push_back({uint32_t(r->slot), uint32_t(v)});
            max_m = std::max<uint32_t>(max_m, r->bp.m);
        }
        // a view needs the halo of its longest pattern only
        std::vector<uint32_t> span(H.views.size(), 1);
        for (auto &r : members) {
            const int32_t v = view_of_text[r->text];
            span[v] = std::max<uint32_t>(span[v], r->bp.m);
        }
        for (size_t v = 0; v < H.views.size(); ++v)
            H.views[v].len = std::min<uint64_t>(H.views[v].len, H.views[v].start_limit + span[v] - 1);
    }
    // geometry for the longest active pattern, rounded up to limit re-tuning
    uint32_t bucket = 64;
    while (bucket < max_m) bucket *= 2;
    if (bucket != D.max_m || D.tile == 0) {
        hc_status st = batch_geometry(D, std::min<uint32_t>(bucket, uint32_t(kMaxM)), table_bytes, uint32_t(w));
        if (st != HC_OK) return fail("geometry", st);
    }
    batch_build(H, pairs, D.tile, kBatchGroup);
    hc_status st = batch_upload(H, D, stream);
    if (st != HC_OK) return fail("upload", st);
    const size_t np = pairs.size();
    if (d_off.ensure((np + 1) * 8) != HC_OK || pinned(h_off, h_off_cap, np + 1) != HC_OK)
        return fail("offsets", HC_ENOMEM);
    int64_t cap = int64_t(np * kResultReserve);
    if (d_pos.bytes / 8 > size_t(cap)) cap = int64_t(d_pos.bytes / 8);
    if (d_pos.ensure(size_t(cap) * 8) != HC_OK) return fail("positions", HC_ENOMEM);
    // a second run, with room for everything the first one counted, fits;
    // two more runs are allowed before the step fails
    unsigned long long reserved_first = 0;
    for (int attempt = 0; attempt < 4; ++attempt) {
        if ((st = batch_enqueue(D, d_pos.as<int64_t>(), cap, d_off.as<int64_t>(), stream)) != HC_OK)
            return fail("launch", st);
        if (hipMemcpyAsync(h_ctl, D.ctl.p, 4 * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipMemcpyAsync(h_off, d_off.p, (np + 1) * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return fail("counts", HC_EHIP);
        const uint64_t total = uint64_t(h_off[np]);
        const bool short_scratch = h_ctl[2] != 0ull, short_out = total > uint64_t(cap);
        if (short_scratch && batch_grow_scratch(D, h_ctl[1], total) != HC_OK) return fail("scratch", HC_ENOMEM);
        if (short_out) {
            cap = int64_t(total);
            if (d_pos.ensure(size_t(cap) * 8) != HC_OK) return fail("positions", HC_ENOMEM);
        }
        if (short_scratch || short_out) {
            if (attempt >= 1)
                std::fprintf(stderr,
                             "hc_serve: second run short (scratch %d, out %d, total %llu, cap %lld, reserved %llu "
                             "then %llu, scratch %llu, grid %u, items %u, entries %llu)\n",
                             int(short_scratch), int(short_out), (unsigned long long)total, (long long)cap,
                             reserved_first, h_ctl[1], (unsigned long long)D.scratch_cap, D.grid, D.n_items,
                             (unsigned long long)D.n_entries);
            reserved_first = h_ctl[1];
            continue;
        }
        if (pinned(h_pos, h_pos_cap, total) != HC_OK) return fail("host positions", HC_ENOMEM);
        if (total && (hipMemcpyAsync(h_pos, d_pos.p, total * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                      hipStreamSynchronize(stream) != hipSuccess))
            return fail("positions copy", HC_EHIP);
        std::vector<int32_t> view_of_text(texts.size(), -1);
        for (size_t v = 0; v < text_of_view.size(); ++v) view_of_text[text_of_view[v]] = int32_t(v);
        bytes = 0;
        for (size_t k = 0; k < np; ++k) {
            Request &r = *members[k];
            const int32_t v = view_of_text[r.text];
            const int64_t base = int64_t(base_of_view[v]);
            for (int64_t i = h_off[k]; i < h_off[k + 1]; ++i) r.pos.push_back(h_pos[i] + base);
            bytes += H.views[v].start_limit;
        }
        return HC_OK;
    }
    return fail("retry", HC_EHIP);
}

void hc_server::run() {
    if (hipSetDevice(device) != hipSuccess) {
        std::fprintf(stderr, "hc_serve: hipSetDevice(%d) failed\n", device);
        std::lock_guard<std::mutex> g(mu);
        fatal = HC_EHIP;
        cv_done.notify_all();
        return;
    }
    for (;;) {
        std::vector<std::shared_ptr<Request>> uploads, members;
        {
            std::unique_lock<std::mutex> g(mu);
            for (;;) {
                if (stop) return;
                admit(uploads);
                bool any = !uploads.empty();
                for (auto &r : active)
                    if (r) any = true;
                if (any) break;
                cv_done.notify_all();   // immediate completions
                cv_work.wait(g);
            }
            for (auto &r : active)
                if (r) members.push_back(r);
        }
        const auto t0 = Clock::now();
        hc_status st = HC_OK;
        if (!uploads.empty()) st = upload(uploads);
        uint64_t bytes = 0;
        if (st == HC_OK) st = step(members, bytes);
        const double dt = std::chrono::duration<double>(Clock::now() - t0).count();
        std::lock_guard<std::mutex> g(mu);
        busy_s += dt;
        bytes_searched += double(bytes);
        std::vector<bool> moved(texts.size(), false);
        for (auto &r : members) {
            Text &t = texts[r->text];
            if (!moved[r->text]) {
                moved[r->text] = true;
                t.cursor = (t.cursor + 1) % t.chunks;
            }
        }
        const auto now = Clock::now();
        for (auto &r : members) {
            const Text &t = texts[r->text];
            if (st != HC_OK) {
                r->status = st;
                r->chunks_left = 1;
            }
            if (!r->wrapped && t.cursor == 0 && r->chunks_left > 1) {
                r->wrapped = true;
                r->wrap_at = r->pos.size();
            }
            if (--r->chunks_left == 0) {
                if (r->wrapped)
                    std::rotate(r->pos.begin(), r->pos.begin() + ptrdiff_t(r->wrap_at), r->pos.end());
                r->done = true;
                done_q.push_back(r->id);
                active[r->slot] = nullptr;
                used_bytes -= per_request;
                lat_us.push_back(std::chrono::duration<double, std::micro>(now - r->t_submit).count());
            }
        }
        if (st != HC_OK) fatal = st;
        cv_done.notify_all();
    }
}

extern "C" {

hc_status hc_serve_create(const uint8_t *const *d_texts, const int64_t *n, int32_t n_texts,
                          int64_t device_mem_budget, const hc_params *params, hc_server **out) {
    if (!out) return HC_EINVAL;
    *out = nullptr;
    if (n_texts < 1 || !d_texts || !n || device_mem_budget <= 0) return HC_EINVAL;
    for (int32_t t = 0; t < n_texts; ++t)
        if (n[t] < 0 || (n[t] > 0 && !d_texts[t])) return HC_EINVAL;
    const DeviceInfo &di = device_info();
    if (!di.ok) return HC_EHIP;
    std::unique_ptr<hc_server> S(new (std::nothrow) hc_server());
    if (!S) return HC_ENOMEM;
    S->device = di.device;
    hc_status st = batch_shape(params, S->alpha, S->w, S->table_bytes);
    if (st != HC_OK) return st;
    S->q_req = params ? params->q : 0;
    if (S->q_req < 0 || S->q_req > kMaxQ) return HC_EINVAL;
    S->texts.resize(size_t(n_texts));
    for (int32_t t = 0; t < n_texts; ++t) {
        Text &x = S->texts[t];
        x.d = d_texts[t];
        x.n = uint64_t(n[t]);
        x.chunks = std::max<uint64_t>(1, (x.n + kServeChunk - 1) / kServeChunk);
    }
    // the budget counts each in-flight request's table, bytes and result room
    S->per_request = uint64_t(S->table_bytes) + kXStride + kResultReserve * 8u;
    S->budget = uint64_t(device_mem_budget);
    if (S->budget < S->per_request) return HC_EINVAL;
    S->slots = uint32_t(std::min<uint64_t>(kMaxSlots, S->budget / S->per_request));
    S->active.assign(S->slots, nullptr);
    if (S->Fpool.ensure(size_t(S->slots) * S->table_bytes) != HC_OK ||
        S->xpool.ensure(size_t(S->slots) * kXStride + 64) != HC_OK)
        return HC_ENOMEM;
    if (hipMemset(S->xpool.p, 0, S->xpool.bytes) != hipSuccess) return HC_EHIP;
    S->D.Fs = S->Fpool.as<uint8_t>();   // pattern index = slot
    S->D.xs = S->xpool.as<uint8_t>();
    S->D.Fs_bytes = S->Fpool.bytes;
    S->D.xs_bytes = S->xpool.bytes;
    if (hipHostMalloc(reinterpret_cast<void **>(&S->h_ctl), 64, hipHostMallocDefault) != hipSuccess)
        return HC_ENOMEM;
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) return HC_EHIP;
    // the texts were written on other streams: make them visible to ours
    if (hipDeviceSynchronize() != hipSuccess) return HC_EHIP;
    hc_server *raw = S.get();
    try {
        S->worker = std::thread([raw] { raw->run(); });
    } catch (...) {
        return HC_ENOMEM;
    }
    *out = S.release();
    return HC_OK;
}

hc_status hc_serve_submit(hc_server *s, int32_t text_id, const uint8_t *x, int64_t m, uint64_t *req_id) {
    if (!s || !req_id || !x || m < 1 || m > kMaxM) return HC_EINVAL;
    if (text_id < 0 || size_t(text_id) >= s->texts.size()) return HC_EINVAL;
    auto r = std::make_shared<Request>();
    r->text = text_id;
    r->x.assign(x, x + m);
    r->F.assign(s->table_bytes, 0);
    // preprocessing runs on the caller's thread
    hc_status st = pack_one(x, m, s->q_req, s->alpha, s->w, s->table_bytes, r->bp, r->F.data());
    if (st != HC_OK) return st;
    std::lock_guard<std::mutex> g(s->mu);
    if (s->fatal != HC_OK) return s->fatal;
    r->id = s->next_id++;
    r->t_submit = Clock::now();
    s->by_id[r->id] = r;
    s->pending.push_back(r);
    *req_id = r->id;
    s->cv_work.notify_one();
    return HC_OK;
}

hc_status hc_serve_poll(hc_server *s, uint64_t req_id, int64_t *out, int64_t cap, int64_t *count,
                        int32_t timeout_us) {
    if (!s || !count || cap < 0 || (cap > 0 && !out)) return HC_EINVAL;
    *count = 0;
    std::unique_lock<std::mutex> g(s->mu);
    auto it = s->by_id.find(req_id);
    if (it == s->by_id.end()) return HC_EINVAL;
    std::shared_ptr<Request> r = it->second;
    if (!r->done && timeout_us > 0)
        s->cv_done.wait_for(g, std::chrono::microseconds(timeout_us),
                            [&] { return r->done || s->fatal != HC_OK; });
    if (!r->done) return s->fatal != HC_OK ? s->fatal : HC_EAGAIN;
    if (r->status != HC_OK) {
        s->by_id.erase(it);
        return r->status;
    }
    const int64_t c = int64_t(r->pos.size());
    *count = c;
    if (cap > 0) std::memcpy(out, r->pos.data(), size_t(std::min(c, cap)) * 8);
    if (c > cap) return HC_EOVERFLOW;   // kept: poll again with room for all
    s->by_id.erase(it);
    if (s->done_q.size() > 2 * s->by_id.size() + 1024) {   // drop released ids
        std::deque<uint64_t> keep;
        for (uint64_t id : s->done_q)
            if (s->by_id.count(id)) keep.push_back(id);
        s->done_q.swap(keep);
    }
    return HC_OK;
}

hc_status hc_serve_next_done(hc_server *s, uint64_t *req_id, int32_t timeout_us) {
    if (!s || !req_id) return HC_EINVAL;
    *req_id = 0;
    std::unique_lock<std::mutex> g(s->mu);
    auto ready = [&] {
        // ids already released by hc_serve_poll are skipped
        while (!s->done_q.empty() && !s->by_id.count(s->done_q.front())) s->done_q.pop_front();
        return !s->done_q.empty() || s->fatal != HC_OK;
    };
    if (!ready() && timeout_us > 0)
        s->cv_done.wait_for(g, std::chrono::microseconds(timeout_us), ready);
    if (s->done_q.empty()) return s->fatal != HC_OK ? s->fatal : HC_EAGAIN;
    *req_id = s->done_q.front();
    s->done_q.pop_front();
    return HC_OK;
}

hc_status hc_serve_stats(hc_server *s, double *p50_us, double *p99_us, double *agg_gbps, int64_t *done) {
    if (!s) return HC_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    std::vector<double> v = s->lat_us;
    auto pct = [&](double p) -> double {
        if (v.empty()) return 0.0;
        const size_t k = std::min(v.size() - 1, size_t(p * double(v.size() - 1) + 0.5));
        std::nth_element(v.begin(), v.begin() + ptrdiff_t(k), v.end());
        return v[k];
    };
    if (p50_us) *p50_us = pct(0.50);
    if (p99_us) *p99_us = pct(0.99);
    if (agg_gbps) *agg_gbps = s->busy_s > 0 ? s->bytes_searched / s->busy_s / 1e9 : 0.0;
    if (done) *done = int64_t(s->lat_us.size());
    return HC_OK;
}

hc_status hc_serve_destroy(hc_server *s) {
    if (!s) return HC_EINVAL;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    delete s;
    return HC_OK;
}

}  // extern "C"
