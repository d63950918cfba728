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
// New requests are admitted whenever a step is built, while a pattern slot and
// the device-memory budget allow; the others wait in FIFO order.
//
// Steps are pipelined: each has its own work list, result buffers and host
// staging (a Step), and up to kSteps of them are in flight on the server's
// stream. While the device runs step k + 1, the host reads back step k's
// counts, copies its positions on a second stream and hands them to the
// requests, then builds and enqueues step k + 2. Results are taken in step
// order, so every request sees its chunks in order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
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

// Text bytes per request per step. Larger chunks mean fewer steps (each with
// a fixed host cost) per request; smaller ones a shorter wait for a request
// that arrives while a step runs.
constexpr uint64_t kServeChunk = 64ull << 20;
constexpr uint32_t kXStride = uint32_t(kMaxM) + 32;  // pattern bytes per slot
constexpr uint64_t kResultReserve = 4096;           // positions per request per step
constexpr uint32_t kMaxSlots = 8192;
constexpr int kSteps = 2;                           // steps in flight

struct Request {
    uint64_t id = 0;
    int32_t text = 0;
    std::vector<uint8_t> x;
    BPat bp{};
    std::vector<uint8_t> F;        // packed table
    Clock::time_point t_submit;
    // scheduler state
    int32_t slot = -1;
    uint64_t to_issue = 0;         // chunks not yet put into a step
    uint64_t to_take = 0;          // chunks whose positions are not yet taken
    bool started = false;          // some chunk was put into a step
    size_t wrap_at = 0;            // positions gathered before the cursor wrapped
    bool wrapped = false;
    std::vector<int64_t> pos;
    bool done = false;             // set under the server lock once pos is final
    hc_status status = HC_OK;
};

struct Text {
    const uint8_t *d = nullptr;
    uint64_t n = 0;
    uint64_t chunks = 0;
    uint64_t cursor = 0;           // next chunk to search
};

// Pinned host array that only grows.
template <typename T>
struct Pinned {
    T *p = nullptr;
    size_t cap = 0;
    Pinned() = default;
    Pinned(const Pinned &) = delete;
    Pinned &operator=(const Pinned &) = delete;
    ~Pinned() {
        if (p) (void)hipHostFree(p);
    }
    hc_status ensure(size_t n) {
        if (cap >= n && p) return HC_OK;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        const size_t c = std::max<size_t>(n, 1024);
        if (hipHostMalloc(reinterpret_cast<void **>(&p), c * sizeof(T), hipHostMallocDefault) != hipSuccess)
            return HC_ENOMEM;
        cap = c;
        return HC_OK;
    }
};

// One step's state. Owned by the scheduler thread; reused once its results
// have been taken (then none of its buffers is read by the device any more).
struct Step {
    BatchDev D;
    BatchHost H;
    DeviceBuf d_pos, d_off, d_up, d_up_slots;
    Pinned<int64_t> h_pos, h_off;
    Pinned<unsigned long long> h_ctl;
    Pinned<uint8_t> h_up;
    Pinned<uint32_t> h_up_slots;
    std::vector<std::shared_ptr<Request>> members;   // pair order
    std::vector<uint64_t> base;                      // per member: text offset of its chunk
    std::vector<uint8_t> wraps;                      // per member: chunk 0 after earlier chunks
    int64_t cap = 0;
    uint64_t bytes = 0;                              // text bytes searched (over members)
    hipEvent_t counted = nullptr, copied = nullptr;
    ~Step() {
        if (counted) (void)hipEventDestroy(counted);
        if (copied) (void)hipEventDestroy(copied);
    }
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
    hipStream_t stream = nullptr;     // steps, in order
    hipStream_t copy_stream = nullptr;   // positions of finished steps
    DeviceBuf Fpool, xpool, patpool;
    Step steps[kSteps];

    // shared state
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_id = 1;
    std::deque<std::shared_ptr<Request>> pending;
    std::vector<std::shared_ptr<Request>> active;   // by slot (null = free)
    std::vector<int32_t> free_slots;                // the null entries of `active`
    std::unordered_map<uint64_t, std::shared_ptr<Request>> by_id;
    std::deque<uint64_t> done_q;   // completed ids not yet taken by hc_serve_next_done
    uint64_t used_bytes = 0;
    std::vector<double> lat_us;
    double busy_s = 0, bytes_searched = 0;
    hc_status fatal = HC_OK;

    std::thread worker;

    ~hc_server() {
        if (stream) (void)hipStreamDestroy(stream);
        if (copy_stream) (void)hipStreamDestroy(copy_stream);
    }

    void complete(Request &r, Clock::time_point now) {   // lock held
        r.done = true;
        done_q.push_back(r.id);
        lat_us.push_back(std::chrono::duration<double, std::micro>(now - r.t_submit).count());
    }

    // Admits pending requests while slots and budget allow (lock held).
    void admit(std::vector<std::shared_ptr<Request>> &uploads) {
        while (!pending.empty()) {
            auto r = pending.front();
            const Text &t = texts[r->text];
            if (t.n < r->x.size()) {   // no window fits: complete at once
                pending.pop_front();
                complete(*r, Clock::now());
                continue;
            }
            if (used_bytes + per_request > budget || free_slots.empty()) break;
            const int32_t slot = free_slots.back();
            free_slots.pop_back();
            pending.pop_front();
            r->slot = slot;
            r->to_issue = r->to_take = t.chunks;
            r->bp.x_off = uint32_t(slot) * kXStride;
            active[slot] = r;
            used_bytes += per_request;
            uploads.push_back(r);
        }
    }

    bool build(Step &S, std::vector<std::shared_ptr<Request>> &uploads, bool may_wait);
    hc_status enqueue(Step &S, const std::vector<std::shared_ptr<Request>> &uploads);
    hc_status collect(Step &S);
    void finish(Step &S, hc_status st);
    void run();
};

// Picks the members of the next step (admitting pending requests first) and
// lays out its work list. Returns false when there is nothing to search (after
// waiting for work when `may_wait`, i.e. no step is in flight) or on stop.
bool hc_server::build(Step &S, std::vector<std::shared_ptr<Request>> &uploads, bool may_wait) {
    S.members.clear();
    S.base.clear();
    S.wraps.clear();
    uploads.clear();
    {
        std::unique_lock<std::mutex> g(mu);
        for (;;) {
            if (stop) return false;
            admit(uploads);
            for (auto &r : active)
                if (r && r->to_issue > 0) S.members.push_back(r);
            if (!S.members.empty()) break;
            cv_done.notify_all();   // immediate completions
            if (!may_wait) return false;
            cv_work.wait(g);
        }
    }
    // the scheduler alone changes the fields below
    BatchHost &H = S.H;
    H.views.clear();
    H.pats.assign(slots, BPat{});
    std::vector<int32_t> view_of_text(texts.size(), -1);
    std::vector<uint32_t> span;
    std::vector<std::pair<uint32_t, uint32_t>> pairs;
    uint32_t max_m = 1;
    S.bytes = 0;
    for (auto &r : S.members) {
        int32_t &v = view_of_text[r->text];
        const Text &t = texts[r->text];
        if (v < 0) {
            v = int32_t(H.views.size());
            const uint64_t base = t.cursor * kServeChunk;
            H.views.push_back(TextView{t.d + base, t.n - base, std::min<uint64_t>(kServeChunk, t.n - base)});
            span.push_back(1);
        }
        span[v] = std::max<uint32_t>(span[v], r->bp.m);
        H.pats[r->slot] = r->bp;
        pairs.push_back({uint32_t(r->slot), uint32_t(v)});
        max_m = std::max<uint32_t>(max_m, r->bp.m);
        S.base.push_back(t.cursor * kServeChunk);
        S.wraps.push_back(uint8_t(t.cursor == 0 && r->started));
        r->started = true;
        --r->to_issue;
        S.bytes += H.views[v].start_limit;
    }
    // a view needs the halo of its longest pattern only
    for (size_t v = 0; v < H.views.size(); ++v)
        H.views[v].len = std::min<uint64_t>(H.views[v].len, H.views[v].start_limit + span[v] - 1);
    // every text of this step moves on by one chunk
    for (size_t t = 0; t < texts.size(); ++t)
        if (view_of_text[t] >= 0) texts[t].cursor = (texts[t].cursor + 1) % texts[t].chunks;
    // geometry for the longest pattern, rounded up to limit re-tuning
    uint32_t bucket = 64;
    while (bucket < max_m) bucket *= 2;
    bucket = std::min<uint32_t>(bucket, uint32_t(kMaxM));
    if (bucket != S.D.max_m || S.D.tile == 0) {
        if (batch_geometry(S.D, bucket, table_bytes, uint32_t(w)) != HC_OK) S.D.tile = 0;
    }
    if (S.D.tile) batch_build(H, pairs, S.D.tile, S.D.group);
    return true;
}

// Stages the tables of newly admitted requests and enqueues the step: the
// scatter of the new tables, the batched search, and the read-back of the
// control words and the per-pair offsets, then records S.counted.
hc_status hc_server::enqueue(Step &S, const std::vector<std::shared_ptr<Request>> &uploads) {
    if (S.D.tile == 0) return HC_EINVAL;
    if (!uploads.empty()) {
        const size_t entry = size_t(table_bytes) + kXStride + sizeof(BPat), need = entry * uploads.size();
        if (S.h_up.ensure(need) != HC_OK || S.h_up_slots.ensure(uploads.size()) != HC_OK ||
            S.d_up.ensure(need) != HC_OK || S.d_up_slots.ensure(uploads.size() * 4) != HC_OK)
            return HC_ENOMEM;
        for (size_t i = 0; i < uploads.size(); ++i) {
            uint8_t *e = S.h_up.p + i * entry;
            std::memcpy(e, uploads[i]->F.data(), table_bytes);
            std::memset(e + table_bytes, 0, kXStride);
            std::memcpy(e + table_bytes, uploads[i]->x.data(), uploads[i]->x.size());
            std::memcpy(e + table_bytes + kXStride, &uploads[i]->bp, sizeof(BPat));
            S.h_up_slots.p[i] = uint32_t(uploads[i]->slot);
        }
        if (hipMemcpyAsync(S.d_up.p, S.h_up.p, need, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(S.d_up_slots.p, S.h_up_slots.p, uploads.size() * 4, hipMemcpyHostToDevice,
                           stream) != hipSuccess)
            return HC_EHIP;
        hc_status st = scatter_patterns(S.d_up.as<uint8_t>(), S.d_up_slots.as<uint32_t>(), uint32_t(uploads.size()),
                                        table_bytes, kXStride, Fpool.as<uint8_t>(), xpool.as<uint8_t>(),
                                        patpool.as<BPat>(), stream);
        if (st != HC_OK) return st;
    }
    S.D.Fs = Fpool.as<uint8_t>();   // pattern index = slot
    S.D.xs = xpool.as<uint8_t>();
    S.D.Fs_bytes = Fpool.bytes;
    S.D.xs_bytes = xpool.bytes;
    S.D.pats_dev = patpool.as<BPat>();
    hc_status st = batch_upload(S.H, S.D, stream);
    if (st != HC_OK) return st;
    const size_t np = S.members.size();
    if (S.d_off.ensure((np + 1) * 8) != HC_OK || S.h_off.ensure(np + 1) != HC_OK || S.h_ctl.ensure(4) != HC_OK)
        return HC_ENOMEM;
    S.cap = std::max<int64_t>(int64_t(np * kResultReserve), int64_t(S.d_pos.bytes / 8));
    if (S.d_pos.ensure(size_t(S.cap) * 8) != HC_OK) return HC_ENOMEM;
    if ((st = batch_enqueue(S.D, S.d_pos.as<int64_t>(), S.cap, S.d_off.as<int64_t>(), stream)) != HC_OK) return st;
    if (hipMemcpyAsync(S.h_ctl.p, S.D.ctl.p, 4 * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(S.h_off.p, S.d_off.p, (np + 1) * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipEventRecord(S.counted, stream) != hipSuccess)
        return HC_EHIP;
    return HC_OK;
}

// Waits for a step's counts, runs it again if its scratch or output was too
// small (once: the second run has room for everything the first counted),
// and copies its positions to the host on the copy stream.
hc_status hc_server::collect(Step &S) {
    if (hipEventSynchronize(S.counted) != hipSuccess) return HC_EHIP;
    const size_t np = S.members.size();
    for (int attempt = 0;; ++attempt) {
        const uint64_t total = uint64_t(S.h_off.p[np]);
        const bool short_scratch = S.h_ctl.p[2] != 0ull, short_out = total > uint64_t(S.cap);
        if (!short_scratch && !short_out) break;
        if (attempt == 1) return HC_EHIP;   // cannot happen (see batch_grow_scratch)
        if (short_scratch && batch_grow_scratch(S.D, S.h_ctl.p[1], total) != HC_OK) return HC_ENOMEM;
        if (short_out) {
            // growing may free the old buffer: nothing of this step is in
            // flight any more (its counts arrived)
            S.cap = int64_t(total);
            if (S.d_pos.ensure(size_t(S.cap) * 8) != HC_OK) return HC_ENOMEM;
        }
        hc_status st = short_scratch
                           ? batch_enqueue(S.D, S.d_pos.as<int64_t>(), S.cap, S.d_off.as<int64_t>(), stream)
                           : batch_emit(S.D, S.d_pos.as<int64_t>(), S.cap, S.d_off.as<int64_t>(), stream);
        if (st != HC_OK) return st;
        if (hipMemcpyAsync(S.h_ctl.p, S.D.ctl.p, 4 * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipMemcpyAsync(S.h_off.p, S.d_off.p, (np + 1) * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipEventRecord(S.counted, stream) != hipSuccess || hipEventSynchronize(S.counted) != hipSuccess)
            return HC_EHIP;
    }
    const uint64_t total = uint64_t(S.h_off.p[np]);
    if (S.h_pos.ensure(total) != HC_OK) return HC_ENOMEM;
    if (total) {
        if (hipStreamWaitEvent(copy_stream, S.counted, 0) != hipSuccess ||
            hipMemcpyAsync(S.h_pos.p, S.d_pos.p, total * 8, hipMemcpyDeviceToHost, copy_stream) != hipSuccess ||
            hipEventRecord(S.copied, copy_stream) != hipSuccess || hipEventSynchronize(S.copied) != hipSuccess)
            return HC_EHIP;
    }
    return HC_OK;
}

// Hands a collected step's positions to its requests (in step order) and
// completes the requests whose last chunk this was.
void hc_server::finish(Step &S, hc_status st) {
    const size_t np = S.members.size();
    const auto now = Clock::now();
    std::lock_guard<std::mutex> g(mu);
    if (st == HC_OK) bytes_searched += double(S.bytes);
    for (size_t k = 0; k < np; ++k) {
        Request &r = *S.members[k];
        if (r.done) continue;   // failed by an earlier step
        if (st != HC_OK) {
            r.status = st;
            r.to_issue = 0;
            r.to_take = 0;
        } else {
            if (S.wraps[k] && !r.wrapped) {
                r.wrapped = true;
                r.wrap_at = r.pos.size();
            }
            const int64_t base = int64_t(S.base[k]);
            for (int64_t i = S.h_off.p[k]; i < S.h_off.p[k + 1]; ++i) r.pos.push_back(S.h_pos.p[i] + base);
            --r.to_take;
        }
        if (r.to_take == 0) {
            if (r.wrapped) std::rotate(r.pos.begin(), r.pos.begin() + ptrdiff_t(r.wrap_at), r.pos.end());
            complete(r, now);
            active[r.slot] = nullptr;
            free_slots.push_back(r.slot);
            used_bytes -= per_request;
        }
    }
    if (st != HC_OK) fatal = st;
    cv_done.notify_all();
}

void hc_server::run() {
    if (hipSetDevice(device) != hipSuccess) {
        std::fprintf(stderr, "hc_serve: hipSetDevice(%d) failed\n", device);
        std::lock_guard<std::mutex> g(mu);
        fatal = HC_EHIP;
        cv_done.notify_all();
        return;
    }
    std::deque<Step *> flight;   // enqueued, results not taken yet (step order)
    std::vector<Step *> idle;
    for (Step &S : steps) idle.push_back(&S);
    std::vector<std::shared_ptr<Request>> uploads;
    Clock::time_point busy_since;
    for (;;) {
        bool stopping = false;
        {
            std::lock_guard<std::mutex> g(mu);
            stopping = stop;
        }
        if (stopping) break;
        // keep kSteps steps in flight while there is work
        if (!idle.empty()) {
            Step &S = *idle.back();
            if (build(S, uploads, flight.empty())) {
                const hc_status st = enqueue(S, uploads);
                if (flight.empty()) busy_since = Clock::now();
                idle.pop_back();
                if (st != HC_OK) {
                    // a failed enqueue leaves nothing of this step to wait for
                    (void)hipStreamSynchronize(stream);
                    finish(S, st);
                    idle.push_back(&S);
                } else {
                    flight.push_back(&S);
                }
                continue;
            }
            if (flight.empty()) continue;   // woken without work, or stopping
        }
        Step &S = *flight.front();
        flight.pop_front();
        finish(S, collect(S));
        idle.push_back(&S);
        if (flight.empty()) {
            std::lock_guard<std::mutex> g(mu);
            busy_s += std::chrono::duration<double>(Clock::now() - busy_since).count();
        }
    }
    (void)hipStreamSynchronize(stream);
    (void)hipStreamSynchronize(copy_stream);
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
    for (uint32_t i = S->slots; i-- > 0;) S->free_slots.push_back(int32_t(i));   // slot 0 first
    if (S->Fpool.ensure(size_t(S->slots) * S->table_bytes) != HC_OK ||
        S->xpool.ensure(size_t(S->slots) * kXStride + 64) != HC_OK ||
        S->patpool.ensure(size_t(S->slots) * sizeof(BPat)) != HC_OK)
        return HC_ENOMEM;
    if (hipMemset(S->xpool.p, 0, S->xpool.bytes) != hipSuccess ||
        hipMemset(S->patpool.p, 0, S->patpool.bytes) != hipSuccess)
        return HC_EHIP;
    for (Step &x : S->steps)
        if (hipEventCreateWithFlags(&x.counted, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&x.copied, hipEventDisableTiming) != hipSuccess)
            return HC_EHIP;
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking) != hipSuccess)
        return HC_EHIP;
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
