// Open-loop load generator for the serving loop (used by the benchmark):
// submitter threads call hc_serve_submit at each request's scheduled arrival
// time, and one collector thread takes completions (hc_serve_next_done,
// hc_serve_poll) as they happen, so that the offered rate does not depend on
// an interpreter. It only drives the public C ABI of libhc.
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hc.h"

namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0) {
    return std::chrono::duration<double>(Clock::now() - t0).count();
}

}  // namespace

extern "C" {

/*
 * Runs n requests against server s. Request i names text[i] and the pattern
 * pat[pat_off[i] .. pat_off[i+1]) and is submitted at arrival_s[i] seconds
 * after the start (ascending). Outputs, per request: submit_s[i] and done_s[i]
 * (seconds since the start, observed by the submitting and the collecting
 * thread), count[i] (occurrences), and, when keep[i] is nonzero, its
 * positions, appended to `pos` (capacity pos_cap) at pos_off[i] (pos_off has
 * n + 1 entries; -1 when they did not fit). Returns 0, or the first hc_status
 * that failed. timeout_s bounds the whole run.
 */
int hc_loadgen_run(hc_server *s, int64_t n, const double *arrival_s, const int32_t *text, const uint8_t *pat,
                   const int64_t *pat_off, const uint8_t *keep, int32_t threads, double timeout_s,
                   double *submit_s, double *done_s, int64_t *count, int64_t *pos, int64_t pos_cap,
                   int64_t *pos_off) {
    if (!s || n < 0 || threads < 1 || !arrival_s || !text || !pat || !pat_off || !submit_s || !done_s || !count)
        return HC_EINVAL;
    std::vector<uint64_t> ids(size_t(n), 0);
    std::vector<std::atomic<int>> submitted(static_cast<size_t>(n));
    for (auto &a : submitted) a.store(0);
    std::atomic<int> failed{0};
    std::atomic<int64_t> n_submitted{0};
    const Clock::time_point t0 = Clock::now();
    std::vector<std::thread> subs;
    for (int32_t t = 0; t < threads; ++t)
        subs.emplace_back([&, t] {
            for (int64_t i = t; i < n; i += threads) {
                while (seconds_since(t0) < arrival_s[i]) {
                    const double ahead = arrival_s[i] - seconds_since(t0);
                    if (ahead > 200e-6) std::this_thread::sleep_for(std::chrono::duration<double>(ahead - 150e-6));
                }
                uint64_t id = 0;
                const int st = hc_serve_submit(s, text[i], pat + pat_off[i], pat_off[i + 1] - pat_off[i], &id);
                submit_s[i] = seconds_since(t0);
                if (st != HC_OK) {
                    failed.store(st);
                    return;
                }
                ids[size_t(i)] = id;
                submitted[size_t(i)].store(1, std::memory_order_release);
                n_submitted.fetch_add(1);
            }
        });
    // collector: completions in the order they happen
    std::unordered_map<uint64_t, int64_t> index;   // id -> request
    int64_t scanned = 0, done = 0, used = 0;
    std::vector<int64_t> buf(1 << 16);
    int rc = HC_OK;
    if (pos_off)
        for (int64_t i = 0; i <= n; ++i) pos_off[i] = -1;
    while (done < n) {
        if (failed.load()) {
            rc = failed.load();
            break;
        }
        if (seconds_since(t0) > timeout_s) {
            rc = HC_EAGAIN;
            break;
        }
        uint64_t id = 0;
        int st = hc_serve_next_done(s, &id, 2000);
        if (st == HC_EAGAIN) continue;
        if (st != HC_OK) {
            rc = st;
            break;
        }
        const double t_done = seconds_since(t0);
        // ids become known once their submit returned
        auto it = index.find(id);
        while (it == index.end() && !failed.load()) {
            while (scanned < n && submitted[size_t(scanned)].load(std::memory_order_acquire)) {
                index[ids[size_t(scanned)]] = scanned;
                ++scanned;
            }
            it = index.find(id);
            if (it == index.end()) std::this_thread::yield();
        }
        if (it == index.end()) continue;   // a submit failed (reported above)
        const int64_t i = it->second;
        index.erase(it);
        int64_t c = 0;
        st = hc_serve_poll(s, id, buf.data(), int64_t(buf.size()), &c, 0);
        if (st == HC_EOVERFLOW) {
            buf.resize(size_t(c));
            st = hc_serve_poll(s, id, buf.data(), int64_t(buf.size()), &c, 0);
        }
        if (st != HC_OK) {
            rc = st;
            break;
        }
        done_s[i] = t_done;
        count[i] = c;
        if (keep && keep[i] && pos && pos_off && used + c <= pos_cap) {
            std::memcpy(pos + used, buf.data(), size_t(c) * 8);
            pos_off[i] = used;
            used += c;
        }
        ++done;
    }
    if (pos_off) pos_off[n] = used;
    for (auto &th : subs) th.join();
    if (rc == HC_OK && failed.load()) rc = failed.load();
    return rc;
}

}  // extern "C"
