// Preprocessing phase of HC (Section 3.1 and Section 3.2 of the paper), host.
//
// F has 2^alpha words of w bits. For every pair of adjacent, non-overlapping
// q-grams u1 = x[i..i+q-1], u2 = x[i+q..i+2q-1] (0 <= i <= m-2q), the word
// of u2 receives the link bit of u1: F[h(u2)] |= lambda(h(u1)) (eq. (1)).
// After all links, each q-gram that starts in the first q positions and
// whose word is still empty gets the word 1 (eq. (2) with the first
// optimisation of Section 3.4: marks go last, and only into empty words).
// H_v is the hash of the leftmost q-gram of the chain of q-grams that ends at
// position m-1 (second optimisation of Section 3.4).
//
// The paper walks the q-gram chains one after another so that each q-gram is
// hashed once. Here every q-gram hash is computed once into an array first
// and the links are read from it; OR is order-independent, so F is the same.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "hc_internal.h"

namespace hc {

int alpha_max(int w) {
    // 2^alpha * w / 8 <= 64 KiB
    int a = 0;
    while ((int64_t(1) << (a + 1)) * w / 8 <= kMaxTableBytes) ++a;
    return a;
}

hc_status validate_params(int64_t m, int q, int alpha, int w) {
    if (m < 1 || m > kMaxM) return HC_EINVAL;
    if (q < 1 || q > kMaxQ || q > m) return HC_EINVAL;
    if (w != 8 && w != 16 && w != 32 && w != 64) return HC_EINVAL;
    if (alpha < 1 || alpha > alpha_max(w)) return HC_EINVAL;
    return HC_OK;
}

namespace {
std::mutex g_tuned_mu;
Tuned g_tuned[kBuckets];
}  // namespace

int m_bucket(int64_t m) {
    int b = 0;
    while ((int64_t(1) << b) < m && b < kBuckets - 1) ++b;
    return b;
}

void set_tuned(int64_t m, const Tuned &t) {
    std::lock_guard<std::mutex> g(g_tuned_mu);
    g_tuned[m_bucket(m)] = t;
}

Tuned get_tuned(int64_t m) {
    std::lock_guard<std::mutex> g(g_tuned_mu);
    return g_tuned[m_bucket(m)];
}

// Built-in priors when the caller leaves a parameter at 0, keyed by the
// pattern length and the number of distinct bytes of x (a stand-in for the
// alphabet of the text). Section 4 reports best variants with q between 3 and
// 8 and alpha 11-12; on gfx950 the fastest choices measured on iid texts over
// 4 to 64 symbols were: for m <= 8 the smallest q with m < 2q (no links:
// the dense schedule tests every window at once, by one hash, or for
// windows of 4 to 8 bytes by comparing them with x directly), longer q-grams
// for small alphabets above that,
// smaller tables (alpha 11, 16-bit words: more workgroups fit in LDS) for m
// up to 128. An entry measured by hc_autotune for the pattern's length bucket
// takes precedence.
void default_params(int64_t m, int distinct, int &q, int &alpha, int &w) {
    const bool small_sigma = distinct <= 4;
    int pq, pa, pw;
    if (m <= 2) { pq = int(m); pa = 8; pw = 8; }
    else if (m <= 8) { pq = int((m + 2) / 2); pa = 10; pw = 16; }
    else if (m <= 16) { pq = small_sigma ? 5 : 4; pa = 12; pw = 32; }
    else if (m <= 128) { pq = 5; pa = 11; pw = 16; }
    else if (m <= 256) { pq = 5; pa = 12; pw = 32; }
    else { pq = 6; pa = 12; pw = 32; }
    const Tuned t = get_tuned(m);
    if (t.set) {   // a tuned entry for this length bucket takes precedence
        pq = t.q;
        pa = t.alpha;
        pw = t.w;
    }
    if (q == 0) q = int(std::min<int64_t>(pq, m));
    if (w == 0) w = pw;
    if (alpha == 0) alpha = std::min(pa, alpha_max(w));
}

int distinct_bytes(const uint8_t *x, int64_t m) {
    bool seen[256] = {false};
    int d = 0;
    for (int64_t i = 0; i < m; ++i)
        if (!seen[x[i]]) {
            seen[x[i]] = true;
            ++d;
        }
    return d;
}

static inline uint32_t qgram_hash(const uint8_t *u, int q, int s, uint32_t mask) {
    // equation (3): the k-th character of the q-gram carries weight 2^(s*k);
    // uint32 arithmetic wraps mod 2^32, which 2^alpha divides
    uint32_t v = 0;
    for (int k = q - 1; k >= 0; --k) v = (v << s) + u[k];
    return v & mask;
}

void build_link_table(const uint8_t *x, int64_t m, int q, int alpha, int w,
                      PatternData &out) {
    out.x.assign(x, x + m);
    out.m = m;
    out.q = q;
    out.alpha = alpha;
    out.w = w;
    out.s = alpha / q;                                  // eq. (4)
    out.mask = uint32_t((uint64_t(1) << alpha) - 1);    // F' = 2^alpha - 1
    out.F.assign(size_t(1) << alpha, 0);

    const int64_t grams = m - q + 1;
    std::vector<uint32_t> h(grams);
    for (int64_t i = 0; i < grams; ++i) h[i] = qgram_hash(x + i, q, out.s, out.mask);

    const uint32_t wmask = uint32_t(w - 1);
    for (int64_t i = 0; i + 2 * q <= m; ++i)            // eq. (1)
        out.F[h[i + q]] |= uint64_t(1) << (h[i] & wmask);
    for (int64_t i = 0; i < std::min<int64_t>(q, grams); ++i)   // eq. (2), empty words only
        if (out.F[h[i]] == 0) out.F[h[i]] = 1;

    out.hv = h[(m - q) % q];   // leftmost q-gram of the chain ending at m-1
}

std::vector<uint8_t> pack_table(const PatternData &p) {
    const size_t words = p.F.size(), bytes = size_t(p.w / 8);
    std::vector<uint8_t> out(words * bytes);
    for (size_t i = 0; i < words; ++i) {
        uint64_t v = p.F[i];
        std::memcpy(out.data() + i * bytes, &v, bytes);   // little-endian low bytes
    }
    return out;
}

}  // namespace hc
