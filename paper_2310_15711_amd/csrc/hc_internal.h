// Internal declarations shared by the host runtime and the HIP kernels of
// libhc. Not part of the public ABI (include/hc.h).
#pragma once

#include <cstdint>
#include <deque>
#include <mutex>
#include <vector>

#include "hc.h"

namespace hc {

constexpr int kMaxQ = 8;          // the paper explores q <= 8 (Section 4)
constexpr int64_t kMaxM = 4096;   // pattern bytes staged on chip
constexpr int kBlock = 256;       // threads per workgroup (4 wavefronts)
constexpr int64_t kMaxTableBytes = 64 * 1024;

// Host-side result of the preprocessing phase plus lazily uploaded device
// copies (per device).
struct DeviceCopy {
    int device = -1;
    void *d_F = nullptr;      // 2^alpha words of w bits, packed
    uint8_t *d_x = nullptr;   // m bytes (padded to 16)
};

struct PatternData {
    std::vector<uint8_t> x;
    int64_t m = 0;
    int32_t q = 0, alpha = 0, w = 0, s = 0;
    uint32_t mask = 0, hv = 0;
    std::vector<uint64_t> F;  // 2^alpha words, low w bits used
};

// Parameters and launch shape chosen by hc_autotune for one pattern-length
// bucket (lengths in (2^(b-1), 2^b]); process-wide, last tuning wins.
struct Tuned {
    bool set = false;
    int q = 0, alpha = 0, w = 0, schedule = 0, segment = 0, variant = 0;
};
constexpr int kBuckets = 13;   // m up to 4096
int m_bucket(int64_t m);
void set_tuned(int64_t m, const Tuned &t);
Tuned get_tuned(int64_t m);

int alpha_max(int w);
hc_status validate_params(int64_t m, int q, int alpha, int w);
void default_params(int64_t m, int distinct, int &q, int &alpha, int &w);
int distinct_bytes(const uint8_t *x, int64_t m);

// Builds F, s, mask and H_v (host).
void build_link_table(const uint8_t *x, int64_t m, int q, int alpha, int w,
                      PatternData &out);

// Packs the low w bits of each word of F into a byte array of w/8 bytes per word.
std::vector<uint8_t> pack_table(const PatternData &p);

}  // namespace hc

struct hc_pattern {
    hc::PatternData data;
    std::mutex mu;
    std::deque<hc::DeviceCopy> dev;   // stable addresses
};
