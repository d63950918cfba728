// Preprocessing phase of HC on the device, for many patterns at once
// (Section 3.1, eqs. (1)-(2); Section 3.4, first and second optimisations).
//
// One workgroup per pattern builds its word vector F in LDS:
//  1. links: every adjacent non-overlapping pair of q-grams (u1 at i, u2 at
//     i + q, 0 <= i <= m - 2q) ORs the link bit of h(u1) into the word of
//     h(u2) with an LDS atomic OR; OR is order-independent, so any number of
//     threads give the word the paper's sequential loop gives;
//  2. a workgroup barrier: every link is in place;
//  3. marks: each q-gram that starts in the first q positions gets the value
//     1 in its word if the word is still empty. Marks only ever write 1 into
//     words that are 0 after step 1, so their order does not matter either.
// The table is then copied out. H_v (the hash of the q-gram at (m - q) mod
// q), s and the mask come from the same hash definition (eqs. (3)-(4)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "hc_batch.h"
#include "hc_device.h"
#include "hc_internal.h"
#include "hc_runtime.h"

namespace hc {

struct PrepArgs {
    const uint8_t *x;          // all patterns' bytes
    const uint32_t *desc;      // per pattern: offset of x, m, q
    uint32_t n, alpha, w;
    uint32_t table_bytes;      // stride of the output tables (>= 2^alpha * w / 8, 16-aligned)
    uint8_t *F;                // n tables
    uint32_t *info;            // per pattern: s, mask, H_v (may be null)
};

// eq. (3): byte k of the q-gram weighs 2^(s*k), reduced mod 2^alpha
__device__ __forceinline__ uint32_t prep_hash(const uint8_t *u, int q, uint32_t s, uint32_t mask) {
    uint32_t v = 0;
    for (int k = q - 1; k >= 0; --k) v = (v << s) + u[k];
    return v & mask;
}

// OR `bits` into the w-bit word `v` of a table held in 32-bit LDS words
// (w = 64 uses 64-bit words).
__device__ __forceinline__ void word_or(uint32_t *T, uint32_t w, uint32_t v, uint64_t bits) {
    if (w == 64) {
        atomicOr(reinterpret_cast<unsigned long long *>(T) + v, (unsigned long long)bits);
    } else {
        const uint32_t bit = v * w;   // first bit of the word
        atomicOr(&T[bit >> 5], uint32_t(bits) << (bit & 31u));
    }
}

__device__ __forceinline__ bool word_empty(const uint32_t *T, uint32_t w, uint32_t v) {
    if (w == 64) return reinterpret_cast<const unsigned long long *>(T)[v] == 0ull;
    const uint32_t bit = v * w;
    const uint32_t field = T[bit >> 5] >> (bit & 31u);
    return w == 32 ? field == 0u : (field & ((1u << w) - 1u)) == 0u;
}

__global__ __launch_bounds__(256) void hc_preprocess_kernel(PrepArgs A) {
    extern __shared__ __align__(16) uint32_t T[];
    const uint32_t p = blockIdx.x;
    if (p >= A.n) return;
    const uint8_t *x = A.x + A.desc[3 * p];
    const int64_t m = A.desc[3 * p + 1];
    const int q = int(A.desc[3 * p + 2]);
    const uint32_t s = A.alpha / uint32_t(q);                           // eq. (4)
    const uint32_t mask = uint32_t((uint64_t(1) << A.alpha) - 1u);
    const uint32_t words32 = A.table_bytes / 4u;
    for (uint32_t i = threadIdx.x; i < words32; i += blockDim.x) T[i] = 0u;
    __syncthreads();
    // eq. (1): links between adjacent non-overlapping q-grams
    for (int64_t i = threadIdx.x; i + 2 * q <= m; i += blockDim.x) {
        const uint32_t h1 = prep_hash(x + i, q, s, mask), h2 = prep_hash(x + i + q, q, s, mask);
        word_or(T, A.w, h2, uint64_t(1) << (h1 & (A.w - 1u)));
    }
    __syncthreads();
    // eq. (2) with the first optimisation: marks into words still empty
    const int64_t first = m - q + 1 < q ? m - q + 1 : q;
    for (int64_t i = threadIdx.x; i < first; i += blockDim.x) {
        const uint32_t h = prep_hash(x + i, q, s, mask);
        if (word_empty(T, A.w, h)) word_or(T, A.w, h, 1u);
    }
    __syncthreads();
    uint32_t *out = reinterpret_cast<uint32_t *>(A.F + uint64_t(p) * A.table_bytes);
    for (uint32_t i = threadIdx.x; i < words32; i += blockDim.x) out[i] = T[i];
    if (threadIdx.x == 0 && A.info) {
        A.info[3 * p + 0] = s;
        A.info[3 * p + 1] = mask;
        A.info[3 * p + 2] = prep_hash(x + (m - q) % q, q, s, mask);   // H_v
    }
}

hc_status device_preprocess(const uint8_t *d_x, const uint32_t *d_desc, uint32_t n, int alpha, int w,
                            uint32_t table_bytes, uint8_t *d_F, uint32_t *d_info, hipStream_t s) {
    if (n == 0) return HC_OK;
    if (table_bytes % 16u || table_bytes < (uint64_t(1) << alpha) * uint64_t(w) / 8u) return HC_EINVAL;
    if (table_bytes > device_info().max_lds_per_block) return HC_EINVAL;
    PrepArgs A{d_x, d_desc, n, uint32_t(alpha), uint32_t(w), table_bytes, d_F, d_info};
    hipLaunchKernelGGL(hc_preprocess_kernel, dim3(n), dim3(256), table_bytes, s, A);
    return hipGetLastError() == hipSuccess ? HC_OK : HC_EHIP;
}

}  // namespace hc

using namespace hc;

extern "C" hc_status hc_preprocess_many(const uint8_t *pat, const int64_t *pat_off, int32_t n,
                                        const hc_params *params, void *d_F, int64_t table_stride,
                                        hc_params *used, uint32_t *info, void *stream) {
    if (n < 0 || (n > 0 && (!pat || !pat_off || !d_F))) return HC_EINVAL;
    if (n == 0) return HC_OK;
    int alpha = params ? params->alpha : 0, w = params ? params->w : 0;
    const int q_req = params ? params->q : 0;
    if (alpha < 0 || w < 0 || q_req < 0) return HC_EINVAL;
    if (w == 0) w = 32;
    if (alpha == 0) alpha = std::min(12, alpha_max(w));
    std::vector<uint32_t> desc(size_t(n) * 3);
    for (int32_t i = 0; i < n; ++i) {
        const int64_t m = pat_off[i + 1] - pat_off[i];
        if (m < 1 || m > kMaxM) return HC_EINVAL;
        int q = q_req, a = alpha, ww = w;
        default_params(m, distinct_bytes(pat + pat_off[i], m), q, a, ww);
        q = int(std::min<int64_t>(q, m));
        if (validate_params(m, q, alpha, w) != HC_OK) return HC_EINVAL;
        desc[3 * i] = uint32_t(pat_off[i] - pat_off[0]);
        desc[3 * i + 1] = uint32_t(m);
        desc[3 * i + 2] = uint32_t(q);
        if (used) used[i] = hc_params{q, alpha, w};
    }
    const uint64_t need = (uint64_t(1) << alpha) * uint64_t(w) / 8u;
    if (table_stride < int64_t(std::max<uint64_t>(16, (need + 15u) & ~uint64_t(15))) || table_stride % 16)
        return HC_EINVAL;
    if (!device_info().ok) return HC_EHIP;
    hipStream_t s = hipStream_t(stream);
    const size_t xb = size_t(pat_off[n] - pat_off[0]);
    if (xb > 0xFFFFFFFFull) return HC_EINVAL;
    uint8_t *d_x = nullptr;
    uint32_t *d_desc = nullptr, *d_info = nullptr;
    hc_status st = HC_OK;
    if (hipMalloc(&d_x, std::max<size_t>(xb, 1)) != hipSuccess ||
        hipMalloc(&d_desc, desc.size() * 4) != hipSuccess || hipMalloc(&d_info, size_t(n) * 12) != hipSuccess)
        st = HC_ENOMEM;
    if (st == HC_OK &&
        (hipMemcpyAsync(d_x, pat + pat_off[0], xb, hipMemcpyHostToDevice, s) != hipSuccess ||
         hipMemcpyAsync(d_desc, desc.data(), desc.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess))
        st = HC_EHIP;
    if (st == HC_OK)
        st = device_preprocess(d_x, d_desc, uint32_t(n), alpha, w, uint32_t(table_stride),
                               static_cast<uint8_t *>(d_F), d_info, s);
    if (st == HC_OK && info &&
        hipMemcpyAsync(info, d_info, size_t(n) * 12, hipMemcpyDeviceToHost, s) != hipSuccess)
        st = HC_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess && st == HC_OK) st = HC_EHIP;
    (void)hipFree(d_x);
    (void)hipFree(d_desc);
    (void)hipFree(d_info);
    return st;
}
