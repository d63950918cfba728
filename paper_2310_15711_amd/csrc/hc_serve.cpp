// Serving loop (placeholder until the continuous-batching scheduler lands).
#include "hc_internal.h"

extern "C" {
hc_status hc_serve_create(const uint8_t *const *, const int64_t *, int32_t, int64_t,
                          const hc_params *, hc_server **out) {
    if (out) *out = nullptr;
    return HC_EINVAL;
}
hc_status hc_serve_submit(hc_server *, int32_t, const uint8_t *, int64_t, uint64_t *) { return HC_EINVAL; }
hc_status hc_serve_poll(hc_server *, uint64_t, int64_t *, int64_t, int64_t *, int32_t) { return HC_EINVAL; }
hc_status hc_serve_stats(hc_server *, double *, double *, double *, int64_t *) { return HC_EINVAL; }
hc_status hc_serve_destroy(hc_server *) { return HC_EINVAL; }
}
