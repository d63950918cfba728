/*
 * Input generator for the synthetic English stand-in: an order-2 Markov walk.
 * Not part of the searching path; it only draws text.
 *
 * cum:   k*k rows of k cumulative probabilities, row index = prev2 * k + prev1
 * state: {prev2, prev1}, updated in place so a walk can be continued in chunks
 * u:     n uniforms in [0, 1)
 * out:   n symbol indices; symbol = first index whose cumulative probability
 *        exceeds u, or k - 1 when rounding leaves none
 */
#include <stdint.h>

void markov2_walk(const double *cum, int k, int32_t *state, const double *u,
                  uint8_t *out, int64_t n)
{
    int32_t a = state[0], b = state[1];
    for (int64_t i = 0; i < n; ++i) {
        const double *row = cum + ((int64_t)a * k + b) * k;
        int c = 0;
        while (c < k - 1 && !(row[c] > u[i]))
            ++c;
        out[i] = (uint8_t)c;
        a = b;
        b = c;
    }
    state[0] = a;
    state[1] = b;
}
