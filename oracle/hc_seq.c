/*
 * The searching phase of HC run sequentially over a whole text, counting
 * which bytes of the text it reads.
 *
 * TEST INFRASTRUCTURE. Only the test-suite and the script that writes the
 * method-bytes table under profiles/ (oracle/method_bytes.py) use it. It
 * shares no code with the HIP path.
 *
 * What it computes, from the paper's definitions:
 *   - the shift s = floor(alpha / q) (eq. (4)) and the hash of a q-gram,
 *     eq. (3): the bytes read from the q-gram's last position backwards,
 *     each step v = v * 2^s + byte, reduced modulo 2^alpha;
 *   - the link hash lambda(v) = 2^(v mod w) (eq. (5));
 *   - the word vector F: for every pair of adjacent non-overlapping q-grams
 *     u1 u2 of x, the word of h(u2) gets the bit lambda(h(u1)) (eq. (1));
 *     then each q-gram that starts in the first min(q, m - q + 1) positions
 *     sets its word to 1 if that word is still empty (eq. (2) and the first
 *     optimisation of Section 3.4);
 *   - H_v: the hash of the leftmost q-gram of the chain that ends at m - 1
 *     (second optimisation of Section 3.4);
 *   - the search of Section 3.3: the q-gram at the window end is hashed; an
 *     empty word shifts the window end by m - q + 1; otherwise the q-grams q,
 *     2q, ... positions back are hashed while a whole one fits in the window,
 *     each checked against the link bits of the word of the q-gram after it;
 *     a missing link moves the window end to (end of that q-gram) + m - q + 1;
 *     a window whose q-grams all link is a candidate: if the last hash equals
 *     H_v it is compared with x at its own start (the reading of the output
 *     step recorded in the design notes) and the window end moves on by one.
 *
 * It reports the number of occurrences and the number of distinct
 * `line`-byte blocks of y (aligned to the text's start) that the search reads:
 * the bytes of every hashed q-gram and of every compared window. Those are
 * the text bytes the method needs, at the granularity of a memory line.
 * With max_hashes > 0 the scan stops once it has hashed that many q-grams;
 * *covered then tells how far it got (every window ending before that
 * position was decided), else *covered = n.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint32_t hash_ending_at(const unsigned char *s, int64_t e, int q, int sh, uint32_t mask)
{
    uint32_t v = 0;
    for (int k = 0; k < q; ++k) v = ((v << sh) + s[e - k]) & mask;
    return v;
}

/* marks the lines holding y[a..b] (inclusive); returns how many were new */
static int64_t touch(uint8_t *seen, int64_t a, int64_t b, int64_t line)
{
    int64_t added = 0;
    for (int64_t l = a / line; l <= b / line; ++l)
        if (!seen[l]) {
            seen[l] = 1;
            ++added;
        }
    return added;
}

/*
 * Returns 0 on success, -1 on bad arguments or allocation failure.
 * *occ = occurrences reported, *lines = distinct lines read.
 */
int oracle_hc_scan(const unsigned char *x, int64_t m, const unsigned char *y, int64_t n, int q, int alpha,
                   int w, int64_t line, int64_t max_hashes, int64_t *occ, int64_t *lines, int64_t *covered)
{
    if (!x || m < 1 || q < 1 || q > m || alpha < 1 || alpha > 24 || w < 1 || w > 64 || line < 1 || !occ ||
        !lines || !covered || n < 0 || (n > 0 && !y))
        return -1;
    const int sh = alpha / q;
    const uint32_t mask = (uint32_t)((1ull << alpha) - 1);
    uint64_t *F = (uint64_t *)calloc((size_t)1 << alpha, sizeof(uint64_t));
    uint8_t *seen = (uint8_t *)calloc((size_t)(n / line + 2), 1);
    if (!F || !seen) {
        free(F);
        free(seen);
        return -1;
    }
    /* links of eq. (1): u1 = x[i..i+q-1], u2 = x[i+q..i+2q-1] */
    for (int64_t i = 0; i + 2 * q <= m; ++i) {
        const uint32_t h1 = hash_ending_at(x, i + q - 1, q, sh, mask);
        const uint32_t h2 = hash_ending_at(x, i + 2 * q - 1, q, sh, mask);
        F[h2] |= 1ull << (h1 % (uint32_t)w);
    }
    /* marks of eq. (2), only into words still empty */
    const int64_t first = q < m - q + 1 ? q : m - q + 1;
    for (int64_t i = 0; i < first; ++i) {
        const uint32_t h = hash_ending_at(x, i + q - 1, q, sh, mask);
        if (F[h] == 0) F[h] = 1;
    }
    /* H_v: leftmost q-gram of the chain ending at m - 1 */
    int64_t head_end = m - 1;
    while (head_end - q >= q - 1) head_end -= q;
    const uint32_t hv = hash_ending_at(x, head_end, q, sh, mask);

    int64_t count = 0, nl = 0, hashes = 0;
    int64_t J = m - 1;
    *covered = n;
    while (J < n) {
        if (max_hashes > 0 && hashes >= max_hashes) {
            *covered = J;
            break;
        }
        ++hashes;
        nl += touch(seen, J - q + 1, J, line);
        uint32_t v = hash_ending_at(y, J, q, sh, mask);
        uint64_t z = F[v];
        if (z == 0) {
            J += m - q + 1;
            continue;
        }
        int64_t e = J;
        int linked = 1;
        while (e - q >= J - m + q) {
            e -= q;
            ++hashes;
            nl += touch(seen, e - q + 1, e, line);
            v = hash_ending_at(y, e, q, sh, mask);
            if ((z & (1ull << (v % (uint32_t)w))) == 0) {
                linked = 0;
                break;
            }
            z = F[v];
        }
        if (linked) {
            const int64_t start = J - m + 1;
            if (v == hv) {
                nl += touch(seen, start, J, line);
                if (memcmp(y + start, x, (size_t)m) == 0) ++count;
            }
            J += 1;
        } else {
            J = e + m - q + 1;
        }
    }
    free(F);
    free(seen);
    *occ = count;
    *lines = nl;
    return 0;
}
