"""Pins for the oracle (CPU only).

The oracle is checked against things other than itself: occurrence lists
derived by hand (tests/golden/hand_cases.txt), a library routine
(bytes.find), closed forms, planted copies, the chain listing printed in
the paper's worked example, hand-computed hash values, hand-derived word
vectors, a special case where F reduces to the q-gram adjacency relation,
and exhaustive agreement of the sequential searching phase with brute force.
"""
import itertools
import random

import numpy as np
import pytest

from conftest import golden_lines
from oracle import hc_oracle as O
from paper_2310_15711_amd import workloads as W


def find_all(x: bytes, y: bytes):
    """Library routine: bytes.find restarted one past each hit."""
    out, i = [], y.find(x)
    while i != -1:
        out.append(i)
        i = y.find(x, i + 1)
    return out


# ---------------------------------------------------------------- brute force

def test_hand_cases():
    rows = golden_lines("hand_cases.txt")
    assert len(rows) >= 10
    for xh, yh, occ in rows:
        x, y = bytes.fromhex(xh), bytes.fromhex(yh)
        want = [] if occ == "-" else [int(t) for t in occ.split(",")]
        assert O.occurrences_py(x, y) == want, (xh, yh)
        assert O.occurrences(x, y).tolist() == want, (xh, yh)
        assert find_all(x, y) == want


@pytest.mark.parametrize("sigma", [2, 4, 20, 256])
def test_brute_vs_library_find(sigma):
    g = random.Random(1000 + sigma)
    for _ in range(300):
        n = g.randint(0, 300)
        m = g.randint(1, 12)
        alpha = [g.randrange(256) for _ in range(sigma)] if sigma < 256 else list(range(256))
        y = bytes(g.choice(alpha) for _ in range(n))
        if n >= m and g.random() < 0.5:
            t = g.randint(0, n - m)
            x = y[t:t + m]
        else:
            x = bytes(g.choice(alpha) for _ in range(m))
        want = find_all(x, y)
        assert O.occurrences_py(x, y) == want
        for th in (1, 3, 8):
            assert O.occurrences(x, y, threads=th).tolist() == want


def test_brute_thread_partition_boundaries():
    # occurrences that straddle every possible block boundary
    y = b"ab" * 50
    for th in range(1, 12):
        got = O.occurrences(b"abab", y, threads=th).tolist()
        assert got == list(range(0, 97, 2))
    assert O.occurrences(b"a", b"", threads=4).tolist() == []
    assert O.count(b"aa", b"a" * 10) == 9


def test_closed_forms():
    for n in (1, 5, 64, 1000):
        for m in (1, 2, 7, 64):
            got = O.occurrences(b"a" * m, b"a" * n).tolist()
            assert got == list(range(0, n - m + 1)), (n, m)
    for N in (1, 3, 50):
        for k in (1, 2, 5):
            got = O.occurrences(b"ab" * k, b"ab" * N).tolist()
            assert got == list(range(0, 2 * (N - k) + 1, 2))


def de_bruijn_binary(k):
    """Linearised binary de Bruijn sequence B(2, k) (Fredricksen-Kessler-Maiorana:
    concatenate the Lyndon words whose length divides k, in lexicographic
    order, then append the first k-1 symbols)."""
    a = [0] * (k + 1)
    seq = []

    def db(t, p):
        if t > k:
            if k % p == 0:
                seq.extend(a[1:p + 1])
        else:
            a[t] = a[t - p]
            db(t + 1, p)
            for j in range(a[t - p] + 1, 2):
                a[t] = j
                db(t + 1, t)

    db(1, 1)
    return seq + seq[:k - 1]


@pytest.mark.parametrize("k", [3, 6, 10])
def test_de_bruijn_each_word_once(k):
    s = de_bruijn_binary(k)
    assert len(s) == 2 ** k + k - 1
    y = bytes(s)
    for word in range(2 ** k):
        x = bytes((word >> (k - 1 - i)) & 1 for i in range(k))
        assert len(O.occurrences(x, y)) == 1


def test_planted_copies_found():
    p = W.planted_config(n=1 << 18, m=32, extra=40)
    got = O.occurrences(p.x, p.y)
    assert set(p.plants + [p.source]) <= set(got.tolist())
    assert np.all(np.diff(got) > 0)
    # every reported start really matches, by a different route
    yb = p.y.tobytes()
    assert all(yb[t:t + 32] == p.x for t in got.tolist())
    assert O.matches_at(p.x, p.y, p.plants[0])
    assert not O.matches_at(p.x, p.y, int(p.y.size))


def test_brute_rejects_empty_pattern():
    with pytest.raises(ValueError):
        O.occurrences(b"", b"abc")


# ------------------------------------------------------------ hash functions

def test_hash_golden_values():
    rows = golden_lines("hash_values.txt")
    hs = [r for r in rows if r[0] == "h"]
    ls = [r for r in rows if r[0] == "lambda"]
    assert len(hs) >= 6 and len(ls) >= 3
    for _, uh, alpha, s_want, h_want in hs:
        u = bytes.fromhex(uh)
        s = O.shift_s(int(alpha), len(u))
        assert s == int(s_want)
        assert O.qgram_hash(u, int(alpha), s) == int(h_want), uh
    for _, v, w, want in ls:
        assert O.link_bit(int(v), int(w)) == int(want)


# ------------------------------------------------------------ word vector F

def test_chains_of_worked_example():
    rows = golden_lines("paper_chains.txt")
    x = rows[0][1].encode()
    q = int(rows[1][1])
    want = {int(r[0]): r[1:] for r in rows[2:]}
    pairs = O.adjacent_pairs(len(x), q)
    nxt = dict(pairs)
    heads = sorted(set(range(len(x) - q + 1)) - set(nxt.values()))
    chains = {}
    for h in heads:
        c, i = [], h
        while True:
            c.append(x[i:i + q].decode())
            if i not in nxt:
                break
            i = nxt[i]
        chains[h] = c
    assert chains == want


@pytest.mark.parametrize("m,q", [(13, 3), (16, 4), (5, 4), (4, 4), (6, 4), (7, 4), (30, 8)])
def test_chain_count(m, q):
    # Section 3.1: m-q+1 chains when m < 2q-1, q chains otherwise
    pairs = O.adjacent_pairs(m, q)
    starts = set(range(m - q + 1))
    heads = starts - {b for _, b in pairs}
    want = m - q + 1 if m < 2 * q - 1 else q
    assert len(heads) == want
    assert len(O.first_qgram_starts(m, q)) == want


def test_chain_head_of_fig1():
    # Fig. 1 (m=13, q=3): hashes are numbered in computation order; the paper
    # names H_11 -- the last of the m-q+1 = 11 chain hashes, i.e. the leftmost
    # q-gram of the chain ending at position 12 (ends 12, 9, 6, 3) -- as H_v.
    assert O.chain_end_qgram_starts(13, 3) == [10, 7, 4, 1]
    x = b"abcdefghijklm"
    assert O.chain_head_hash(x, 3, 8) == O.qgram_hash(x[1:4], 8, O.shift_s(8, 3))


def test_link_table_golden_cases():
    rows = [r for r in golden_lines("link_table_cases.txt") if r[0] == "table"]
    assert len(rows) >= 4
    for r in rows:
        x = bytes.fromhex(r[1])
        q, alpha, w, hv = (int(v) for v in r[2:6])
        want = {int(k): int(v) for k, v in (e.split(":") for e in r[6:])}
        F, s, mask, Hv = O.link_table(x, q, alpha, w)
        assert mask == (1 << alpha) - 1 and s == alpha // q
        assert Hv == hv
        got = {i: v for i, v in enumerate(F) if v}
        assert got == want, r[1]


@pytest.mark.parametrize("q", [1, 2])
def test_link_table_is_adjacency_when_hashes_are_injective(q):
    # alpha = 6, w = 64, bytes < 2^s: h is the base-2^s value of the q-gram
    # (no reduction happens) and lambda(v) = 2^v, so F[h(u2)] has exactly the
    # bits of the q-grams u1 that precede u2 in x, plus bit 0 for an empty
    # first-q word. Codes start at 1 so bit 0 cannot come from a link.
    alpha, w = 6, 64
    s = alpha // q
    g = random.Random(7 + q)
    for _ in range(200):
        m = g.randint(q, 24)
        x = bytes(g.randint(1, (1 << s) - 1) for _ in range(m))
        code = lambda u: sum(c << (s * k) for k, c in enumerate(u))
        want = {}
        for i in range(0, m - 2 * q + 1):
            want[code(x[i + q:i + 2 * q])] = want.get(code(x[i + q:i + 2 * q]), 0) | (1 << code(x[i:i + q]))
        for i in range(min(q, m - q + 1)):
            c = code(x[i:i + q])
            if want.get(c, 0) == 0:
                want[c] = 1
        F, _, _, _ = O.link_table(x, q, alpha, w)
        assert {i: v for i, v in enumerate(F) if v} == want


def test_link_table_invariants():
    g = random.Random(11)
    for _ in range(300):
        m = g.randint(1, 40)
        q = g.randint(1, min(m, 8))
        alpha = g.randint(1, 12)
        w = g.choice([1, 2, 8, 16, 32, 64])
        x = bytes(g.randrange(256) for _ in range(m))
        F, s, mask, Hv = O.link_table(x, q, alpha, w)
        hs = {O.qgram_hash(x[i:i + q], alpha, s) for i in range(m - q + 1)}
        nz = {i for i, v in enumerate(F) if v}
        assert nz <= hs                     # only q-gram words are touched
        assert all(F[h] for h in hs)        # every q-gram of x is recognised
        for i1, i2 in O.adjacent_pairs(m, q):   # every adjacent pair is linked
            h1 = O.qgram_hash(x[i1:i1 + q], alpha, s)
            h2 = O.qgram_hash(x[i2:i2 + q], alpha, s)
            assert F[h2] & O.link_bit(h1, w)
        assert all(v < (1 << w) for v in F)
        head = (m - q) % q
        assert Hv == O.qgram_hash(x[head:head + q], alpha, s)


# ------------------------------------------------ sequential searching phase

ENCODINGS = [(0, 1), (ord("a"), ord("b")), (0xFE, 0xFF)]


@pytest.mark.parametrize("enc", ENCODINGS)
def test_sequential_hc_exhaustive_binary(enc):
    # every text of length <= 8 and every pattern of length <= 4 over a
    # two-letter alphabet, for every q <= m and parameter sets that force
    # hash collisions (alpha 1, 2) and that do not (alpha 8)
    texts = [bytes(enc[b] for b in bits)
             for n in range(0, 9) for bits in itertools.product((0, 1), repeat=n)]
    for m in range(1, 5):
        for bits in itertools.product((0, 1), repeat=m):
            x = bytes(enc[b] for b in bits)
            for q in range(1, m + 1):
                for alpha, w in ((1, 8), (2, 1), (8, 32)):
                    table = O.link_table(x, q, alpha, w)
                    for y in texts:
                        got = O.hc_search_sequential(x, y, q, alpha, w, table)
                        assert got == find_all(x, y), (x, y, q, alpha, w)


def test_sequential_hc_random():
    g = random.Random(5)
    for _ in range(1500):
        sigma = g.choice([2, 4, 20, 256])
        n = g.randint(0, 400)
        m = g.randint(1, 24)
        y = bytes(g.randrange(sigma) * (1 if sigma == 256 else 7) % 256 for _ in range(n))
        if n >= m and g.random() < 0.7:
            t = g.randint(0, n - m)
            x = y[t:t + m]
        else:
            x = bytes(g.randrange(sigma) * (1 if sigma == 256 else 7) % 256 for _ in range(m))
        q = g.randint(1, min(m, 8))
        alpha = g.randint(1, 12)
        w = g.choice([8, 16, 32, 64])
        assert O.hc_search_sequential(x, y, q, alpha, w) == find_all(x, y)


def _chain_order_table(x, q, alpha, w):
    """F and H_v built in the order of the preprocessing figure of Section
    3.2: chain by chain (the chain ending at m - i for i = min(m - q + 1, q)
    down to 1), each walked from its last q-gram backwards, linking every
    q-gram's word to the q-gram before it; H_v is the last hash the walks
    compute; then the q-grams ending at q - 1 .. min(2q - 1, m) - 1 are marked
    with 1 where their word is still empty. Hashes are read backwards from a
    q-gram's end and reduced at every step (independent of the oracle's
    start-to-end form reduced once)."""
    m = len(x)
    s, mask = alpha // q, (1 << alpha) - 1

    def hash_ending_at(e):
        v = 0
        for k in range(q):
            v = ((v << s) + x[e - k]) & mask
        return v

    F = [0] * (1 << alpha)
    hv = None
    for i in range(min(m - q + 1, q), 0, -1):
        right = hash_ending_at(m - i)
        e = m - i - q
        while e >= q - 1:
            left = hash_ending_at(e)
            F[right] |= 1 << (left & (w - 1))
            right = left
            e -= q
        hv = right
    for e in range(q - 1, min(2 * q - 1, m)):
        v = hash_ending_at(e)
        if F[v] == 0:
            F[v] = 1
    return F, hv


def test_link_table_equals_chain_order():
    """The oracle's F (equation (1) over the pairs in index order, then the
    marks) and H_v equal the chain-order construction, on random patterns
    over small and large alphabets (repeated q-grams, bytes >= 0x80), every
    q up to min(m, 8), tiny and usual alpha, every w."""
    g = np.random.default_rng(3101)
    for case in range(400):
        m = int(g.integers(1, 70))
        sigma = int(g.choice([2, 3, 4, 256]))
        x = bytes((g.integers(0, sigma, size=m) * (255 // max(sigma - 1, 1))).astype(np.uint8))
        q = int(g.integers(1, min(m, 8) + 1))
        alpha = int(g.choice([1, 3, 8, 12]))
        w = int(g.choice([8, 16, 32, 64]))
        F, s, mask, hv = O.link_table(x, q, alpha, w)
        F2, hv2 = _chain_order_table(x, q, alpha, w)
        assert F == F2, (case, x.hex(), q, alpha, w)
        assert hv == hv2, (case, x.hex(), q, alpha, w)


def test_hc_scan_finds_the_brute_force_occurrences():
    """The C sequential searching phase reports exactly as many occurrences
    as the brute force, over random texts with planted copies, every q, tiny
    and usual alpha, every w."""
    g = np.random.default_rng(717)
    for case in range(300):
        sigma = int(g.choice([2, 4, 20, 256]))
        n = int(g.integers(0, 20000))
        m = int(g.integers(1, 80))
        y = g.integers(0, sigma, size=n).astype(np.uint8)
        if n >= m and g.random() < 0.7:
            t = int(g.integers(0, n - m + 1))
            x = y[t:t + m].tobytes()
        else:
            x = g.integers(0, sigma, size=m).astype(np.uint8).tobytes()
        q = int(g.integers(1, min(m, 8) + 1))
        alpha = int(g.choice([1, 4, 8, 12]))
        w = int(g.choice([8, 16, 32, 64]))
        occ, lines, cov = O.hc_scan(x, y, q, alpha, w)
        assert occ == O.count(x, y), (case, n, m, q, alpha, w)
        assert 0 <= lines <= n // 128 + 1 and cov == n
        # stopped early: the windows decided so far are the brute force's
        occ2, _, cov2 = O.hc_scan(x, y, q, alpha, w, max_hashes=50)
        assert occ2 == (O.count(x, y[:cov2]) if cov2 >= m else 0), (case, cov2)


def test_hc_scan_lines_equal_sequential_reads():
    """The lines the C scan reads are those holding the positions the
    Python sequential search reads (the same algorithm written separately),
    at line sizes from 1 byte (every position read) to 128 bytes."""
    g = np.random.default_rng(718)
    for case in range(150):
        sigma = int(g.choice([2, 4, 27]))
        n = int(g.integers(0, 1500))
        m = int(g.integers(1, 60))
        y = g.integers(0, sigma, size=n).astype(np.uint8).tobytes()
        if n >= m and g.random() < 0.6:
            t = int(g.integers(0, n - m + 1))
            x = y[t:t + m]
        else:
            x = g.integers(0, sigma, size=m).astype(np.uint8).tobytes()
        q = int(g.integers(1, min(m, 8) + 1))
        alpha = int(g.choice([2, 8, 12]))
        w = int(g.choice([8, 32]))
        touched = set()
        occ = O.hc_search_sequential(x, y, q, alpha, w, touched=touched)
        for line in (1, 4, 16, 128):
            c_occ, c_lines, _ = O.hc_scan(x, y, q, alpha, w, line=line)
            assert c_occ == len(occ)
            assert c_lines == len({p // line for p in touched}), (case, line)
