"""Exhaustive binary parity on the GPU: every text over two symbols of length
1..12 against every pattern of length 1..6 (1,031,940 pairs), searched as one
batch, for a grid of (q, alpha, w) and three byte encodings of the two
symbols. Small alpha forces hash collisions (and s = 0 when q > alpha), so
verification is exercised; the expected lists come from the definition of
an occurrence, computed with numpy on bit patterns."""
import sys

import numpy as np
import pytest

from paper_2310_15711_amd import binding as B

pytestmark = pytest.mark.gpu

N_MAX, M_MAX = 12, 6


def announce(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def bits_table(n):
    """All 2^n binary strings of length n, one per row (bit t of the row's
    index is symbol t)."""
    v = np.arange(1 << n, dtype=np.int64)
    return ((v[:, None] >> np.arange(n)) & 1).astype(np.uint8)


@pytest.fixture(scope="module")
def expected():
    texts = [bits_table(n) for n in range(1, N_MAX + 1)]
    pats = [bits_table(m) for m in range(1, M_MAX + 1)]
    # window values: bit k of a window starting at t is symbol t + k
    counts, positions = [], []
    for m, P in enumerate(pats, start=1):
        pv = np.arange(1 << m, dtype=np.int64)
        per_n = []
        for n, T in enumerate(texts, start=1):
            if n < m:
                per_n.append((np.zeros((1 << m, 1 << n), np.int64), [np.zeros(0, np.int64)] * ((1 << m) << n)))
                continue
            tv = np.arange(1 << n, dtype=np.int64)
            win = (tv[:, None] >> np.arange(n - m + 1)) & ((1 << m) - 1)       # (texts, starts)
            E = win[None, :, :] == pv[:, None, None]                             # (pats, texts, starts)
            per_n.append((E.sum(axis=2), E))
        for p in range(1 << m):
            for n in range(1, N_MAX + 1):
                c, E = per_n[n - 1]
                counts.append(c[p])
                if n >= m:
                    t_idx, start = np.nonzero(E[p])
                    positions.append(start.astype(np.int64))
    cnt = np.concatenate(counts).astype(np.int64)
    off = np.zeros(cnt.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(cnt)
    pos = np.concatenate(positions) if positions else np.zeros(0, np.int64)
    assert pos.size == off[-1]
    # the bit-pattern computation agrees with the oracle's definition
    from oracle import hc_oracle as O

    tl = [r for T in texts for r in T]
    pl = [r for P in pats for r in P]
    g = np.random.default_rng(1)
    for _ in range(500):
        p, t = int(g.integers(0, len(pl))), int(g.integers(0, len(tl)))
        k = p * len(tl) + t
        assert pos[off[k]:off[k + 1]].tolist() == O.occurrences_py(pl[p].tobytes(), tl[t].tobytes())
    return texts, pats, off, pos


def run_batch(texts, pats, enc, params):
    import torch

    dev = torch.device("cuda:0")
    lut = np.array(enc, dtype=np.uint8)
    text_rows = [lut[T] for T in texts]
    flat = np.concatenate([r.reshape(-1) for r in text_rows])
    lens = np.concatenate([np.full(r.shape[0], r.shape[1], np.int64) for r in text_rows])
    toff = np.zeros(lens.size + 1, dtype=np.int64)
    toff[1:] = np.cumsum(lens)
    patterns = [lut[row].tobytes() for P in pats for row in P]
    n_t, n_p = lens.size, len(patterns)
    pair_pat = np.repeat(np.arange(n_p, dtype=np.int32), n_t)      # pattern-major
    pair_text = np.tile(np.arange(n_t, dtype=np.int32), n_p)
    d_text = torch.from_numpy(flat).to(dev)
    plan = B.BatchPlan(d_text, toff, patterns, pair_pat, pair_text, params=params)
    d_off = torch.empty(pair_pat.size + 1, dtype=torch.int64, device=dev)
    st, total = plan.run(torch.empty(0, dtype=torch.int64, device=dev), d_off)
    d_pos = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
    st, total = plan.run(d_pos, d_off)
    assert st == B.HC_OK
    return d_off.cpu().numpy(), d_pos[:total].cpu().numpy()


GRID = [(q, a, w) for w in (16, 32) for a in (1, 2, 3, 4, 8, 12) for q in range(1, 7)]


@pytest.mark.parametrize("enc", [(ord("a"), ord("b")), (0, 1), (0xFE, 0xFF)])
def test_all_binary_texts_and_patterns(expected, enc):
    texts, pats, off, pos = expected
    for params in GRID:
        announce("exhaustive", enc, params)
        got_off, got_pos = run_batch(texts, pats, enc, params)
        assert np.array_equal(got_off, off), (enc, params)
        assert np.array_equal(got_pos, pos), (enc, params)
