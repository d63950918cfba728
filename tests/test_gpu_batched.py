"""GPU parity of the batched searching phase (hc_search_batched and batch
plans through the C ABI) against the oracle, pair by pair."""
import random
import sys

import numpy as np
import pytest

from oracle import hc_oracle as O
from paper_2310_15711_amd import binding as B
from paper_2310_15711_amd import workloads as W

pytestmark = pytest.mark.gpu


def announce(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def pack(texts, dev):
    import torch

    off = np.zeros(len(texts) + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in texts])
    allb = np.concatenate(texts) if texts else np.zeros(0, np.uint8)
    return torch.from_numpy(np.ascontiguousarray(allb)).to(dev), off


def check(texts, pats, pairs, d_text, off, pos, pair_off, cap):
    po = pair_off.cpu().numpy()
    pp = pos.cpu().numpy()
    assert po[0] == 0 and np.all(np.diff(po) >= 0)
    for k, (p, t) in enumerate(pairs):
        want = O.occurrences(pats[p], texts[t])
        assert po[k + 1] - po[k] == want.size, (k, p, t)
        lo, hi = po[k], min(po[k + 1], cap)
        if lo < hi:
            assert np.array_equal(pp[lo:hi], want[:hi - lo]), (k, p, t)


def make_case(seed, n_texts, n_pats, max_n, max_m, sigma):
    g = random.Random(seed)
    rs = np.random.default_rng(seed)
    alph = np.array(g.sample(range(256), sigma), dtype=np.uint8)
    texts = [alph[rs.integers(0, sigma, size=g.randint(0, max_n))] for _ in range(n_texts)]
    pats = []
    for _ in range(n_pats):
        m = g.randint(1, max_m)
        src = [t for t in texts if t.size >= m]
        if src and g.random() < 0.8:
            t = g.choice(src)
            o = g.randint(0, t.size - m)
            pats.append(t[o:o + m].tobytes())
        else:
            pats.append(alph[rs.integers(0, sigma, size=m)].tobytes())
    pairs = [(p, t) for p in range(n_pats) for t in range(n_texts) if g.random() < 0.6]
    g.shuffle(pairs)
    return texts, pats, pairs


@pytest.mark.parametrize("seed,sigma,w", [(1, 4, 16), (2, 20, 32), (3, 2, 16), (4, 256, 32)])
def test_batched_random(seed, sigma, w):
    import torch

    dev = torch.device("cuda:0")
    texts, pats, pairs = make_case(seed, 7, 40, 150_000, 300, sigma)
    d_text, off = pack(texts, dev)
    total_want = sum(O.count(pats[p], texts[t]) for p, t in pairs)
    cap = total_want + 5
    pos = torch.full((cap,), -1, dtype=torch.int64, device=dev)
    pair_off = torch.empty(len(pairs) + 1, dtype=torch.int64, device=dev)
    announce("batched", seed, sigma, w, len(pairs), total_want)
    st, total = B.hc_search_batched(d_text, off, pats, [p for p, _ in pairs], [t for _, t in pairs],
                                    pos, pair_off, params=(0, 12, w))
    assert st == B.HC_OK and total == total_want
    check(texts, pats, pairs, d_text, off, pos, pair_off, cap)


@pytest.mark.parametrize("q", [5, 6, 7, 8])
def test_batched_long_qgrams_without_links(q):
    """Patterns of length q..2q-1 with an explicit q (no links: the dense
    test in the batched kernel, q-grams of 5-8 bytes) next to longer ones
    (the searching loop), one plan, tables of 8 and 16 KiB."""
    import torch

    dev = torch.device("cuda:0")
    g = random.Random(40 + q)
    rs = np.random.default_rng(40 + q)
    for sigma, alpha, w in ((4, 12, 16), (3, 12, 32)):
        alph = np.array(g.sample(range(256), sigma), dtype=np.uint8)
        texts = [alph[rs.integers(0, sigma, size=g.randint(1, 200_000))] for _ in range(5)]
        pats = []
        for _ in range(24):
            m = g.randint(q, 2 * q - 1) if g.random() < 0.75 else g.randint(2 * q, 40)
            t = g.choice(texts)
            if t.size >= m and g.random() < 0.8:
                o = g.randint(0, t.size - m)
                pats.append(t[o:o + m].tobytes())
            else:
                pats.append(alph[rs.integers(0, sigma, size=m)].tobytes())
        pairs = [(p, t) for p in range(len(pats)) for t in range(len(texts))]
        d_text, off = pack(texts, dev)
        total_want = sum(O.count(pats[p], texts[t]) for p, t in pairs)
        cap = total_want + 5
        pos = torch.full((cap,), -1, dtype=torch.int64, device=dev)
        pair_off = torch.empty(len(pairs) + 1, dtype=torch.int64, device=dev)
        announce("batched long q-grams", q, sigma, alpha, w, len(pairs), total_want)
        st, total = B.hc_search_batched(d_text, off, pats, [p for p, _ in pairs], [t for _, t in pairs],
                                        pos, pair_off, params=(q, alpha, w))
        assert st == B.HC_OK and total == total_want
        check(texts, pats, pairs, d_text, off, pos, pair_off, cap)


def test_batched_overflow_and_scratch_growth():
    import torch

    dev = torch.device("cuda:0")
    # dense: "aa" and a^40 in a long run of a's, more positions (about 9 M)
    # than the initial scratch (8 Mi), so the run grows it and runs again
    texts = [np.full(4_500_000, 97, dtype=np.uint8), np.full(300, 97, dtype=np.uint8)]
    pats = [b"aa", b"a" * 40, b"b"]
    pairs = [(0, 0), (1, 0), (2, 0), (0, 1), (1, 1)]
    d_text, off = pack(texts, dev)
    total_want = sum(O.count(pats[p], texts[t]) for p, t in pairs)
    pair_off = torch.empty(len(pairs) + 1, dtype=torch.int64, device=dev)
    pos = torch.empty(total_want, dtype=torch.int64, device=dev)
    announce("dense batched", total_want)
    st, total = B.hc_search_batched(d_text, off, pats, [p for p, _ in pairs], [t for _, t in pairs],
                                    pos, pair_off)
    assert st == B.HC_OK and total == total_want
    check(texts, pats, pairs, d_text, off, pos, pair_off, total_want)
    # a capacity below the total: offsets complete, positions below cap written
    cap = 1000
    pos2 = torch.empty(cap, dtype=torch.int64, device=dev)
    st, total = B.hc_search_batched(d_text, off, pats, [p for p, _ in pairs], [t for _, t in pairs],
                                    pos2, pair_off)
    assert st == B.HC_EOVERFLOW and total == total_want
    check(texts, pats, pairs, d_text, off, pos2, pair_off, cap)


def test_batched_edges():
    import torch

    dev = torch.device("cuda:0")
    texts = [np.frombuffer(b"abracadabra", np.uint8).copy(), np.zeros(0, np.uint8),
             np.frombuffer(b"ab", np.uint8).copy()]
    pats = [b"abra", b"a", b"abracadabraX", b"ab"]
    pairs = [(0, 0), (1, 0), (2, 0), (0, 1), (3, 2), (2, 2), (1, 2), (0, 0)]
    d_text, off = pack(texts, dev)
    pos = torch.empty(64, dtype=torch.int64, device=dev)
    pair_off = torch.empty(len(pairs) + 1, dtype=torch.int64, device=dev)
    announce("edges batched")
    st, total = B.hc_search_batched(d_text, off, pats, [p for p, _ in pairs], [t for _, t in pairs],
                                    pos, pair_off)
    assert st == B.HC_OK
    check(texts, pats, pairs, d_text, off, pos, pair_off, 64)
    # no pairs at all
    st, total = B.hc_search_batched(d_text, off, pats, [], [], pos, pair_off[:1])
    assert st == B.HC_OK and total == 0 and int(pair_off[0]) == 0


def test_plan_graph_replays_match_eager():
    """A plan replays its captured graph; every replay, with other GPU work
    in between, gives the same CSR result as a fresh one-shot search."""
    import torch

    dev = torch.device("cuda:0")
    b = W.batched_config(n_texts=9, n_patterns=60, median=200_000, lo=20_000, hi=600_000)
    d_text, off = pack(b.texts, dev)
    pairs = [tuple(x) for x in b.pairs.tolist()]
    pp, pt = [p for p, _ in pairs], [t for _, t in pairs]
    total_want = sum(O.count(b.patterns[p], b.texts[t]) for p, t in pairs)
    cap = total_want + 1
    ref_pos = torch.empty(cap, dtype=torch.int64, device=dev)
    ref_off = torch.empty(len(pairs) + 1, dtype=torch.int64, device=dev)
    announce("plan eager")
    st, total = B.hc_search_batched(d_text, off, b.patterns, pp, pt, ref_pos, ref_off)
    assert total == total_want
    check(b.texts, b.patterns, pairs, d_text, off, ref_pos, ref_off, cap)
    plan = B.BatchPlan(d_text, off, b.patterns, pp, pt)
    pos = torch.empty(cap, dtype=torch.int64, device=dev)
    pair_off = torch.empty(len(pairs) + 1, dtype=torch.int64, device=dev)
    for r in range(4):
        announce("plan replay", r)
        pos.fill_(-7)
        pair_off.fill_(-7)
        junk = torch.randn(1 << 20, device=dev).sum()   # unrelated eager work in between
        st, total = plan.run(pos, pair_off)
        torch.cuda.synchronize()
        assert st == B.HC_OK and total == total_want
        assert torch.equal(pair_off, ref_off)
        assert torch.equal(pos[:total], ref_pos[:total])
        del junk


def test_batched_workload_sample_against_oracle():
    """The full batched workload (64 texts of log-normal length, 4096
    patterns of log-uniform length 4..1024, about 87 K pairs) run as one plan;
    1,200 seeded pairs compared element by element with the oracle, and the
    plan's per-pair counts summed over those pairs."""
    import torch

    dev = torch.device("cuda:0")
    b = W.batched_config()
    d_text, off = pack(b.texts, dev)
    pp, pt = b.pairs[:, 0].copy(), b.pairs[:, 1].copy()
    announce("batched workload", len(b.texts), len(b.patterns), len(pp))
    plan = B.BatchPlan(d_text, off, b.patterns, pp, pt)
    pair_off = torch.empty(len(pp) + 1, dtype=torch.int64, device=dev)
    st, total = plan.run(torch.empty(0, dtype=torch.int64, device=dev), pair_off)
    pos = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
    st, total2 = plan.run(pos, pair_off)
    assert st == B.HC_OK and total2 == total
    po = pair_off.cpu().numpy()
    assert po[0] == 0 and po[-1] == total and np.all(np.diff(po) >= 0)
    g = np.random.default_rng([231015711, 4, 9, 1])
    for k in np.sort(g.choice(len(pp), size=1200, replace=False)):
        want = O.occurrences(b.patterns[int(pp[k])], b.texts[int(pt[k])])
        lo, hi = int(po[k]), int(po[k + 1])
        assert hi - lo == want.size, (int(k), hi - lo, want.size)
        assert np.array_equal(pos[lo:hi].cpu().numpy(), want), int(k)
    del plan, d_text, pos
    torch.cuda.empty_cache()
