"""The autotuner (hc_autotune through the C ABI): its choices are valid, they
become the defaults of the tuned length buckets, and searches and batches run
with them stay identical to the oracle's brute force."""
import sys

import numpy as np
import pytest

from oracle import hc_oracle as O
from paper_2310_15711_amd import binding as B
from paper_2310_15711_amd import workloads as W

pytestmark = pytest.mark.gpu


def announce(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def text():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    y = W.iid_text(24 << 20, W.ALPHABETS[4], W.rng(W.TEST_CFG, 0, 41))
    return y, torch.from_numpy(y).to("cuda:0")


def test_autotune_choices_are_used_and_exact(text):
    y, yd = text
    lengths = [2, 4, 8, 32, 300, 1024]
    announce("autotune", lengths)
    try:
        tuned = B.hc_autotune(yd, lengths, patterns=3)
        assert [t["m"] for t in tuned] == lengths
        for t in tuned:
            q, alpha, w = t["params"]
            seg, sched, variant, wg = t["launch"]
            assert 1 <= q <= min(t["m"], 8)
            assert (alpha, w) in {(8, 8), (10, 16), (11, 16), (12, 16), (12, 32)} or \
                (t["m"] == 2 and (q, alpha, w) == (2, 16, 8))
            if variant == B.HC_VARIANT_SPARSE:
                assert t["m"] >= 256 and sched == B.HC_SCHED_SEGMENT
                assert seg in {min(k * (t["m"] - q + 1), 4096) for k in (1, 2, 4, 8)}   # whole shifts
            else:
                assert variant == B.HC_VARIANT_HC
                assert sched in (B.HC_SCHED_SEGMENT, B.HC_SCHED_DENSE) and seg in (48, 64, 80, 100)
            assert t["gbps"] > 0
        rs = np.random.default_rng(3)
        for t in tuned:
            m = t["m"]
            for _ in range(3):
                off = int(rs.integers(0, y.size - m))
                x = y[off:off + m].tobytes()
                p = B.hc_preprocess(x)   # defaults: the tuned entry of m's bucket
                info = B.hc_pattern_info(p)
                assert (info["q"], info["alpha"], info["w"]) == t["params"]
                announce("tuned search", m, off)
                got = B.find_all(p, yd).cpu().numpy()
                assert np.array_equal(got, O.occurrences(x, y))
        # a batch after tuning: q per pattern from the tuned buckets
        import torch

        texts = [y[: 3 << 20], y[5 << 20: 6 << 20]]
        off = np.array([0, texts[0].size, texts[0].size + texts[1].size], dtype=np.int64)
        d_text = torch.from_numpy(np.concatenate(texts)).to("cuda:0")
        pats = [y[o:o + m].tobytes() for o, m in ((100, 4), (7000, 32), (99999, 300), (12, 2))]
        pairs = [(p, t) for p in range(len(pats)) for t in range(len(texts))]
        want = [O.occurrences(pats[p], texts[t]) for p, t in pairs]
        total_want = sum(w.size for w in want)
        d_pos = torch.empty(total_want + 1, dtype=torch.int64, device="cuda:0")
        d_off = torch.empty(len(pairs) + 1, dtype=torch.int64, device="cuda:0")
        announce("tuned batch")
        st, total = B.hc_search_batched(d_text, off, pats, [p for p, _ in pairs], [t for _, t in pairs],
                                        d_pos, d_off)
        assert st == B.HC_OK and total == total_want
        po = d_off.cpu().numpy()
        pos = d_pos.cpu().numpy()
        for k, w in enumerate(want):
            assert np.array_equal(pos[po[k]:po[k + 1]], w), pairs[k]
    finally:
        B.hc_autotune_reset()


def test_batch_autotune_choice_is_used_and_exact():
    """hc_batch_autotune on a batch of the batched workload's shape: a valid
    choice, installed for plans and servers created afterwards, and the
    plans built with it give the oracle's lists."""
    import torch

    dev = torch.device("cuda:0")
    b = W.batched_config(n_texts=12, n_patterns=300, median=1 << 20, lo=64 << 10, hi=4 << 20)
    off = np.zeros(len(b.texts) + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in b.texts])
    d_text = torch.from_numpy(np.concatenate(b.texts)).to(dev)
    pp, pt = b.pairs[:, 0].copy(), b.pairs[:, 1].copy()
    try:
        announce("batch autotune", len(pp))
        t = B.hc_batch_autotune(d_text, off, b.patterns, pp, pt, max_pairs=800)
        assert (t["alpha"], t["w"]) in {(10, 16), (11, 16), (12, 16), (13, 16), (12, 32)}
        assert t["segment"] in (64, 80, 100) and t["group"] in (32, 64, 128) and t["wg_per_cu"] in (0, 2)
        assert t["gbps"] > 0
        plan = B.BatchPlan(d_text, off, b.patterns, pp, pt)
        d_off = torch.empty(len(pp) + 1, dtype=torch.int64, device=dev)
        st, total = plan.run(torch.empty(0, dtype=torch.int64, device=dev), d_off)
        d_pos = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
        st, total = plan.run(d_pos, d_off)
        assert st == B.HC_OK
        po, pos = d_off.cpu().numpy(), d_pos.cpu().numpy()
        g = np.random.default_rng(5)
        for k in np.sort(g.choice(len(pp), size=min(400, len(pp)), replace=False)):
            want = O.occurrences(b.patterns[int(pp[k])], b.texts[int(pt[k])])
            assert np.array_equal(pos[po[k]:po[k + 1]], want), int(k)
        # a server created now uses the tuned table shape; results unchanged
        srv = B.Server([d_text[int(off[i]):int(off[i + 1])] for i in range(3)], 64 << 20)
        ids = [srv.submit(i % 3, b.patterns[i]) for i in range(0, 60, 3)]
        for j, rid in enumerate(ids):
            i = 3 * j
            assert np.array_equal(srv.result(rid), O.occurrences(b.patterns[i], b.texts[i % 3]))
        srv.close()
    finally:
        B.hc_autotune_reset()
