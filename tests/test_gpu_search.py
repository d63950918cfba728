"""GPU parity of the single-pattern searching phase (hc_search through the C
ABI) against the oracle's brute force: element-by-element equality of the
occurrence lists (integer results, so bit-exact)."""
import random
import sys

import numpy as np
import pytest

from conftest import golden_lines
from oracle import hc_oracle as O
from paper_2310_15711_amd import binding as B
from paper_2310_15711_amd import workloads as W

pytestmark = pytest.mark.gpu


def announce(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def to_dev(y_np, dev):
    import torch

    return torch.from_numpy(np.ascontiguousarray(y_np)).to(dev)


def gpu_occ(x, y_dev, params=None, launch=None, cap=None):
    """Occurrences via hc_search_async + explicit capacity; returns numpy."""
    import torch

    p = B.hc_preprocess(x, params)
    n = int(y_dev.numel())
    if cap is None:
        cap = max(1, n)
    out = torch.empty(max(cap, 1), dtype=torch.int64, device=y_dev.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=y_dev.device)
    if n < len(x):
        st, c = B.hc_search(p, y_dev, out)
        return out[:0].cpu().numpy(), c
    B.hc_search_async(p, y_dev, out, cnt, launch=launch)
    torch.cuda.synchronize()
    c = int(cnt.item())
    return out[:min(c, cap)].cpu().numpy(), c


def test_hand_cases(torch_dev):
    for xh, yh, occ in golden_lines("hand_cases.txt"):
        x, y = bytes.fromhex(xh), bytes.fromhex(yh)
        want = [] if occ == "-" else [int(t) for t in occ.split(",")]
        announce("hand", xh, yh)
        yd = to_dev(np.frombuffer(y, dtype=np.uint8), torch_dev)
        p = B.hc_preprocess(x)
        got = B.find_all(p, yd).cpu().tolist()
        assert got == want, (xh, yh)


SCHEDS = [B.HC_SCHED_SEGMENT, B.HC_SCHED_WAVE, B.HC_SCHED_DENSE]


@pytest.mark.parametrize("sched", SCHEDS)
def test_random_against_oracle(torch_dev, sched):
    g = random.Random(2024 + sched)
    for case in range(160):
        sigma = g.choice([2, 4, 20, 64, 256])
        n = g.choice([g.randint(0, 3000), g.randint(3000, 200000)])
        m = g.choice([g.randint(1, 12), g.randint(12, 300), g.randint(300, 1200)])
        alphabet = np.array(g.sample(range(256), sigma), dtype=np.uint8)
        rs = np.random.default_rng(case * 7 + sched)
        y = alphabet[rs.integers(0, sigma, size=n)]
        if n >= m and g.random() < 0.8:
            t = g.randint(0, n - m)
            x = y[t:t + m].tobytes()
            for _ in range(g.randint(0, 5)):          # plant a few more copies
                u = g.randint(0, n - m)
                y[u:u + m] = np.frombuffer(x, dtype=np.uint8)
        else:
            x = alphabet[rs.integers(0, sigma, size=m)].tobytes()
        q = g.randint(1, min(m, 8))
        w = g.choice([8, 16, 32, 64])
        alpha = g.randint(1, {8: 16, 16: 15, 32: 14, 64: 13}[w])
        seg = g.choice([8, 12, 36, 132, 200])
        announce("random", sched, case, f"n={n} m={m} sigma={sigma} q={q} a={alpha} w={w} seg={seg}")
        yd = to_dev(y, torch_dev)
        got, c = gpu_occ(x, yd, (q, alpha, w), (seg, sched, 0, 0))
        want = O.occurrences(x, y)
        assert c == len(want)
        assert np.array_equal(got, want), (case, n, m, q, alpha, w, seg)


@pytest.mark.parametrize("sched", SCHEDS)
def test_planted_config(torch_dev, sched):
    p = W.planted_config()
    announce("planted", sched)
    yd = to_dev(p.y, torch_dev)
    got, c = gpu_occ(p.x, yd, None, (0, sched, 0, 0))
    want = O.occurrences(p.x, p.y)
    assert np.array_equal(got, want)
    assert set(p.plants) | {p.source} <= set(got.tolist())
    assert len(got) >= 101


@pytest.mark.parametrize("sched", SCHEDS)
def test_closed_forms(torch_dev, sched):
    n = 100_000
    ya = np.full(n, ord("a"), dtype=np.uint8)
    yd = to_dev(ya, torch_dev)
    for m in (1, 2, 7, 8, 33, 500):
        for q in sorted({1, min(m, 3), min(m, 8)}):
            announce("a^n", sched, m, q)
            got, c = gpu_occ(b"a" * m, yd, (q, 10, 32), (36, sched, 0, 0))
            assert c == n - m + 1
            assert np.array_equal(got, np.arange(n - m + 1))
    yab = np.frombuffer(b"ab" * (n // 2), dtype=np.uint8)
    yd = to_dev(yab, torch_dev)
    for k in (1, 3, 40):
        announce("(ab)^N", sched, k)
        got, c = gpu_occ(b"ab" * k, yd, None, (36, sched, 0, 0))
        assert np.array_equal(got, np.arange(0, n - 2 * k + 1, 2))


def test_overflow_reports_total_and_prefix(torch_dev):
    import torch

    n = 50_000
    yd = to_dev(np.full(n, 7, dtype=np.uint8), torch_dev)
    p = B.hc_preprocess(bytes([7, 7]))
    out = torch.full((1000,), -1, dtype=torch.int64, device=torch_dev)
    announce("overflow")
    st, c = B.hc_search(p, yd, out)
    assert st == B.HC_EOVERFLOW and c == n - 1
    assert np.array_equal(out.cpu().numpy(), np.arange(1000))
    # capacity 0: count only
    empty = torch.empty(0, dtype=torch.int64, device=torch_dev)
    st, c = B.hc_search(p, yd, empty)
    assert st == B.HC_EOVERFLOW and c == n - 1


def test_dense_output_every_tile_size(torch_dev):
    """Tiles whose occurrences are kept as bitmaps, at every tile size the
    launches use (one to many batches of bitmap words per tile), full and
    periodic densities, and capacities that end inside a tile."""
    n = 300_007
    cases = [(np.full(n, 7, dtype=np.uint8), bytes([7, 7]), 1),
             (np.frombuffer(b"abc" * (n // 3), dtype=np.uint8), b"ab", 3),
             (np.frombuffer(b"aaaab" * (n // 5), dtype=np.uint8), b"aa", None)]
    # a few to a few hundred occurrences per tile
    g = np.random.default_rng(17)
    for sigma, m in ((4, 4), (2, 6), (20, 2)):
        y = g.integers(0, sigma, size=n, dtype=np.uint8) + 65
        cases.append((y, y[1000:1000 + m].tobytes(), None))
    for y, x, period in cases:
        yd = to_dev(y, torch_dev)
        want = O.occurrences(x, y)
        if period:
            assert np.array_equal(want, np.arange(0, y.size - len(x) + 1, period))
        for launch in [(36, 0, 0, 0), (64, B.HC_SCHED_DENSE, 0, 0), (100, 0, 0, 0), (132, 0, 0, 0),
                       (200, 0, 0, 0), (512, 0, B.HC_VARIANT_SPARSE, 0), (4096, 0, B.HC_VARIANT_SPARSE, 0)]:
            for cap in (want.size, 40_017):
                announce("dense output", x, launch, cap)
                got, c = gpu_occ(x, yd, (2, 10, 16), launch, cap=cap)
                assert c == want.size
                assert np.array_equal(got, want[:cap]), (x, launch, cap)


def test_edges(torch_dev):
    import torch

    announce("edges")
    p = B.hc_preprocess(b"abc")
    out = torch.empty(16, dtype=torch.int64, device=torch_dev)
    for y in (b"", b"a", b"ab"):
        yd = torch.tensor(list(y), dtype=torch.uint8, device=torch_dev)
        assert B.hc_search(p, yd, out) == (B.HC_OK, 0)
    yd = torch.tensor(list(b"abc"), dtype=torch.uint8, device=torch_dev)
    assert B.hc_search(p, yd, out) == (B.HC_OK, 1) and int(out[0]) == 0
    # m = 1, every byte value
    y = np.arange(256, dtype=np.uint8).repeat(3)
    yd = to_dev(y, torch_dev)
    for b in (0, 1, 127, 128, 255):
        got, c = gpu_occ(bytes([b]), yd)
        assert got.tolist() == [3 * b, 3 * b + 1, 3 * b + 2]


def test_misaligned_text_pointers(torch_dev):
    g = np.random.default_rng(5)
    base = g.integers(0, 4, size=70_000, dtype=np.uint8) + ord("A")
    x = base[1234:1234 + 20].tobytes()
    bd = to_dev(base, torch_dev)
    for off in range(0, 17):
        for tail in (0, 1, 5, 15):
            announce("misaligned", off, tail)
            view = bd[off:bd.numel() - tail]
            got, c = gpu_occ(x, view, None, (12, 1, 0, 0))
            want = O.occurrences(x, base[off:base.size - tail])
            assert np.array_equal(got, want)


def test_parameter_invariance(torch_dev):
    y = W.markov_text(300_000, cfg=W.TEST_CFG)
    rs = np.random.default_rng(9)
    for m in (3, 16, 64, 257):
        t = int(rs.integers(0, y.size - m))
        x = y[t:t + m].tobytes()
        want = O.occurrences(x, y)
        yd = to_dev(y, torch_dev)
        for q in sorted({1, 2, min(m, 4), min(m, 8)}):
            for alpha, w in ((4, 8), (11, 16), (12, 32), (13, 64)):
                for seg, sched in ((16, 1), (132, 1), (64, 2), (100, 3)):
                    announce("invariance", m, q, alpha, w, seg, sched)
                    got, c = gpu_occ(x, yd, (q, alpha, w), (seg, sched, 0, 0))
                    assert np.array_equal(got, want), (m, q, alpha, w, seg, sched)


def test_repeated_launches_and_streams(torch_dev):
    import torch

    rs = np.random.default_rng(3)
    y = (rs.integers(0, 4, size=2_000_000, dtype=np.uint8) + 65)
    yd = to_dev(y, torch_dev)
    x = y[777:777 + 6].tobytes()
    want = O.occurrences(x, y)
    p = B.hc_preprocess(x)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for i in range(40):
        s = (s1, s2, None)[i % 3]
        n = int(rs.integers(1, y.size))
        out = torch.empty(n, dtype=torch.int64, device=torch_dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=torch_dev)
        announce("repeat", i, n)
        if s is not None:   # the buffers above were filled on the current stream
            s.wait_stream(torch.cuda.current_stream())
        B.hc_search_async(p, yd[:n], out, cnt, launch=(int(rs.choice([8, 36, 132])), 1, 0, 0),
                          stream=s)
        outs.append((n, out, cnt))
    torch.cuda.synchronize()
    for n, out, cnt in outs:
        w = want[want <= n - 6]
        assert int(cnt.item()) == w.size
        assert np.array_equal(out[:w.size].cpu().numpy(), w)


@pytest.mark.parametrize("sigma", [4, 20, 64])
def test_full_size_sampled(torch_dev, sigma):
    """The full 256 MiB single-pattern texts, launch shape as benchmarked,
    two sampled patterns per length, complete lists compared."""
    import torch

    y = W.single_text(sigma)
    yd = to_dev(y, torch_dev)
    for m in W.SINGLE_LENGTHS:
        for off, x in W.single_patterns(y, sigma, m, count=2):
            announce("full", sigma, m, off)
            want = O.occurrences(x, y)
            got, c = gpu_occ(x, yd, None, None, cap=int(want.size) + 16)
            assert c == want.size
            assert np.array_equal(got, want), (sigma, m, off)
    del yd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("variant", [B.HC_VARIANT_SPARSE, B.HC_VARIANT_SENTINEL])
def test_variants_against_oracle(torch_dev, variant):
    """The sparse variant (text read in place, no staging) and the sentinel
    variant (SHC) on random cases, closed forms and misaligned views."""
    g = random.Random(77 + variant)
    for case in range(120):
        sigma = g.choice([2, 4, 20, 256])
        n = g.choice([g.randint(0, 5000), g.randint(5000, 400000)])
        m = g.choice([g.randint(1, 12), g.randint(12, 300), g.randint(300, 2000)])
        alphabet = np.array(g.sample(range(256), sigma), dtype=np.uint8)
        rs = np.random.default_rng(case + 500)
        y = alphabet[rs.integers(0, sigma, size=n)]
        if n >= m and g.random() < 0.8:
            t = g.randint(0, n - m)
            x = y[t:t + m].tobytes()
            for _ in range(g.randint(0, 5)):
                u = g.randint(0, n - m)
                y[u:u + m] = np.frombuffer(x, dtype=np.uint8)
        else:
            x = alphabet[rs.integers(0, sigma, size=m)].tobytes()
        q = g.randint(1, min(m, 8))
        w = g.choice([8, 16, 32, 64])
        alpha = g.randint(1, {8: 16, 16: 15, 32: 14, 64: 13}[w])
        seg = g.choice([0, 32, 100, 1024, 4096])
        off = g.randint(0, 3)
        announce("variant", variant, case, f"n={n} m={m} sigma={sigma} q={q} a={alpha} w={w} seg={seg} off={off}")
        buf = to_dev(np.concatenate([np.zeros(off, np.uint8), y]), torch_dev)
        yd = buf[off:]
        got, c = gpu_occ(x, yd, (q, alpha, w), (seg, 0, variant, 0))
        want = O.occurrences(x, y)
        assert c == len(want)
        assert np.array_equal(got, want), (case, n, m, q, alpha, w, seg)
    n = 60_000
    yd = to_dev(np.full(n, ord("a"), dtype=np.uint8), torch_dev)
    for m in (1, 9, 300):
        announce("variant a^n", variant, m)
        got, c = gpu_occ(b"a" * m, yd, (min(m, 4), 10, 32), (64, 0, variant, 0))
        assert c == n - m + 1 and np.array_equal(got, np.arange(n - m + 1))


@pytest.mark.parametrize("sigma", [4, 64])
def test_variants_full_size(torch_dev, sigma):
    y = W.single_text(sigma)
    yd = to_dev(y, torch_dev)
    for variant, lengths in ((B.HC_VARIANT_SPARSE, (64, 256, 1024)), (B.HC_VARIANT_SENTINEL, (4, 32, 1024))):
        for m in lengths:
            for off, x in W.single_patterns(y, sigma, m, count=2):
                announce("variant full", variant, sigma, m, off)
                want = O.occurrences(x, y)
                got, c = gpu_occ(x, yd, None, (0, 0, variant, 0), cap=int(want.size) + 16)
                assert c == want.size and np.array_equal(got, want)
    del yd


def test_dense_without_links(torch_dev):
    """Dense schedule with m < 2q (the window-end hash alone, 16-bit packed),
    q up to 8, every alpha up to 16, all byte values, misaligned views."""
    g = np.random.default_rng(11)
    for sigma in (2, 4, 256):
        base = g.integers(0, sigma, size=300_011, dtype=np.uint8) * (255 // max(sigma - 1, 1))
        for m in range(1, 16):
            for q in range((m + 2) // 2, min(m, 8) + 1):
                for alpha, w in ((4, 8), (8, 8), (12, 16), (16, 8)):
                    off = int(g.integers(0, 4))
                    y = base[off:]
                    t = int(g.integers(0, y.size - m))
                    x = y[t:t + m].tobytes()
                    announce("dense no links", sigma, m, q, alpha, w, off)
                    yd = to_dev(base, torch_dev)[off:]
                    got, c = gpu_occ(x, yd, (q, alpha, w), (64, B.HC_SCHED_DENSE, 0, 0))
                    want = O.occurrences(x, y)
                    assert c == want.size and np.array_equal(got, want), (sigma, m, q, alpha, w)


def test_dense_direct_comparison_edges(torch_dev):
    """Windows of 4-8 bytes without links are compared with x directly (sums
    of absolute byte differences over the first and last 4 bytes): copies of
    x planted at both text ends and across tile boundaries, next to near
    misses that differ in one byte only (first, middle or last), patterns
    holding the byte values 0x00 and 0xFF."""
    g = np.random.default_rng(29)
    seg = 64
    tile = 256 * seg
    n = 3 * tile + 17
    for m in range(4, 9):
        for q in range((m + 2) // 2, min(m, 8) + 1):
            y = g.integers(0, 256, size=n, dtype=np.uint8)
            x = g.integers(0, 256, size=m, dtype=np.uint8)
            x[0], x[-1] = 0x00, 0xFF
            spots = [0, n - m, tile - 1, tile - m + 1, 2 * tile - 3, int(g.integers(0, n - m))]
            for t in spots:
                y[t:t + m] = x
            for k, t in enumerate((tile + 100, tile + 200, tile + 300)):
                miss = x.copy()
                j = (0, m // 2, m - 1)[k]
                miss[j] ^= 0x01
                y[t:t + m] = miss
            xb = x.tobytes()
            want = O.occurrences(xb, y)
            for alpha, w in ((8, 8), (12, 16)):
                announce("dense direct comparison", m, q, alpha, w)
                got, c = gpu_occ(xb, to_dev(y, torch_dev), (q, alpha, w), (seg, B.HC_SCHED_DENSE, 0, 0))
                assert c == want.size and np.array_equal(got, want), (m, q, alpha, w)


def test_markov_full_size_sampled(torch_dev):
    """The 256 MiB order-2 Markov text (the skewed-text workload), library
    defaults, two sampled patterns per length, complete lists compared."""
    y = W.markov_text(256 << 20)
    yd = to_dev(y, torch_dev)
    for m in W.MARKOV_LENGTHS:
        for off, x in W.markov_patterns(y, m, count=2):
            announce("markov full", m, off)
            want = O.occurrences(x, y)
            got, c = gpu_occ(x, yd, None, None, cap=int(want.size) + 16)
            assert c == want.size and np.array_equal(got, want), (m, off)
    del yd


def test_repeated_runs_identical(torch_dev):
    """The same searches repeated give byte-identical output (catches races in
    marking, parked chain walks and compaction): a periodic text where long
    patterns occur often and most windows need long chain walks."""
    import torch

    g = np.random.default_rng(21)
    block = g.integers(0, 4, size=5003, dtype=np.uint8) + ord("a")
    y = np.tile(block, 400)
    yd = to_dev(y, torch_dev)
    for m, q, sched in ((1000, 8, 1), (1000, 3, 1), (64, 4, 1), (4, 2, 3), (300, 5, 2)):
        x = y[777:777 + m].tobytes()
        want = O.occurrences(x, y)
        p = B.hc_preprocess(x, (q, 12, 32))
        out = torch.empty(want.size + 16, dtype=torch.int64, device=torch_dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=torch_dev)
        first = None
        for rep in range(12):
            announce("repeat identical", m, q, sched, rep)
            B.hc_search_async(p, yd, out, cnt, launch=(0, sched, 0, 0))
            torch.cuda.synchronize()
            got = out[:int(cnt.item())].cpu().numpy().copy()
            if first is None:
                first = got
                assert np.array_equal(got, want), (m, q)
            else:
                assert np.array_equal(got, first), (m, q, rep)


def test_threads_share_the_default_stream(torch_dev):
    """Host threads searching at once on the default stream (the workspace of
    that stream is shared): each call's lists equal the oracle's, also while
    other threads' calls make the workspace grow."""
    import threading

    import torch

    g = np.random.default_rng(41)
    y = (g.integers(0, 4, size=3_000_000, dtype=np.uint8) + 65)
    yd = to_dev(y, torch_dev)
    torch.cuda.synchronize()
    jobs = []
    for t in range(4):
        for k in range(12):
            n = int(g.integers(1000, y.size))   # text lengths vary: tile counts grow and shrink
            m = int(g.choice([3, 6, 16, 200]))
            o = int(g.integers(0, n - m))
            launch = (int(g.choice([8, 36, 100, 512])), 0,
                      B.HC_VARIANT_SPARSE if m >= 200 and k % 2 else 0, 0)
            jobs.append((t, n, y[o:o + m].tobytes(), launch))
    results, errors = {}, []

    def worker(t):
        try:
            for i, (tt, n, x, launch) in enumerate(jobs):
                if tt != t:
                    continue
                p = B.hc_preprocess(x)
                want_cap = n
                out = torch.empty(want_cap, dtype=torch.int64, device=torch_dev)
                cnt = torch.zeros(1, dtype=torch.int64, device=torch_dev)
                B.hc_search_async(p, yd[:n], out, cnt, launch=launch, stream=0)
                torch.cuda.synchronize()
                c = int(cnt.item())
                results[i] = out[:c].cpu().numpy()
        except Exception as e:   # reported by the main thread
            errors.append(repr(e))

    announce("threads on the default stream", len(jobs))
    ths = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    assert not errors, errors
    for i, (t, n, x, launch) in enumerate(jobs):
        assert np.array_equal(results[i], O.occurrences(x, y[:n])), (i, n, len(x), launch)
