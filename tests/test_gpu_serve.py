"""GPU parity of the serving loop (hc_serve_* through the C ABI): every
request's occurrence list equals the oracle's brute force over its text, the
same when the request runs alone and inside a mix of other requests, under a
budget that admits only a few requests at a time, across chunk boundaries."""
import sys
import threading

import numpy as np
import pytest

from oracle import hc_oracle as O
from paper_2310_15711_amd import binding as B
from paper_2310_15711_amd import workloads as W

pytestmark = pytest.mark.gpu

MiB = 1 << 20
CHUNK = 64 * MiB   # chunk of a text searched per step (hc.h)


def announce(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def texts():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    g = np.random.default_rng(77)
    a = (g.integers(0, 4, size=2 * CHUNK + 4 * MiB + 37, dtype=np.uint8) + ord("A")).astype(np.uint8)
    b = W.markov_text(CHUNK + 1234567, cfg=W.TEST_CFG)
    c = g.integers(0, 256, size=200_003, dtype=np.uint8)
    d = np.frombuffer(b"ACGTA", dtype=np.uint8).copy()
    # occurrences across the chunk boundaries of text a
    x0 = a[1000:1000 + 300].copy()
    for k in (1, 2):
        for back in (1, 17, 299):
            a[k * CHUNK - back:k * CHUNK - back + 300] = x0
    host = [a, b, c, d]
    dev = [torch.from_numpy(t).to("cuda:0") for t in host]
    torch.cuda.synchronize()
    return host, dev


def pick(g, y, m, extracted):
    m = min(m, y.size)
    if extracted:
        off = int(g.integers(0, y.size - m + 1))
        return y[off:off + m].tobytes()
    alphabet = np.unique(y[:65536])
    return alphabet[g.integers(0, alphabet.size, size=m)].astype(np.uint8).tobytes()


def requests(host, count, seed):
    g = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        t = int(g.integers(0, len(host)))
        m = int(round(float(np.exp(g.uniform(np.log(1), np.log(4096))))))
        out.append((t, pick(g, host[t], m, g.random() < 0.5)))
    return out


def check(host, reqs, got):
    for (t, x), pos in zip(reqs, got):
        want = O.occurrences(x, host[t]) if len(x) <= host[t].size else np.zeros(0, np.int64)
        assert np.array_equal(pos, want), (t, len(x))


def test_serve_against_oracle(texts):
    host, dev = texts
    srv = B.Server(dev, 256 * MiB)
    try:
        reqs = requests(host, 120, 1)
        # boundary-straddling pattern and extremes of m
        reqs += [(0, host[0][1000:1300].tobytes()), (0, host[0][5:6].tobytes()),
                 (1, host[1][CHUNK - 2:CHUNK + 2046].tobytes()), (3, b"ACGTA"), (3, b"ACGTAC"),
                 (2, host[2][-4096:].tobytes())]
        announce("serve oracle", len(reqs))
        ids = [srv.submit(t, x) for t, x in reqs]
        got = [srv.result(i) for i in ids]
        check(host, reqs, got)
        st = srv.stats()
        assert st["done"] == len(reqs)
        assert 0 < st["p50_us"] <= st["p99_us"]
        assert st["agg_gbps"] > 0
    finally:
        srv.close()


def test_alone_and_in_mix_identical(texts):
    host, dev = texts
    probe = [(0, host[0][CHUNK - 9:CHUNK + 23].tobytes()), (1, host[1][777:777 + 8].tobytes()),
             (2, host[2][100:104].tobytes())]
    srv = B.Server(dev, 512 * MiB)
    try:
        announce("serve alone")
        alone = [srv.result(srv.submit(t, x)) for t, x in probe]
        announce("serve mix")
        mix = requests(host, 300, 2)
        ids = [srv.submit(t, x) for t, x in mix[:150]]
        pids = [srv.submit(t, x) for t, x in probe]
        ids += [srv.submit(t, x) for t, x in mix[150:]]
        in_mix = [srv.result(i) for i in pids]
        others = [srv.result(i) for i in ids]
    finally:
        srv.close()
    for a, b in zip(alone, in_mix):
        assert np.array_equal(a, b)
    check(host, probe, alone)
    check(host, mix[:40], others[:40])


def test_small_budget_admission(texts):
    host, dev = texts
    # two requests' share: table 8 KiB (alpha 12, w 16) + 4128 + 32 KiB each
    per = 8192 + 4128 + 4096 * 8
    with pytest.raises(B.HCError):
        B.Server(dev, per - 1)
    srv = B.Server(dev, 2 * per)
    try:
        reqs = requests(host, 24, 3)
        announce("serve budget", len(reqs))
        ids = [srv.submit(t, x) for t, x in reqs]
        got = [srv.result(i) for i in ids]
        assert srv.stats()["done"] == len(reqs)
    finally:
        srv.close()
    check(host, reqs, got)


def test_overflowing_poll_keeps_request(texts):
    host, dev = texts
    srv = B.Server(dev, 64 * MiB)
    try:
        x = b"A"
        announce("serve overflow")
        rid = srv.submit(0, x)
        while True:
            r = srv.poll(rid, cap=10, timeout_us=100_000)
            if r is not None:
                break
        st, pos, cnt = r
        want = O.occurrences(x, host[0])
        assert st == B.HC_EOVERFLOW and cnt == want.size
        assert np.array_equal(pos, want[:10])
        st, pos, cnt = srv.poll(rid, cap=cnt)
        assert st == B.HC_OK and np.array_equal(pos, want)
        with pytest.raises(B.HCError):   # released
            srv.poll(rid, cap=cnt)
    finally:
        srv.close()


def test_invalid_requests(texts):
    _, dev = texts
    srv = B.Server(dev, 64 * MiB)
    try:
        for t, x in ((4, b"abc"), (-1, b"abc"), (0, b""), (0, b"a" * 4097)):
            with pytest.raises(B.HCError):
                srv.submit(t, x)
        with pytest.raises(B.HCError):
            srv.poll(12345)
        with pytest.raises(B.HCError):
            B.Server(dev, 64 * MiB, params=(0, 12, 64))   # w must be 16 or 32
    finally:
        srv.close()


def test_concurrent_submitters(texts):
    host, dev = texts
    srv = B.Server(dev, 128 * MiB)
    reqs = requests(host, 160, 4)
    got = [None] * len(reqs)
    errors = []

    def client(k):
        try:
            mine = list(range(k, len(reqs), 4))
            ids = [(i, srv.submit(*reqs[i])) for i in mine]
            for i, rid in ids:
                got[i] = srv.result(rid)
        except Exception as e:   # reported below
            errors.append(e)

    announce("serve threads")
    th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    srv.close()
    assert not errors, errors
    check(host, reqs, got)


def test_completion_queue_reports_each_request_once(texts):
    host, dev = texts
    srv = B.Server(dev, 128 * MiB)
    try:
        reqs = requests(host, 50, 5) + [(3, b"ACGTAC")]   # the last one completes at admission
        announce("serve next_done", len(reqs))
        ids = [srv.submit(t, x) for t, x in reqs]
        seen = []
        while len(seen) < len(ids):
            rid = srv.next_done(timeout_us=2_000_000)
            assert rid is not None, "a request did not complete"
            seen.append(rid)
        assert sorted(seen) == sorted(ids)
        assert srv.next_done() is None
        got = [srv.result(i) for i in ids]
    finally:
        srv.close()
    check(host, reqs, got)


def test_destroy_with_work_in_flight(texts):
    """Destroying a server while requests are queued and running neither
    hangs nor faults; a new server afterwards serves correctly."""
    host, dev = texts
    srv = B.Server(dev, 4 * (8192 + 4128 + 4096 * 8))   # four slots: most requests wait
    reqs = requests(host, 200, 6)
    announce("serve destroy in flight")
    for t, x in reqs:
        srv.submit(t, x)
    srv.close()
    srv = B.Server(dev, 64 * MiB)
    try:
        got = [srv.result(srv.submit(t, x)) for t, x in reqs[:20]]
    finally:
        srv.close()
    check(host, reqs[:20], got)


def test_served_workload_against_oracle():
    """Requests shaped like the served workload (four iid byte texts and four
    order-2 Markov texts, Poisson arrivals, m log-uniform in 4..2048,
    extracted with probability 1/2), submitted as they arrive; every one of
    the 1,000+ requests compared with the oracle."""
    import time

    import torch

    host = W.served_texts(n_each=24 * MiB)
    dev = [torch.from_numpy(t).to("cuda:0") for t in host]
    torch.cuda.synchronize()
    reqs = W.request_stream(host, rate=5000.0, duration=0.22, sub=7)
    assert len(reqs) >= 1000
    srv = B.Server(dev, 512 * MiB)
    announce("served workload", len(reqs))
    t0 = time.perf_counter()
    ids = []
    for r in reqs:
        ahead = t0 + r.arrival - time.perf_counter()
        if ahead > 0:
            time.sleep(ahead)
        ids.append(srv.submit(r.text, r.pattern))
    got = [srv.result(i, timeout_s=120) for i in ids]
    srv.close()
    for r, pos in zip(reqs, got):
        want = O.occurrences(r.pattern, host[r.text])
        assert np.array_equal(pos, want), (r.text, len(r.pattern), r.extracted_at)
    del dev
    torch.cuda.empty_cache()
