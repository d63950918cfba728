"""Exhaustive binary parity of the single-pattern kernels (hc_search_async
through the C ABI) for every schedule and variant: each of the 126 binary
patterns of length 1..6, searched with every (q, alpha, w) point of a grid
(q capped at m), against

  - every binary text of length 1..12 at once: all of them concatenated,
    each followed by a separator byte that no pattern holds, so a window
    matches only inside one of the short texts;
  - a linearised de Bruijn sequence B(2, 12) (every 12-bit word once);
  - texts whose length puts the last window start at a tile boundary of
    the launch and inside a lane's block of starts.

Each list is compared element by element with the oracle's brute force.
Small alpha forces hash collisions (s = 0 when q > alpha), so the
verification of candidates runs often."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import hc_oracle as O
from paper_2310_15711_amd import binding as B

pytestmark = pytest.mark.gpu

M_MAX, N_MAX = 6, 12
GRID = ([(q, a, w) for w in (16, 32) for a in (1, 2, 3, 4, 8, 12) for q in range(1, 7)] +
        [(q, a, w) for w in (8, 64) for a in (2, 8) for q in (1, 3, 6)] +
        [(q, 16, 8) for q in (1, 2)])   # one-to-one hashes (s >= 8)
# (label, segment, schedule, variant): every schedule and variant
LAUNCHES = [
    ("segment-36", 36, B.HC_SCHED_SEGMENT, B.HC_VARIANT_HC),
    ("segment-100", 100, B.HC_SCHED_SEGMENT, B.HC_VARIANT_HC),
    ("wave-64", 64, B.HC_SCHED_WAVE, B.HC_VARIANT_HC),
    ("dense-64", 64, B.HC_SCHED_DENSE, B.HC_VARIANT_HC),
    ("sentinel-36", 36, B.HC_SCHED_SEGMENT, B.HC_VARIANT_SENTINEL),
    ("sparse-32", 32, B.HC_SCHED_AUTO, B.HC_VARIANT_SPARSE),
    ("sparse-1024", 1024, B.HC_SCHED_AUTO, B.HC_VARIANT_SPARSE),
]
# symbol bytes (0, 1) and the separator of the concatenated short texts
ENCODINGS = [(ord("a"), ord("b"), ord("c")), (0, 1, 2), (0xFE, 0xFF, 0x00), (0x80, 0x7F, 0x81)]


def announce(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def binary_patterns():
    return [np.array([(v >> k) & 1 for k in range(m)], dtype=np.uint8)
            for m in range(1, M_MAX + 1) for v in range(1 << m)]


def all_short_texts(sep_code=2):
    """Every binary string of length 1..N_MAX, each followed by sep_code."""
    parts = []
    for n in range(1, N_MAX + 1):
        v = np.arange(1 << n, dtype=np.int64)
        rows = ((v[:, None] >> np.arange(n)) & 1).astype(np.uint8)
        rows = np.concatenate([rows, np.full((rows.shape[0], 1), sep_code, np.uint8)], axis=1)
        parts.append(rows.reshape(-1))
    return np.concatenate(parts)


def de_bruijn(k=2, n=N_MAX):
    """Linearised de Bruijn sequence B(k, n) (the recursive construction of
    Fredricksen, Kessler and Maiorana), followed by its first n-1 symbols."""
    a = [0] * (k * n)
    seq = []

    def db(t, p):
        if t > n:
            if n % p == 0:
                seq.extend(a[1:p + 1])
        else:
            a[t] = a[t - p]
            db(t + 1, p)
            for j in range(a[t - p] + 1, k):
                a[t] = j
                db(t + 1, t)

    db(1, 1)
    s = np.array(seq + seq[:n - 1], dtype=np.uint8)
    return s


def test_de_bruijn_has_every_word_once():
    s = de_bruijn()
    assert s.size == (1 << N_MAX) + N_MAX - 1
    words = {int("".join(map(str, s[i:i + N_MAX][::-1])), 2) for i in range(s.size - N_MAX + 1)}
    assert len(words) == 1 << N_MAX


def boundary_texts(segment, variant, g):
    """Texts of 2 * tile + 5 and 2 * tile + segment + 3 bytes (tile = 256 *
    segment starts): the last window start lands on a tile boundary for
    m = 6 and inside a lane's block for the other lengths."""
    tile = 256 * segment
    return [g.integers(0, 2, size=2 * tile + 5, dtype=np.uint8),
            g.integers(0, 2, size=2 * tile + segment + 3, dtype=np.uint8)]


def run_text(y_codes, enc, pats, handles, launch, dev):
    """All (pattern, grid point) searches of one text with one launch shape,
    each into its own slice of one output buffer; compared with the oracle."""
    import torch

    lut = np.array(enc, dtype=np.uint8)
    y = lut[y_codes]
    want = [O.occurrences(lut[p].tobytes(), y) for p in pats]
    jobs = [(i, h) for i, hs in enumerate(handles) for h in hs]
    sizes = np.array([want[i].size for i, _ in jobs], dtype=np.int64)
    off = np.zeros(len(jobs) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    yd = torch.from_numpy(y).to(dev)
    out = torch.full((max(int(off[-1]), 1),), -1, dtype=torch.int64, device=dev)
    cnt = torch.full((len(jobs),), -1, dtype=torch.int64, device=dev)
    lc = B.hc_launch(launch[1], launch[2], launch[3], 0)
    L = B.lib()
    yp, op, cp = yd.data_ptr(), out.data_ptr(), cnt.data_ptr()
    stream = B._stream_ptr(None)
    for k, (i, h) in enumerate(jobs):
        st = L.hc_search_async(h.handle, yp, int(y.size), op + 8 * int(off[k]) if sizes[k] else None,
                               int(sizes[k]), cp + 8 * k, ctypes.byref(lc), stream)
        assert st == B.HC_OK, (launch, k, st)
    torch.cuda.synchronize()
    got_cnt = cnt.cpu().numpy()
    got = out.cpu().numpy()
    for k, (i, h) in enumerate(jobs):
        assert got_cnt[k] == sizes[k], (launch[0], enc, pats[i].tolist(), h.params, got_cnt[k], sizes[k])
    exp = np.concatenate([want[i] for i, _ in jobs]) if off[-1] else np.zeros(0, np.int64)
    if not np.array_equal(got[:off[-1]], exp):
        bad = int(np.nonzero(got[:off[-1]] != exp)[0][0])
        k = int(np.searchsorted(off, bad, side="right") - 1)
        i, h = jobs[k]
        raise AssertionError((launch[0], enc, pats[i].tolist(), h.params))
    return len(jobs)


class _Handle:
    def __init__(self, p, params):
        self.p, self.handle, self.params = p, p.handle, params


# a smaller grid for the texts that test tile and segment edges: every q,
# heavy collisions (alpha 3) and a usual table (alpha 12, w 32)
SMALL_GRID = [(q, a, w) for (a, w) in ((3, 16), (12, 32)) for q in range(1, 7)]


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def handles():
    """Pattern handles per (encoding, grid), built once for all launches."""
    pats = binary_patterns()
    cache = {}

    def get(enc, grid):
        key = (enc, tuple(grid))
        if key not in cache:
            lut = np.array(enc, dtype=np.uint8)
            cache[key] = [[_Handle(B.hc_preprocess(lut[p].tobytes(), prm), prm) for prm in grid
                           if prm[0] <= p.size] for p in pats]
        return cache[key]

    return pats, get


@pytest.mark.parametrize("launch", LAUNCHES, ids=[x[0] for x in LAUNCHES])
def test_exhaustive_binary(dev, handles, launch):
    """One launch shape: every binary text up to length 12 and the de Bruijn
    text with the full (q, alpha, w) grid; texts ending at and inside tile
    and segment boundaries, and the short texts again under two more byte
    encodings, with the smaller grid."""
    pats, get = handles
    g = np.random.default_rng([231015711, 7, launch[1], launch[3]])
    short, dbs = all_short_texts(), de_bruijn()
    jobs = [("all texts of length 1..12", short, ENCODINGS[0], GRID),
            ("de Bruijn B(2,12)", dbs, ENCODINGS[1], GRID)]
    for t in boundary_texts(launch[1], launch[3], g):
        jobs.append((f"{t.size} bytes", t, ENCODINGS[2], SMALL_GRID))
    jobs.append(("all texts of length 1..12", short, ENCODINGS[3], SMALL_GRID))
    launches = 0
    for name, t, enc, grid in jobs:
        announce("exhaustive single", launch[0], enc, name)
        launches += run_text(t, enc, pats, get(enc, grid), launch, dev)
    announce("exhaustive single launches", launch[0], launches)
