"""Seeded synthetic workloads for the HC searching phase.

This module only draws inputs: texts, patterns, planted copies, request
streams. It holds none of the method's arithmetic, and both the product
tests and the oracle consume what it produces.

The paper measures on 100 MB genome, protein and English texts of the
Pizza&Chili corpus (Section 4); those are not available here, so they are
stood in for by

* iid uniform text over ACGT (sigma = 4) for the genome,
* iid uniform text over the 20 amino-acid letters for the protein,
* an order-2 Markov chain over 26 lower-case letters and space, with
  Dirichlet(0.3) transition rows, for the English text,

plus iid base64 text (sigma = 64) and iid bytes (sigma = 256). Patterns are
copied out of the text at seeded offsets, as the paper extracts them at
random (Section 4).

Every generator draws from ``numpy.random.default_rng([SEED, cfg, stream, sub])``
with stream 0 = text, 1 = patterns/offsets/lengths, 2 = plants/arrivals,
3 = Markov uniforms.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED = 231015711
KiB = 1 << 10
MiB = 1 << 20

ALPHABETS = {
    4: b"ACGT",
    20: b"ACDEFGHIKLMNPQRSTVWY",
    64: b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/",
    256: bytes(range(256)),
}
MARKOV_SYMBOLS = b"abcdefghijklmnopqrstuvwxyz "  # 27 symbols

# configuration ids used in the seeds
CFG_PLANTED, CFG_SINGLE, CFG_MARKOV, CFG_BATCHED, CFG_SERVED = 1, 2, 3, 4, 5
TEST_CFG = 99


def rng(cfg: int, stream: int, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED, cfg, stream, sub])


def iid_text(n: int, alphabet: bytes, g: np.random.Generator) -> np.ndarray:
    """n bytes drawn iid uniformly from ``alphabet``."""
    table = np.frombuffer(alphabet, dtype=np.uint8)
    if len(alphabet) == 256:
        return g.integers(0, 256, size=n, dtype=np.uint8)
    idx = g.integers(0, len(alphabet), size=n, dtype=np.uint8)
    return table[idx]


# ---------------------------------------------------------------------------
# Order-2 Markov text (stand-in for English)
# ---------------------------------------------------------------------------

_WALK_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "markov_walk.c")
_WALK_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmarkov_walk.so")
_walk = None


def build_walker(force: bool = False) -> str:
    import subprocess

    if force or not os.path.exists(_WALK_LIB) or (
        os.path.getmtime(_WALK_LIB) < os.path.getmtime(_WALK_SRC)
    ):
        tmp = _WALK_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               _WALK_SRC, "-o", tmp])
        os.replace(tmp, _WALK_LIB)
    return _WALK_LIB


def _walker():
    global _walk
    if _walk is None:
        if not os.path.exists(_WALK_LIB):
            build_walker()
        lib = ctypes.CDLL(_WALK_LIB)
        p, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.markov2_walk.restype = None
        lib.markov2_walk.argtypes = [p, ctypes.c_int, p, p, p, i64]
        _walk = lib
    return _walk


def markov_rows(cfg: int, sub: int = 0, k: int = 27, conc: float = 0.3) -> np.ndarray:
    """k*k rows (state = (prev2, prev1), row-major) of Dirichlet(conc) transitions."""
    g = rng(cfg, 0, sub)
    return g.dirichlet(np.full(k, conc), size=k * k)


def markov_text(n: int, cfg: int = CFG_MARKOV, sub: int = 0,
                rows: Optional[np.ndarray] = None, walk_sub: Optional[int] = None) -> np.ndarray:
    """Order-2 Markov walk over ``MARKOV_SYMBOLS``.

    The initial pair is uniform; each next symbol is the first index whose
    cumulative row probability exceeds a uniform u (the last index takes the
    remainder). Uniforms come from stream 3, in chunks, and the walk itself
    runs in a small C loop.
    """
    k = len(MARKOV_SYMBOLS)
    if rows is None:
        rows = markov_rows(cfg, sub, k)
    cum = np.ascontiguousarray(np.cumsum(rows, axis=1), dtype=np.float64)
    ws = sub if walk_sub is None else walk_sub
    g = rng(cfg, 3, ws)
    out = np.empty(n, dtype=np.uint8)
    if n == 0:
        return out
    first = g.integers(0, k, size=2)
    state = np.array([first[0], first[1]], dtype=np.int32)
    syms = np.frombuffer(MARKOV_SYMBOLS, dtype=np.uint8)
    lib = _walker()
    chunk = 1 << 24
    pos = 0
    while pos < n:
        c = min(chunk, n - pos)
        u = g.random(c)
        lib.markov2_walk(cum.ctypes.data, k, state.ctypes.data,
                         u.ctypes.data, out[pos:].ctypes.data, c)
        pos += c
    return syms[out]


# ---------------------------------------------------------------------------
# Patterns and plants
# ---------------------------------------------------------------------------

def extract_patterns(y: np.ndarray, m: int, count: int, g: np.random.Generator
                     ) -> List[Tuple[int, bytes]]:
    """``count`` patterns of length m copied from y at offsets ~ U[0, n-m]."""
    n = int(y.size)
    offs = g.integers(0, n - m + 1, size=count)
    return [(int(t), y[int(t):int(t) + m].tobytes()) for t in offs]


def plant(y: np.ndarray, x: bytes, count: int, g: np.random.Generator,
          avoid: Sequence[int] = ()) -> List[int]:
    """Write x at ``count`` offsets chosen by rejection so that all planted
    intervals (and those in ``avoid``) are pairwise disjoint; returns the
    offsets, ascending. Modifies y in place."""
    m, n = len(x), int(y.size)
    taken = sorted(avoid)
    chosen: List[int] = []
    xa = np.frombuffer(x, dtype=np.uint8)
    while len(chosen) < count:
        t = int(g.integers(0, n - m + 1))
        if all(abs(t - u) >= m for u in taken):
            taken.append(t)
            chosen.append(t)
    for t in chosen:
        y[t:t + m] = xa
    return sorted(chosen)


@dataclass
class Planted:
    y: np.ndarray
    x: bytes
    source: int
    plants: List[int]


def planted_config(n: int = 1 * MiB, m: int = 32, extra: int = 100) -> Planted:
    """One iid ACGT text, a pattern copied from it, and ``extra`` disjoint
    planted copies of that pattern."""
    y = iid_text(n, ALPHABETS[4], rng(CFG_PLANTED, 0))
    g1 = rng(CFG_PLANTED, 1)
    t0 = int(g1.integers(0, n - m + 1))
    x = y[t0:t0 + m].tobytes()
    plants = plant(y, x, extra, rng(CFG_PLANTED, 2), avoid=[t0])
    return Planted(y=y, x=x, source=t0, plants=plants)


SINGLE_SIGMAS = (4, 20, 64)
SINGLE_LENGTHS = (2, 4, 8, 16, 32, 64, 128, 256, 512, 1024)
MARKOV_LENGTHS = (4, 8, 16, 32, 64, 128, 256, 512, 1024)


def single_text(sigma: int, n: int = 256 * MiB) -> np.ndarray:
    """Text of the single-pattern workload for one alphabet size."""
    return iid_text(n, ALPHABETS[sigma], rng(CFG_SINGLE, 0, sigma))


def single_patterns(y: np.ndarray, sigma: int, m: int, count: int = 100):
    return extract_patterns(y, m, count, rng(CFG_SINGLE, 1, sigma * 4096 + m))


def markov_patterns(y: np.ndarray, m: int, count: int = 100):
    return extract_patterns(y, m, count, rng(CFG_MARKOV, 1, m))


# ---------------------------------------------------------------------------
# Batched workload
# ---------------------------------------------------------------------------

@dataclass
class Batch:
    texts: List[np.ndarray]
    text_sigma: List[int]
    patterns: List[bytes]
    pattern_sigma: List[int]
    pairs: np.ndarray            # (k, 2) int32: pattern index, text index
    pattern_source: List[Tuple[int, int]] = field(default_factory=list)


def batched_config(n_texts: int = 64, n_patterns: int = 4096,
                   median: int = 4 * MiB, lo: int = 64 * KiB, hi: int = 16 * MiB,
                   m_lo: int = 4, m_hi: int = 1024, cfg: int = CFG_BATCHED) -> Batch:
    """Texts with log-normal lengths clipped to [lo, hi], alphabet (4,20,64)
    by index mod 3; patterns with log-uniform lengths in [m_lo, m_hi], each
    copied from a seeded text of its alphabet; every pattern is paired with
    every text of its alphabet."""
    g = rng(cfg, 1, 0)
    lens = np.clip(np.round(np.exp(g.normal(np.log(median), 1.0, size=n_texts))), lo, hi)
    lens = lens.astype(np.int64)
    sig = [SINGLE_SIGMAS[i % 3] for i in range(n_texts)]
    texts = [iid_text(int(lens[i]), ALPHABETS[sig[i]], rng(cfg, 0, i)) for i in range(n_texts)]
    gp = rng(cfg, 1, 1)
    ms = np.round(np.exp(gp.uniform(np.log(m_lo), np.log(m_hi), size=n_patterns))).astype(np.int64)
    pats, psig, src = [], [], []
    by_sigma = {s: [i for i in range(n_texts) if sig[i] == s] for s in SINGLE_SIGMAS}
    for p in range(n_patterns):
        s = SINGLE_SIGMAS[p % 3]
        cands = [i for i in by_sigma[s] if texts[i].size >= ms[p]]
        ti = cands[int(gp.integers(0, len(cands)))]
        t = int(gp.integers(0, texts[ti].size - ms[p] + 1))
        pats.append(texts[ti][t:t + int(ms[p])].tobytes())
        psig.append(s)
        src.append((ti, t))
    pairs = [(p, t) for p in range(n_patterns) for t in by_sigma[psig[p]]]
    return Batch(texts=texts, text_sigma=sig, patterns=pats, pattern_sigma=psig,
                 pairs=np.asarray(pairs, dtype=np.int32).reshape(-1, 2),
                 pattern_source=src)


# ---------------------------------------------------------------------------
# Served workload
# ---------------------------------------------------------------------------

@dataclass
class Request:
    arrival: float      # scheduled arrival, seconds from stream start
    text: int
    pattern: bytes
    extracted_at: int   # -1 when the pattern was drawn at random


def served_texts(n_each: int = 128 * MiB, cfg: int = CFG_SERVED) -> List[np.ndarray]:
    """Four iid byte texts, then four order-2 Markov texts (one shared chain,
    separate walks)."""
    texts = [iid_text(n_each, ALPHABETS[256], rng(cfg, 0, i)) for i in range(4)]
    rows = markov_rows(CFG_MARKOV, 0)
    for i in range(4):
        texts.append(markov_text(n_each, cfg=cfg, rows=rows, walk_sub=100 + i))
    return texts


def request_stream(texts: Sequence[np.ndarray], rate: float, duration: float,
                   m_lo: int = 4, m_hi: int = 2048, cfg: int = CFG_SERVED,
                   sub: int = 0) -> List[Request]:
    """Open-loop Poisson arrivals at ``rate`` per second for ``duration`` s."""
    g = rng(cfg, 2, sub)
    out: List[Request] = []
    alphabets = {}   # symbols of each text's first 64 KiB, computed once per text
    t = 0.0
    while True:
        t += float(g.exponential(1.0 / rate))
        if t >= duration:
            break
        ti = int(g.integers(0, len(texts)))
        y = texts[ti]
        m = int(round(float(np.exp(g.uniform(np.log(m_lo), np.log(m_hi))))))
        m = min(m, int(y.size))
        if g.random() < 0.5:
            off = int(g.integers(0, y.size - m + 1))
            x = y[off:off + m].tobytes()
        else:
            off = -1
            if ti not in alphabets:
                alphabets[ti] = np.unique(y[: min(int(y.size), 1 << 16)])
            alphabet = alphabets[ti]
            x = alphabet[g.integers(0, alphabet.size, size=m)].astype(np.uint8).tobytes()
        out.append(Request(arrival=t, text=ti, pattern=x, extracted_at=off))
    return out
