"""Oracle for the Hash Chain (HC) searching phase.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module or load
``liboracle.so``. The product path never does, and nothing here is shared
with the HIP path (no kernels, headers, helpers or tables).

What is here, each written from the paper's definitions rather than from
its printed listings:

* ``occurrences`` / ``occurrences_py``: the plain definition of the
  problem (Section 1; notation of Section 2) -- every start t with
  y[t..t+m-1] = x -- by direct comparison (C, multi-threaded) and in pure
  Python for tiny inputs. HC reaches exactly this set, so this is the
  oracle for every occurrence list.
* ``shift_s``, ``qgram_hash``, ``link_bit``: the hash h of equation (3),
  the bit shift s of equation (4), the final reduction modulo 2^alpha, and
  the link hash lambda of equation (5).
* ``link_table``: the word vector F as the paper defines it -- equation (1)
  applied to every adjacent non-overlapping pair of q-grams, then equation
  (2) for the q-grams that start in the first q positions, applied only to
  words still empty after all links (Section 3.4, first optimisation).
* ``chain_head_hash``: H_v, the hash of the first q-gram of the chain that
  ends at the last pattern position (Section 3.4, second optimisation).
* ``hc_scan`` (C, ``hc_seq.c``): the same searching phase over a whole
  text, reporting the occurrences it finds and how many distinct memory
  lines of the text it reads -- the text bytes the method itself needs.
  Pinned against the brute force (occurrences) and against
  ``hc_search_sequential`` (lines read) in the tests.
* ``hc_search_sequential``: the searching phase of Section 3.3 run one
  window at a time, for tiny inputs. It exists to pin ``link_table`` and
  ``chain_head_hash`` against brute force. It uses the verification reading
  recorded in the design notes: a window whose q-grams all link is compared
  with x at its own start (window end minus m plus 1), and that start is
  reported.

Parity pins live in ``tests/test_oracle.py``. Nothing here is "parity
unpinned" except the printed F of the paper's Fig. 2 example, whose figure
body is missing from the source and is therefore not compared.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCE_PATH = os.path.join(_HERE, "brute.c")
SEQ_SOURCE_PATH = os.path.join(_HERE, "hc_seq.c")

_lib = None


def build(force: bool = False) -> str:
    """Compile brute.c and hc_seq.c into liboracle.so with gcc (plain C, -O2)."""
    import subprocess

    if force or not os.path.exists(LIB_PATH) or any(
        os.path.getmtime(LIB_PATH) < os.path.getmtime(src) for src in (SOURCE_PATH, SEQ_SOURCE_PATH)
    ):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
             SOURCE_PATH, SEQ_SOURCE_PATH, "-o", tmp]
        )
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.oracle_occurrences.restype = i64
        lib.oracle_occurrences.argtypes = [p, i64, p, i64, p, i64, ctypes.c_int]
        lib.oracle_count.restype = i64
        lib.oracle_count.argtypes = [p, i64, p, i64, ctypes.c_int]
        lib.oracle_matches_at.restype = ctypes.c_int
        lib.oracle_matches_at.argtypes = [p, i64, p, i64, i64]
        i32 = ctypes.c_int
        lib.oracle_hc_scan.restype = i32
        lib.oracle_hc_scan.argtypes = [p, i64, p, i64, i32, i32, i32, i64, i64, p, p, p]
        _lib = lib
    return _lib


def _as_u8(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(a), dtype=np.uint8)
    a = np.ascontiguousarray(a)
    if a.dtype != np.uint8:
        raise TypeError("oracle inputs are uint8 arrays or bytes")
    return a


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


# ---------------------------------------------------------------------------
# The problem itself (Section 1; Section 2 notation)
# ---------------------------------------------------------------------------

def occurrences_py(x: bytes, y: bytes) -> List[int]:
    """Every t, 0 <= t <= n-m, with y[t..t+m-1] = x; pure Python, tiny inputs."""
    m, n = len(x), len(y)
    if m < 1:
        raise ValueError("pattern must be non-empty")
    return [t for t in range(n - m + 1) if y[t:t + m] == x]


def occurrences(x, y, threads: int | None = None) -> np.ndarray:
    """Same set as occurrences_py, by the C brute force; int64 ascending."""
    xa, ya = _as_u8(x), _as_u8(y)
    m, n = int(xa.size), int(ya.size)
    if m < 1:
        raise ValueError("pattern must be non-empty")
    th = threads or default_threads()
    lib = _load()
    total = lib.oracle_count(xa.ctypes.data, m, ya.ctypes.data, n, th)
    if total < 0:
        raise RuntimeError(f"oracle failed ({total})")
    out = np.empty(max(total, 1), dtype=np.int64)
    got = lib.oracle_occurrences(xa.ctypes.data, m, ya.ctypes.data, n,
                                 out.ctypes.data, total, th)
    if got != total:
        raise RuntimeError("oracle count changed between calls")
    return out[:total]


def count(x, y, threads: int | None = None) -> int:
    xa, ya = _as_u8(x), _as_u8(y)
    th = threads or default_threads()
    c = _load().oracle_count(xa.ctypes.data, int(xa.size), ya.ctypes.data,
                             int(ya.size), th)
    if c < 0:
        raise RuntimeError(f"oracle failed ({c})")
    return int(c)


def matches_at(x, y, t: int) -> bool:
    """Whether x occurs at start t of y (the definition for a single t)."""
    xa, ya = _as_u8(x), _as_u8(y)
    return bool(_load().oracle_matches_at(xa.ctypes.data, int(xa.size),
                                          ya.ctypes.data, int(ya.size), int(t)))


# ---------------------------------------------------------------------------
# Hash functions (Section 3.2, equations (3)-(5))
# ---------------------------------------------------------------------------

def shift_s(alpha: int, q: int) -> int:
    """Equation (4): s = floor(alpha / q)."""
    return alpha // q


def qgram_hash(u: Sequence[int], alpha: int, s: int) -> int:
    """Equation (3): h(empty) = 0, h(u) = h(u[1..]) * 2^s + u[0], all mod 2^alpha.

    Unbounded Python integers, reduced once at the end, which is the same
    residue as reducing at every step.
    """
    v = 0
    for c in reversed(list(u)):  # innermost term of the recursion first
        v = v * (1 << s) + int(c)
    return v % (1 << alpha)


def link_bit(v: int, w: int) -> int:
    """Equation (5): lambda(v) = 2^(v mod w)."""
    return 1 << (v % w)


# ---------------------------------------------------------------------------
# The word vector F and H_v (Sections 3.1 and 3.4)
# ---------------------------------------------------------------------------

def adjacent_pairs(m: int, q: int) -> List[Tuple[int, int]]:
    """Start positions (i, i+q) of every pair u1 = x[i..i+q-1], u2 = x[i+q..i+2q-1],
    0 <= i <= m - 2q: the pairs that equation (1) links (Section 3.1)."""
    return [(i, i + q) for i in range(0, m - 2 * q + 1)]


def first_qgram_starts(m: int, q: int) -> List[int]:
    """Starts of the q-grams that lie in the first q positions and have no
    q-gram to their left (equation (2)); only those that exist in x."""
    return list(range(0, min(q, m - q + 1)))


def link_table(x: bytes, q: int, alpha: int, w: int):
    """F, s, F' (the mask 2^alpha - 1) and H_v for pattern x.

    F has 2^alpha words of w bits, returned as Python ints in a list.
    Links first (equation (1), an OR, so their order does not matter), then
    the first-q marks (equation (2)) on words that are still zero.
    """
    m = len(x)
    if not (1 <= q <= m):
        raise ValueError("need 1 <= q <= m")
    s = shift_s(alpha, q)
    mask = (1 << alpha) - 1
    F = [0] * (1 << alpha)
    h = lambda i: qgram_hash(x[i:i + q], alpha, s)
    for i1, i2 in adjacent_pairs(m, q):
        F[h(i2)] |= link_bit(h(i1), w)
    for i in first_qgram_starts(m, q):
        if F[h(i)] == 0:
            F[h(i)] = 1
    return F, s, mask, chain_head_hash(x, q, alpha)


def chain_end_qgram_starts(m: int, q: int) -> List[int]:
    """Starts of the q-grams of the chain that ends at position m-1, from the
    end of the pattern backwards (Section 3.1 defines chains by their end)."""
    starts = []
    end = m - 1
    while end - q + 1 >= 0:
        starts.append(end - q + 1)
        end -= q
    return starts


def chain_head_hash(x: bytes, q: int, alpha: int) -> int:
    """H_v: hash of the first (leftmost) q-gram of the chain ending at m-1."""
    head = chain_end_qgram_starts(len(x), q)[-1]
    return qgram_hash(x[head:head + q], alpha, shift_s(alpha, q))


# ---------------------------------------------------------------------------
# Sequential searching phase (Section 3.3), tiny inputs only
# ---------------------------------------------------------------------------

def hc_scan(x, y, q: int, alpha: int, w: int, line: int = 128, max_hashes: int = 0):
    """(occurrences, distinct line-byte blocks of y read, covered) of the
    searching phase over y, by the C implementation in hc_seq.c. With
    max_hashes > 0 the scan stops after hashing that many q-grams; every
    window ending before `covered` was decided (covered = len(y) otherwise)."""
    xa, ya = _as_u8(x), _as_u8(y)
    occ, lines, cov = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    rc = _load().oracle_hc_scan(xa.ctypes.data, int(xa.size), ya.ctypes.data if ya.size else None,
                                int(ya.size), int(q), int(alpha), int(w), int(line), int(max_hashes),
                                ctypes.byref(occ), ctypes.byref(lines), ctypes.byref(cov))
    if rc != 0:
        raise ValueError("oracle_hc_scan: bad arguments")
    return occ.value, lines.value, cov.value


def hc_search_sequential(x: bytes, y: bytes, q: int, alpha: int, w: int,
                         table=None, touched=None) -> List[int]:
    """Slide a window of length m; read q-grams backwards from its end.

    * The q-gram ending at the window end is hashed; an empty word means no
      q-gram of x hashes there, and the window end moves on by m - q + 1.
    * Otherwise the q-grams ending q, 2q, ... positions earlier are hashed in
      turn while they stay inside the window; each must have its link bit set
      in the word of the q-gram after it. When one does not, the window end
      moves to (end of that q-gram) + m - q + 1.
    * When every q-gram in the window links, the window is a candidate: if the
      last hash read equals H_v and the window equals x, its start is
      reported; the window then advances by one position.

    When ``touched`` is a set, the positions of y the search reads (every
    hashed q-gram, every compared window) are added to it.
    """
    m, n = len(x), len(y)
    F, s, mask, Hv = link_table(x, q, alpha, w)

    def H(e):  # q-gram ending at e
        if touched is not None:
            touched.update(range(e - q + 1, e + 1))
        return qgram_hash(y[e - q + 1:e + 1], alpha, s)

    out = []
    J = m - 1                          # window end
    while J < n:
        v = H(J)
        z = F[v]
        if z == 0:
            J += m - q + 1
            continue
        e = J                          # end of the q-gram just read
        linked = True
        while e - q >= J - m + q:      # a whole q-gram still fits before e
            e -= q
            v = H(e)
            if z & link_bit(v, w) == 0:
                linked = False
                break
            z = F[v]
        if linked:
            start = J - m + 1
            if v == Hv:
                if touched is not None:
                    touched.update(range(start, start + m))
                if y[start:start + m] == x:
                    out.append(start)
            J += 1
        else:
            J = e + m - q + 1
    return out
