"""C ABI checks that need no GPU: the library loads, exports what
include/hc.h declares, and its host preprocessing builds exactly the
oracle's F, s, mask and H_v."""
import os
import random
import re

import numpy as np
import pytest

from conftest import ROOT
from oracle import hc_oracle as O
from paper_2310_15711_amd import binding as B


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(hc_[a-z_]+)\s*\(", text))


def test_exports_every_declared_symbol():
    import ctypes

    syms = declared_symbols()
    assert {"hc_preprocess", "hc_search", "hc_search_batched", "hc_serve_submit",
            "hc_serve_poll"} <= syms
    L = ctypes.CDLL(B.LIB_PATH)
    for s in sorted(syms):
        assert hasattr(L, s), s
    assert syms == set(B.EXPORTED)
    B.lib()


def test_strerror_names_every_status():
    for st in (0, -1, -2, -3, -4, -5):
        assert B.strerror(st) and B.strerror(st) != "unknown status"


def check_against_oracle(x, q, alpha, w):
    p = B.hc_preprocess(x, (q, alpha, w))
    info = B.hc_pattern_info(p)
    F, s, mask, hv = O.link_table(x, q, alpha, w)
    assert (info["q"], info["alpha"], info["w"]) == (q, alpha, w)
    assert info["s"] == s and info["mask"] == mask and info["hv"] == hv
    assert info["m"] == len(x)
    assert info["F"].tolist() == F, (x, q, alpha, w)


def test_link_table_matches_oracle_golden_cases():
    from conftest import golden_lines

    for r in golden_lines("link_table_cases.txt"):
        x = bytes.fromhex(r[1])
        check_against_oracle(x, int(r[2]), int(r[3]), int(r[4]))


def test_link_table_matches_oracle_random():
    g = random.Random(3)
    for _ in range(400):
        m = g.randint(1, 300)
        q = g.randint(1, min(m, 8))
        w = g.choice([8, 16, 32, 64])
        alpha = g.randint(1, {8: 16, 16: 15, 32: 14, 64: 13}[w])
        sigma = g.choice([2, 4, 20, 64, 256])
        x = bytes(g.randrange(256 - sigma, 256) if g.random() < 0.3 else g.randrange(sigma)
                  for _ in range(m))
        check_against_oracle(x, q, alpha, w)


def test_link_table_long_patterns():
    g = np.random.default_rng(1)
    for m in (1024, 2048, 4096):
        x = g.integers(0, 4, size=m, dtype=np.uint8).tobytes()
        check_against_oracle(x, 8, 12, 32)
        check_against_oracle(x, 3, 11, 64)


def test_defaults_are_valid_and_q_within_m():
    for m in (1, 2, 3, 4, 5, 8, 9, 16, 17, 256, 257, 4096):
        p = B.hc_preprocess(b"a" * m)
        info = B.hc_pattern_info(p)
        assert 1 <= info["q"] <= min(m, 8)
        assert info["w"] in (8, 16, 32, 64)
        assert 8 <= info["alpha"] <= 16


@pytest.mark.parametrize("x,params", [
    (b"", None),                  # m = 0
    (b"a" * 4097, None),          # m beyond the on-chip limit
    (b"abc", (4, 8, 32)),         # q > m
    (b"a" * 20, (9, 8, 32)),      # q > 8
    (b"abcd", (2, 8, 12)),        # w not a power-of-two word size
    (b"abcd", (2, 14, 64)),       # F beyond 64 KiB
    (b"abcd", (2, 17, 8)),        # alpha beyond the limit
    (b"abcd", (-1, 8, 32)),       # negative field
])
def test_preprocess_rejects_invalid(x, params):
    with pytest.raises(B.HCError) as e:
        B.hc_preprocess(x, params)
    assert e.value.status == B.HC_EINVAL


def test_null_arguments_are_rejected():
    L = B.lib()
    import ctypes

    out = ctypes.c_void_p()
    assert L.hc_preprocess(None, 4, None, ctypes.byref(out)) == B.HC_EINVAL
    assert L.hc_preprocess(b"abcd", 4, None, None) == B.HC_EINVAL
    assert L.hc_pattern_info(None, None, None, None, None, None, None, None) == B.HC_EINVAL
    cnt = ctypes.c_int64()
    assert L.hc_search(None, None, 0, None, 0, ctypes.byref(cnt), None) == B.HC_EINVAL
    L.hc_pattern_free(None)
    # argument checks that come before any device call
    ms = (ctypes.c_int64 * 1)(8)
    assert L.hc_autotune(None, 1 << 20, ms, 1, 3, None, None) == B.HC_EINVAL
    assert L.hc_autotune(ctypes.c_void_p(16), 1 << 20, ms, 0, 3, None, None) == B.HC_EINVAL
    assert L.hc_autotune(ctypes.c_void_p(16), 1 << 20, ms, 1, 0, None, None) == B.HC_EINVAL
    big = (ctypes.c_int64 * 1)(4097)
    assert L.hc_autotune(ctypes.c_void_p(16), 1 << 20, big, 1, 3, None, None) == B.HC_EINVAL
    assert L.hc_serve_next_done(None, None, 0) == B.HC_EINVAL
    assert L.hc_serve_create(None, None, 0, 1 << 20, None, ctypes.byref(out)) == B.HC_EINVAL
    assert L.hc_serve_submit(None, 0, b"abc", 3, None) == B.HC_EINVAL
    assert L.hc_serve_stats(None, None, None, None, None) == B.HC_EINVAL
    assert L.hc_serve_destroy(None) == B.HC_EINVAL
    assert L.hc_batch_plan_create(None, None, ctypes.byref(out)) == B.HC_EINVAL
    total = ctypes.c_int64()
    assert L.hc_search_batched(None, None, None, 0, None, ctypes.byref(total), None) == B.HC_EINVAL
    assert L.hc_batch_plan_run(None, None, 0, None, ctypes.byref(total), None) == B.HC_EINVAL
    L.hc_batch_plan_free(None)
    assert L.hc_preprocess_many(None, None, 1, None, None, 4096, None, None, None) == B.HC_EINVAL
    assert L.hc_preprocess_many(None, None, 0, None, None, 4096, None, None, None) == B.HC_OK
    L.hc_autotune_reset()


def test_bucket_defaults_after_reset():
    """With no tuned entries the priors apply; q never exceeds m."""
    B.hc_autotune_reset()
    for m in (1, 2, 3, 5, 17, 100, 1000, 4096):
        p = B.hc_preprocess(bytes((7 * i) % 256 for i in range(m)))
        info = B.hc_pattern_info(p)
        assert 1 <= info["q"] <= min(m, 8)


def test_short_patterns_default_to_no_links():
    """Untuned, every m <= 8 gets the smallest q with m < 2q (no links: the
    dense schedule's single-hash test, or its direct comparison of windows
    of 4 to 8 bytes), with s = floor(alpha / q) >= 1."""
    B.hc_autotune_reset()
    for m in range(1, 9):
        for x in (b"ACGTACGT"[:m], bytes(range(40, 40 + m))):
            info = B.hc_pattern_info(B.hc_preprocess(x))
            q = info["q"]
            assert m < 2 * q and (q == 1 or m >= 2 * (q - 1)), (m, q)
            assert info["s"] == info["alpha"] // q >= 1
