"""Device-side preprocessing (hc_preprocess_many through the C ABI): every
table equals the host preprocessing's bit for bit (the host tables are pinned
to the oracle's definition of F by the CPU tests), and s, mask and H_v
agree, for random patterns, every word width and small and large tables."""
import random
import sys

import numpy as np
import pytest

from oracle import hc_oracle as O
from paper_2310_15711_amd import binding as B

pytestmark = pytest.mark.gpu


def announce(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def packed_host(p, stride):
    info = B.hc_pattern_info(p)
    w = info["w"]
    words = info["F"].astype(np.uint64)
    raw = words.astype({8: np.uint8, 16: np.uint16, 32: np.uint32, 64: np.uint64}[w]).tobytes()
    return raw + bytes(stride - len(raw)), info


@pytest.mark.parametrize("alpha,w", [(8, 8), (11, 16), (12, 32), (13, 64), (4, 8), (14, 32)])
def test_device_tables_equal_host(alpha, w):
    import torch

    g = random.Random(alpha * 100 + w)
    pats = []
    for _ in range(60):
        sigma = g.choice([2, 4, 20, 256])
        m = g.choice([g.randint(1, 12), g.randint(12, 300), g.randint(300, 4096)])
        pats.append(bytes(g.randrange(sigma) for _ in range(m)))
    for q in (0, 1, 3, 8):
        stride = max(16, ((1 << alpha) * w // 8 + 15) // 16 * 16)
        d_F = torch.zeros(len(pats) * stride, dtype=torch.uint8, device="cuda:0")
        announce("device preprocessing", alpha, w, q)
        used, info = B.hc_preprocess_many(pats, d_F, stride, params=(q, alpha, w))
        F = d_F.cpu().numpy()
        for i, x in enumerate(pats):
            qq, aa, ww = used[i]
            assert (aa, ww) == (alpha, w) and 1 <= qq <= min(len(x), 8)
            if q:
                assert qq == min(q, len(x))
            p = B.hc_preprocess(x, (qq, alpha, w))
            want, hinfo = packed_host(p, stride)
            assert F[i * stride:(i + 1) * stride].tobytes() == want, (i, len(x), qq)
            assert info[i] == (hinfo["s"], hinfo["mask"], hinfo["hv"])


def test_device_tables_match_oracle_definition():
    import torch

    pats = [b"acgacgacg", b"GCAGAGAG", bytes(range(200, 256)) * 3, b"a", b"ab" * 50]
    alpha, w, stride = 10, 32, 4096
    d_F = torch.zeros(len(pats) * stride, dtype=torch.uint8, device="cuda:0")
    used, info = B.hc_preprocess_many(pats, d_F, stride, params=(3, alpha, w))
    F = d_F.cpu().numpy()
    for i, x in enumerate(pats):
        q = used[i][0]
        want, s, mask, hv = O.link_table(x, q, alpha, w)
        got = np.frombuffer(F[i * stride:i * stride + (1 << alpha) * 4].tobytes(), dtype=np.uint32)
        assert got.tolist() == [int(v) for v in want], i
        assert info[i] == (s, mask, hv)


def test_rejects_bad_arguments():
    import torch

    d_F = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda:0")
    for pats, stride, params in (([b""], 4096, None), ([b"a" * 4097], 4096, None),
                                 ([b"abc"], 15, (0, 4, 8)), ([b"abc"], 16, (0, 12, 32)),
                                 ([b"abc"], 16, (0, 4, 12))):
        with pytest.raises(B.HCError):
            B.hc_preprocess_many(pats, d_F, stride, params=params)
