"""hc_search_async_noalloc (per-tile results in the library's fixed device
array, no allocation) against hc_search_async (the per-stream workspace):
the same lists, element by element, on two calls in a row with the second
on a smaller text, for the streaming, dense and sparse kernels; the cases it
must refuse without launching anything."""
import sys

import numpy as np
import pytest

from oracle import hc_oracle as O
from paper_2310_15711_amd import binding as B
from paper_2310_15711_amd import workloads as W

pytestmark = pytest.mark.gpu

NOALLOC_BYTES = 64 << 20   # the fixed array (hc.h)


def announce(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def scratch_bytes(n_tiles, tile):
    """Bytes of per-tile results: counts, 128 slots per tile, the bitmaps,
    the first two parts rounded up to 256 bytes."""
    t = max(n_tiles, 1)
    up = lambda v: (v + 255) // 256 * 256
    return up(4 * t) + up(512 * t) + t * (tile // 32) * 4


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def run_both(p, yd, launch, cap):
    import torch

    out_a = torch.full((cap,), -1, dtype=torch.int64, device=yd.device)
    out_b = torch.full((cap,), -2, dtype=torch.int64, device=yd.device)
    ca = torch.zeros(1, dtype=torch.int64, device=yd.device)
    cb = torch.zeros(1, dtype=torch.int64, device=yd.device)
    B.hc_search_async(p, yd, out_a, ca, launch=launch)
    st = B.hc_search_async_noalloc(p, yd, out_b, cb, launch=launch)
    torch.cuda.synchronize()
    assert st == B.HC_OK
    na, nb = int(ca.item()), int(cb.item())
    return na, nb, out_a[:min(na, cap)].cpu().numpy(), out_b[:min(nb, cap)].cpu().numpy()


@pytest.mark.parametrize("sigma,m,launch", [
    (4, 32, None),                                  # tuned-or-prior streaming kernel
    (4, 3, (64, B.HC_SCHED_DENSE, 0, 0)),           # dense kernel, many occurrences
    (20, 700, (1024, 0, B.HC_VARIANT_SPARSE, 0)),   # sparse kernel
    (64, 8, (36, B.HC_SCHED_SEGMENT, 0, 0)),        # small tiles
])
def test_noalloc_equals_workspace_path(dev, sigma, m, launch):
    import torch

    y = W.iid_text((96 << 20) + 777, W.ALPHABETS[sigma], W.rng(W.TEST_CFG, 0, 300 + sigma))
    yd = torch.from_numpy(y).to(dev)
    g = np.random.default_rng([231015711, 11, sigma, m])
    t = int(g.integers(0, y.size - m))
    x = y[t:t + m].tobytes()
    p = B.hc_preprocess(x)
    # two calls in a row, the second on a smaller text (a prefix)
    for n in (y.size, 3_000_001):
        announce("noalloc", sigma, m, launch, n)
        want = O.occurrences(x, y[:n])
        na, nb, a, b = run_both(p, yd[:n], launch, int(want.size) + 8)
        assert na == nb == want.size, (na, nb, want.size)
        assert np.array_equal(a, b) and np.array_equal(b, want)
    del yd
    torch.cuda.empty_cache()


def test_noalloc_refusals(dev):
    import torch

    y = torch.zeros(1 << 20, dtype=torch.uint8, device=dev)
    out = torch.empty(16, dtype=torch.int64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    # a pattern without a device copy: refused (uploading would allocate)
    fresh = B.hc_preprocess(b"abcdef")
    assert B.hc_search_async_noalloc(fresh, y, out, cnt) == B.HC_EINVAL
    # a text whose per-tile results exceed the fixed array: refused before
    # any launch (tiles of 2048 starts over 256 MiB need about 100 MiB)
    big = torch.zeros(256 << 20, dtype=torch.uint8, device=dev)
    p = B.hc_preprocess(b"abcdefgh", (4, 10, 16))
    B.hc_search_async(p, y, out, cnt, launch=(8, 1, 0, 0))   # makes the pattern resident
    torch.cuda.synchronize()
    n_tiles = -(-(big.numel() - 8 + 1) // 2048)
    assert scratch_bytes(n_tiles, 2048) > NOALLOC_BYTES
    assert B.hc_search_async_noalloc(p, big, out, cnt, launch=(8, 1, 0, 0)) == B.HC_EINVAL
    # within the limit on the same text with large tiles: accepted and exact
    n_tiles = -(-(big.numel() - 8 + 1) // 25600)
    assert scratch_bytes(n_tiles, 25600) <= NOALLOC_BYTES
    cnt.zero_()
    assert B.hc_search_async_noalloc(p, big, out, cnt, launch=(100, 1, 0, 0)) == B.HC_OK
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    del big
    torch.cuda.empty_cache()
