"""GPU parity of the single-pattern search with the tuned launch choices.

- The full 256 MiB texts over 4, 20 and 64 symbols, each (sigma, m) cell run
  with the (q, alpha, w, segment, schedule, variant) tuple the tuner chose
  for it in the stored profile (profiles/hc_search_single_pattern_tuned.json),
  complete lists compared with the oracle's brute force.
- The 256 MiB order-2 Markov text, tuned inside the test (hc_autotune on that
  text), each length run with the tuple it chose.
- Every candidate the tuner can choose (q, alpha, w, schedule, segment and,
  for m >= 256, the sparse variant with 1, 2, 4 or 8 shifts per lane) on
  12 MiB texts, so that whatever a tuning run picks has been compared with
  the oracle over hundreds of tiles."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import hc_oracle as O
from paper_2310_15711_amd import binding as B
from paper_2310_15711_amd import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNED = os.path.join(ROOT, "profiles", "hc_search_single_pattern_tuned.json")


def announce(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def search(x, yd, params, launch, want_size):
    import torch

    p = B.hc_preprocess(x, params)
    out = torch.empty(want_size + 16, dtype=torch.int64, device=yd.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=yd.device)
    B.hc_search_async(p, yd, out, cnt, launch=launch)
    torch.cuda.synchronize()
    c = int(cnt.item())
    return out[:min(c, want_size + 16)].cpu().numpy(), c


def load_tuned():
    with open(TUNED) as f:
        raw = json.load(f)
    return {int(s): {int(m): (tuple(r["params"]), tuple(r["launch"])) for m, r in d.items()}
            for s, d in raw.items()}


@pytest.mark.parametrize("sigma", [4, 20, 64])
def test_stored_tuned_choices_full_size(dev, sigma):
    import torch

    tuned = load_tuned()[sigma]
    y = W.single_text(sigma)
    yd = torch.from_numpy(y).to(dev)
    for m in W.SINGLE_LENGTHS:
        params, launch = tuned[m]
        for off, x in W.single_patterns(y, sigma, m, count=2):
            announce("tuned full", sigma, m, off, params, launch)
            want = O.occurrences(x, y)
            got, c = search(x, yd, params, launch, int(want.size))
            assert c == want.size, (sigma, m, off, params, launch)
            assert np.array_equal(got, want), (sigma, m, off, params, launch)
    del yd
    torch.cuda.empty_cache()


def test_markov_tuned_full_size(dev):
    import torch

    y = W.markov_text(256 << 20)
    yd = torch.from_numpy(y).to(dev)
    announce("markov tune")
    choice = {r["m"]: r for r in B.hc_autotune(yd, list(W.MARKOV_LENGTHS), patterns=3)}
    B.hc_autotune_reset()
    for m in W.MARKOV_LENGTHS:
        params, launch = choice[m]["params"], choice[m]["launch"]
        for off, x in W.markov_patterns(y, m, count=2):
            announce("markov tuned full", m, off, params, launch)
            want = O.occurrences(x, y)
            got, c = search(x, yd, params, launch, int(want.size))
            assert c == want.size and np.array_equal(got, want), (m, off, params, launch)
    del yd
    torch.cuda.empty_cache()


SHAPES = [(8, 8), (10, 16), (11, 16), (12, 16), (12, 32)]


def tuner_candidates(m):
    """Every (params, launch) the tuner can return for length m."""
    out = []
    for q in range(1, min(8, m) + 1):
        for a, w in SHAPES:
            scheds = [B.HC_SCHED_SEGMENT]
            if m < 2 * q or (q <= 4 and m // q - 1 <= 3):
                scheds.append(B.HC_SCHED_DENSE)
            for sc in scheds:
                for seg in (48, 64, 80, 100):
                    out.append(((q, a, w), (seg, sc, B.HC_VARIANT_HC, 0)))
            if m >= 256 and q >= 3:   # 1, 2, 4 or 8 shifts per lane, at most 4096 starts
                for k in (1, 2, 4, 8):
                    seg = min(k * (m - q + 1), 4096)
                    out.append(((q, a, w), (seg, B.HC_SCHED_SEGMENT, B.HC_VARIANT_SPARSE, 0)))
    if m == 2:   # one-to-one hash on the window, no comparison with x
        for seg in (48, 64, 80, 100):
            out.append(((2, 16, 8), (seg, B.HC_SCHED_DENSE, B.HC_VARIANT_HC, 0)))
    return out


@pytest.mark.parametrize("sigma", [4, 20, 64])
def test_every_tuner_candidate(dev, sigma):
    import torch

    n = (12 << 20) + 13
    y = W.iid_text(n, W.ALPHABETS[sigma], W.rng(W.TEST_CFG, 0, sigma))
    yd = torch.from_numpy(y).to(dev)
    g = np.random.default_rng([231015711, 8, sigma])
    for m in W.SINGLE_LENGTHS:
        t = int(g.integers(0, n - m + 1))
        x = y[t:t + m].tobytes()
        want = O.occurrences(x, y)
        wd = torch.from_numpy(want).to(dev)
        out = torch.empty(want.size + 16, dtype=torch.int64, device=dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        cands = tuner_candidates(m)
        announce("tuner candidates", sigma, m, len(cands), int(want.size))
        for params, launch in cands:
            p = B.hc_preprocess(x, params)
            B.hc_search_async(p, yd, out, cnt, launch=launch)
            c = int(cnt.item())
            assert c == want.size, (sigma, m, params, launch, c, want.size)
            assert torch.equal(out[:c], wd), (sigma, m, params, launch)
    del yd
    torch.cuda.empty_cache()
