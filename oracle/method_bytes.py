"""Writes profiles/hc_method_bytes.json and .md: the share of a text's
128-byte lines that HC's searching phase reads, per (alphabet, m, q, alpha,
w), measured by the oracle's sequential scan (hc_seq.c) over the benchmark's
own texts and patterns.

TEST INFRASTRUCTURE (like the rest of oracle/): run by hand; the benchmark
only reads the table it writes, to price each launch on the bytes the method
needs rather than on the whole text.

For m <= 32 every line is read (the longest shift, m - q + 1, is below the
line size), so the table starts at m = 64.

Usage: python oracle/method_bytes.py [--patterns 4] [--jobs 8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import hc_oracle as O  # noqa: E402
from paper_2310_15711_amd import workloads as W  # noqa: E402

LINE = 128
LENGTHS = (64, 128, 256, 512, 1024)
SHAPES = ((8, 8), (10, 16), (11, 16), (12, 16), (12, 32))   # the tuner's (alpha, w)
TEXTS = {4: "iid ACGT", 20: "iid 20 amino-acid letters", 64: "iid base64", 27: "order-2 Markov, 27 symbols"}

_text = {}


def _get_text(sigma):
    if sigma not in _text:
        _text[sigma] = W.markov_text(256 << 20) if sigma == 27 else W.single_text(sigma)
    return _text[sigma]


def _cell(args):
    sigma, m, n_pat, budget = args
    y = _get_text(sigma)
    pats = (W.markov_patterns(y, m, n_pat) if sigma == 27 else W.single_patterns(y, sigma, m, n_pat))
    out = {}
    for q in range(1, min(m, 8) + 1):
        for a, w in SHAPES:
            fr = []
            for _, x in pats:
                # a budget of hashed q-grams keeps degenerate choices (q = 1
                # over 4 symbols walks whole windows) from running for hours;
                # the share is taken over the part of the text decided
                _, lines, covered = O.hc_scan(x, y, q, a, w, LINE, budget)
                fr.append(lines / max(1, -(-covered // LINE)))
            out[f"{q},{a},{w}"] = round(float(np.mean(fr)), 5)
    return sigma, m, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--patterns", type=int, default=4)
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--budget", type=int, default=4_000_000, help="q-grams hashed per scan at most")
    ap.add_argument("--md-only", action="store_true",
                    help="rewrite the markdown summary from the stored JSON table (after the tuned choices "
                         "changed) without scanning again")
    args = ap.parse_args()
    json_path = os.path.join(ROOT, "profiles", "hc_method_bytes.json")
    if args.md_only:
        doc = json.load(open(json_path))
        table = doc["read_fraction"]
        args.patterns = doc["patterns_per_cell"]
        args.budget = doc.get("budget", args.budget)
    else:
        O.build()
        cells = [(s, m, args.patterns, args.budget) for s in (4, 20, 64, 27) for m in LENGTHS]
        table = {}
        with ProcessPoolExecutor(max_workers=args.jobs) as ex:
            for sigma, m, out in ex.map(_cell, cells):
                table.setdefault(str(sigma), {})[str(m)] = out
                print(f"sigma {sigma} m {m}: {min(out.values()):.3f}..{max(out.values()):.3f}", flush=True)
        doc = {"line_bytes": LINE, "text_bytes": 256 << 20, "patterns_per_cell": args.patterns,
               "budget": args.budget, "read_fraction": table,
               "note": "mean share of the text's 128-byte lines read by the sequential searching phase "
                       "(oracle/hc_seq.c) for the benchmark's first patterns of each (alphabet, m); keys "
                       "'q,alpha,w'; m <= 32 reads every line"}
        with open(json_path, "w") as f:
            json.dump(doc, f, indent=1)
    tuned_path = os.path.join(ROOT, "profiles", "hc_search_single_pattern_tuned.json")
    tuned = json.load(open(tuned_path)) if os.path.exists(tuned_path) else {}
    lines = ["# Text bytes the HC searching phase reads (method bytes)", "",
             "Share of a 256 MiB text's 128-byte lines read by the sequential searching phase",
             "(`oracle/hc_seq.c`: every hashed q-gram and every compared window), mean over the",
             f"benchmark's first {args.patterns} patterns of each cell. Written by",
             "`python oracle/method_bytes.py`; the full table (every q and the tuner's (alpha, w)) is",
             "`hc_method_bytes.json`. m <= 32: every line. Each scan stops after hashing "
             f"{args.budget} q-grams; the share is over the part of the text it decided.", "",
             "| text | m | min over (q, alpha, w) | max | at the stored tuned choice |", "|---|---|---|---|---|"]
    for s in ("4", "20", "64", "27"):
        for m in map(str, LENGTHS):
            v = table[s][m]
            t = tuned.get(s, {}).get(m)
            key = ",".join(map(str, t["params"])) if t else None
            at = f"{v[key]:.4f} ({key})" if key in v else "-"
            lines.append(f"| {TEXTS[int(s)]} | {m} | {min(v.values()):.4f} | {max(v.values()):.4f} | {at} |")
    with open(os.path.join(ROOT, "profiles", "hc_method_bytes.md"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
