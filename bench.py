"""Benchmark of the HC searching phase on one MI355X.

Default workload (single pattern per launch): three 256 MiB iid texts over
sigma = 4, 20, 64 symbols; for each, 100 patterns of each length
m in {2, 4, ..., 1024} copied from the text at seeded offsets; one step
searches all 3000 (pattern, text) pairs, one launch each, with the texts
resident in HBM. value = text bytes scanned per second over the timed steps.

Prints one JSON line (rank 0). Extra objects:
  roofline      the search kernel's algorithmic bytes per launch over its
                average launch time (HIP events around each launch on the
                launch stream), against the 8 TB/s HBM peak;
  cpu_baseline  the oracle (C brute force, all host cores) on a bounded
                sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="single",
                    choices=["single", "markov", "planted", "batched", "served"])
    ap.add_argument("--no-extras", action="store_true",
                    help="single workload: leave out the batched and served summaries")
    ap.add_argument("--serve-rates", default="1000,3000,10000,30000,100000")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-tune-requests", type=int, default=1000,
                    help="served workload: sample requests hc_batch_autotune times the batch knobs on")
    ap.add_argument("--serve-threads", type=int, default=4, help="native submitter threads")
    ap.add_argument("--serve-text-mib", type=int, default=128)
    ap.add_argument("--serve-budget-mib", type=int, default=2048)
    ap.add_argument("--serve-check", type=int, default=1000,
                    help="served requests per rate compared with hc_search alone")
    ap.add_argument("--batch-texts", type=int, default=64)
    ap.add_argument("--batch-patterns", type=int, default=4096)
    ap.add_argument("--batch-params", default=None, help="q,alpha,w for the batch plan (0 = library choice)")
    ap.add_argument("--no-batch-tune", action="store_true",
                    help="batched and served workloads: skip hc_batch_autotune")
    ap.add_argument("--batch-tune-pairs", type=int, default=22000,
                    help="batched workload: pairs sampled by hc_batch_autotune")
    ap.add_argument("--batch-oracle-pairs", type=int, default=1000,
                    help="batched workload: seeded pairs compared with the oracle")
    ap.add_argument("--serve-oracle", type=int, default=1000,
                    help="served requests (over all rates) compared with the oracle")
    ap.add_argument("--no-per-pattern", action="store_true",
                    help="batched workload: skip the per-pattern launch baseline")
    ap.add_argument("--per-length", type=int, default=100, help="patterns per (sigma, m)")
    ap.add_argument("--sigmas", default="4,20,64")
    ap.add_argument("--lengths", default=None, help="comma list of m (default: the workload's)")
    ap.add_argument("--text-mib", type=int, default=256)
    ap.add_argument("--segment", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--params", default=None, help="q,alpha,w for every pattern")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip hc_autotune (built-in priors choose q, alpha, w and the launch shape)")
    ap.add_argument("--tune-patterns", type=int, default=5)
    ap.add_argument("--save-tuned", default=None, help="write the autotuned choices to this JSON file")
    ap.add_argument("--load-tuned", default=None,
                    help="use the choices in this JSON file instead of tuning (profiling runs)")
    ap.add_argument("--lds-dir", default=None, help="with --summarize: rocprofv3 LDS counter pass")
    ap.add_argument("--summarize-stats", nargs=3, metavar=("STATS_DIR", "NAME", "TITLE"),
                    help="write profiles/NAME.md: the kernel table of a rocprofv3 --stats run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-patterns", type=int, default=12,
                    help="oracle sample: patterns per (sigma, m)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--detail", action="store_true", help="print per-(sigma, m) figures to stderr")
    ap.add_argument("--write-cells", default=None, help="write the per-(sigma, m) markdown table here")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run only a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--summarize", nargs=4, metavar=("STATS_DIR", "FETCH_DIR", "WRITE_DIR", "CALIB_PREFIX"),
                    help="turn rocprofv3 outputs into profiles/ summaries and traffic.json")
    ap.add_argument("--summary-cmd", default="", help="command lines quoted in the summary")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("PMC_DIR", "NAME", "TITLE"),
                    help="write profiles/NAME.md: per-instance SQ counter means of a rocprofv3 --pmc run")
    ap.add_argument("--per-unit", type=float, default=None,
                    help="with --summarize-counters: units (e.g. windows) per dispatch")
    ap.add_argument("--unit", default="window", help="with --summarize-counters: the unit's name")
    return ap.parse_args()


def kernel_source_hash():
    """Hash of the search kernel's sources: traffic figures taken with other
    sources are not reported."""
    import hashlib

    h = hashlib.sha256()
    for f in ("hc_search.hip", "hc_device.h"):
        with open(os.path.join(ROOT, "paper_2310_15711_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def calib_copy():
    """A plain device copy of 256 MiB (reads 256 MiB, writes 256 MiB): the
    FETCH_SIZE / WRITE_SIZE it reports give the scale of those counters."""
    import torch

    n = 256 << 20
    # four sources, copied in rotation: 1 GiB does not fit the 256 MB
    # last-level cache, so each copy reads its source from HBM
    srcs = [torch.empty(n, dtype=torch.uint8, device="cuda").fill_(i) for i in range(4)]
    b = torch.empty_like(srcs[0])
    torch.cuda.synchronize()
    for i in range(8):
        b.copy_(srcs[i % 4])
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": n, "copies": 8}), flush=True)


def _read_csv(path):
    import csv

    with open(path) as f:
        return list(csv.DictReader(f))


def _find(d, suffix):
    for root, _, files in os.walk(d):
        for fn in files:
            if fn.endswith(suffix):
                return os.path.join(root, fn)
    raise FileNotFoundError(f"{suffix} under {d}")


def _counter_per_dispatch(d, counter, name_part):
    """Mean of a counter over the dispatches of kernels whose name contains
    name_part, summed per dispatch (rocprofv3 lists one row per dispatch)."""
    rows = _read_csv(_find(d, "counter_collection.csv"))
    per = {}
    for r in rows:
        if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]:
            per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return (sum(per.values()) / len(per)) if per else None, len(per)


def _counter_sum(d, counter, name_parts):
    """Sum of a counter over the dispatches of kernels whose name contains one
    of name_parts, and the number of those dispatches."""
    rows = _read_csv(_find(d, "counter_collection.csv"))
    per = {}
    for r in rows:
        if r["Counter_Name"] == counter and any(p in r["Kernel_Name"] for p in name_parts):
            per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return sum(per.values()), len(per)


# the first kernel of a single-pattern search call (streaming or sparse);
# hc_emit_kernel follows each
SEARCH_KERNELS = ("hc_search_kernel", "hc_sparse_kernel")


def summarize_stats(stats_dir, name, title, cmd):
    """Kernel table of one rocprofv3 --kernel-trace --stats run."""
    stats = _read_csv(_find(stats_dir, "kernel_stats.csv"))
    lines = [f"# rocprofv3 kernel statistics: {title}", "", "Command(s):", "", "```", cmd.strip(), "```", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |",
             "|---|---|---|---|---|---|"]
    for r in stats:
        short = r["Name"].split("(")[0].replace("void ", "")[:90]
        lines.append(f"| `{short}` | {r['Calls']} | {float(r['AverageNs'])/1e3:.2f} | "
                     f"{float(r['MinNs'])/1e3:.2f} | {float(r['MaxNs'])/1e3:.2f} | {float(r['Percentage']):.2f}% |")
    with open(os.path.join(ROOT, "profiles", f"{name}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize_lds(lds_dir, cmd):
    """LDS bank conflicts of the search kernels from a rocprofv3 --pmc pass."""
    rows = _read_csv(_find(lds_dir, "counter_collection.csv"))
    tot = {}
    for r in rows:
        if any(p in r["Kernel_Name"] for p in SEARCH_KERNELS):
            tot[r["Counter_Name"]] = tot.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    conf, active = tot.get("SQ_LDS_BANK_CONFLICT", 0.0), tot.get("SQ_ACTIVE_INST_LDS", 0.0)
    insts = tot.get("SQ_INSTS_LDS", 0.0)
    lines = ["# LDS bank conflicts of the single-pattern search kernels (rocprofv3 --pmc)", "",
             "Command(s):", "", "```", cmd.strip(), "```", "",
             "| counter (summed over hc_search_kernel and hc_sparse_kernel dispatches) | value |", "|---|---|"]
    lines += [f"| {k} | {v:.0f} |" for k, v in sorted(tot.items())]
    lines += ["", f"- Bank-conflict cycles per cycle of LDS instruction activity "
                  f"(SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS): {conf / active:.3f}" if active else "",
              f"- Bank-conflict cycles per LDS instruction (SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS): "
              f"{conf / insts:.3f}" if insts else "", ""]
    with open(os.path.join(ROOT, "profiles", "hc_search_single_pattern_lds.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    return {"lds_conflict_per_active_cycle": conf / active if active else None,
            "lds_conflict_cycles_per_inst": conf / insts if insts else None}


def summarize_counters(pmc_dir, name, title, cmd, per_unit=None, unit=""):
    """Per-kernel-instance means of an SQ counter pass (rocprofv3 --pmc), with
    the VALU time they imply (a wavefront VALU instruction takes 4 cycles on
    a 16-lane SIMD; 1024 SIMDs at 2.4 GHz) and LDS bank conflicts per LDS
    instruction; per_unit (e.g. windows per dispatch) adds per-unit columns."""
    rows = _read_csv(_find(pmc_dir, "counter_collection.csv"))
    per, disp = {}, {}
    for r in rows:
        k = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("hc::", "")
        if not k.startswith("hc_"):
            continue
        per.setdefault(k, {})
        per[k][r["Counter_Name"]] = per[k].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        disp.setdefault(k, set()).add(r["Dispatch_Id"])
    lines = [f"# rocprofv3 SQ counters per kernel instance: {title}", "", "Command(s):", "", "```",
             cmd.strip(), "```", "",
             "Means per dispatch. VALU time = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x 2.4 GHz)"
             + (f"; per {unit}: counter x 64 lanes / {per_unit:.4g} {unit}s per dispatch" if per_unit else "")
             + ".", "",
             "| kernel | dispatches | SQ_INSTS_VALU | VALU time (us) | SQ_INSTS_LDS | bank-conflict cycles / LDS instr "
             "| SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES |" + (f" VALU lane-ops / {unit} | LDS lane-ops / {unit} |" if per_unit else ""),
             "|---|---|---|---|---|---|---|" + ("---|---|" if per_unit else "")]
    for k, cs in sorted(per.items()):
        n = len(disp[k])
        c = {a: v / n for a, v in cs.items()}
        valu, lds = c.get("SQ_INSTS_VALU", 0.0), c.get("SQ_INSTS_LDS", 0.0)
        line = (f"| `{k}` | {n} | {valu:.4g} | {valu * 4 / 1024 / 2.4e3:.1f} | {lds:.4g} | "
                f"{c.get('SQ_LDS_BANK_CONFLICT', 0.0) / max(lds, 1.0):.2f} | "
                f"{c.get('SQ_WAIT_INST_LDS', 0.0) / max(c.get('SQ_WAVE_CYCLES', 1.0), 1.0):.3f} |")
        if per_unit:
            line += f" {valu * 64 / per_unit:.2f} | {lds * 64 / per_unit:.3f} |"
        lines.append(line)
    with open(os.path.join(ROOT, "profiles", f"{name}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize(stats_dir, fetch_dir, write_dir, calib_prefix, cmd):
    stats = _read_csv(_find(stats_dir, "kernel_stats.csv"))
    lines = ["# rocprofv3 kernel statistics: single-pattern HC search, sigma in {4,20,64}, "
             "m in {2..1024}, 256 MiB texts", "", "Command(s):", "", "```", cmd.strip(), "```", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |",
             "|---|---|---|---|---|---|"]
    avg = {}
    for r in stats:
        name = r["Name"]
        short = name.split("(")[0].replace("void ", "")[:90]
        a = float(r["AverageNs"]) / 1e3
        avg[short] = (int(r["Calls"]), a)
        lines.append(f"| `{short}` | {r['Calls']} | {a:.2f} | {float(r['MinNs'])/1e3:.2f} | "
                     f"{float(r['MaxNs'])/1e3:.2f} | {float(r['Percentage']):.2f}% |")
    search = [v for k, v in avg.items() if any(p in k for p in SEARCH_KERNELS)]
    emit = [v for k, v in avg.items() if "hc_emit_kernel" in k]
    if search and emit:
        calls = sum(c for c, _ in search)
        s_avg = sum(c * a for c, a in search) / calls
        e_avg = sum(c * a for c, a in emit) / sum(c for c, _ in emit)
        lines += ["", f"Search call = `hc_search_kernel` or `hc_sparse_kernel`, then `hc_emit_kernel`: "
                      f"average {s_avg:.2f} + {e_avg:.2f} = {s_avg + e_avg:.2f} us per call ({calls} calls)."]
    out = os.path.join(ROOT, "profiles", "hc_search_single_pattern_kernel_stats.md")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    # traffic: HBM bytes per search call, scaled by the copy kernel's counters
    # per call: the search (or sparse) kernel and the emit kernel that follows
    fs, nf = _counter_sum(fetch_dir, "FETCH_SIZE", SEARCH_KERNELS)
    fe, _ = _counter_sum(fetch_dir, "FETCH_SIZE", ("hc_emit_kernel",))
    ws, nw = _counter_sum(write_dir, "WRITE_SIZE", SEARCH_KERNELS)
    we, _ = _counter_sum(write_dir, "WRITE_SIZE", ("hc_emit_kernel",))
    fetch_s, fetch_e = fs / max(nf, 1), fe / max(nf, 1)
    write_s, write_e = ws / max(nw, 1), we / max(nw, 1)
    # the copy kernel only (the fills that create the sources read nothing)
    cf, _ = _counter_per_dispatch(calib_prefix + "_fetch", "FETCH_SIZE", "copyBuffer")
    cw, _ = _counter_per_dispatch(calib_prefix + "_write", "WRITE_SIZE", "copyBuffer")
    copy_bytes = 256 << 20
    kf = copy_bytes / (cf * 1024.0)    # bytes per counted KiB
    kw = copy_bytes / (cw * 1024.0)
    fetch = ((fetch_s or 0) + (fetch_e or 0)) * 1024.0 * kf
    write = ((write_s or 0) + (write_e or 0)) * 1024.0 * kw
    tj = {"workload": "single", "kernel_source": kernel_source_hash(),
          "bytes_per_launch": round(fetch + write),
          "fetch_bytes_per_launch": round(fetch), "write_bytes_per_launch": round(write),
          "dispatches": nf, "copy_fetch_kib": cf, "copy_write_kib": cw,
          "fetch_scale": kf, "write_scale": kw}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(tj, f, indent=1)
    lines = ["# HBM traffic of the single-pattern search call (rocprofv3 --pmc)", "",
             "Command(s):", "", "```", cmd.strip(), "```", "",
             f"- FETCH_SIZE per call (search + emit kernels): {(fetch_s or 0) + (fetch_e or 0):.0f} KiB "
             f"over {nf} calls; WRITE_SIZE per call: {(write_s or 0) + (write_e or 0):.0f} KiB.",
             f"- Calibration: a plain 256 MiB device copy (`__amd_rocclr_copyBuffer`, sources "
             f"rotated over 1 GiB) reads FETCH_SIZE = {cf:.0f} KiB and WRITE_SIZE = {cw:.0f} KiB "
             f"per dispatch (it moves 262144 KiB each way); scale factors {kf:.4f} and {kw:.4f}.",
             f"- Scaled HBM bytes per call: fetch {fetch/1e6:.1f} MB + write {write/1e6:.1f} MB = "
             f"{(fetch + write)/1e6:.1f} MB.",
             "- Workload: the bench's single-pattern mix (sigma 4/20/64, m 2..1024), 10 patterns "
             "per (sigma, m), with the tuned choices in `hc_search_single_pattern_tuned.json`.", ""]
    with open(os.path.join(ROOT, "profiles", "hc_search_single_pattern_traffic.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps(tj))


# int32 lane-ops per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def alu_roofline(ops, seconds, kernel):
    """Roofline of a run bound by integer ALU work: the searching phase's own
    operations (per pattern and text byte, (2q + 6) / (m - q + 1): one attempt
    per shift, each hashing q bytes and testing one word) over the run time."""
    achieved = ops / seconds / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2),
            "unit": "Tops/s", "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": None,
            "kernel": kernel, "ops_per_run": round(ops),
            "ops_model": "per (pattern, text byte): (2q + 6) / (m - q + 1) int32 lane-ops"}


def method_read_fractions(pats, infos):
    """Per launch: the share of the text's 128-byte lines the method reads
    (1 for m <= 32; else from profiles/hc_method_bytes.json; None when the
    table has no entry for that sigma, m, q, alpha, w)."""
    path = os.path.join(ROOT, "profiles", "hc_method_bytes.json")
    table = json.load(open(path))["read_fraction"] if os.path.exists(path) else {}
    out = []
    for (s, m, _, _), inf in zip(pats, infos):
        if m <= 32:
            out.append(1.0)
            continue
        out.append(table.get(str(s), {}).get(str(m), {}).get(f"{inf['q']},{inf['alpha']},{inf['w']}"))
    return out


def write_cells(args, cells, pats, launch_ms, texts, cnt, infos, read_frac, launches, workload):
    """Markdown table per (sigma, m): median call time, text GB/s, the
    method's read share and method GB/s (HIP events around each call)."""
    lines = [f"# Single-pattern search per cell: {workload}", "",
             "Per (sigma, m): the launch tuple used, median call time (search + emit kernels, HIP events "
             "on the launch stream, mean over steps per pattern, median over patterns), text GB/s = n / "
             "time, the share of 128-byte text lines the sequential searching phase reads with the same "
             "(q, alpha, w) (`hc_method_bytes.json`; 1 for m <= 32), and method GB/s = (that share x n + "
             "8 x occurrences + table + m) / time.", "",
             "Command: `" + " ".join(sys.argv) + "`", "",
             "| sigma | m | q, alpha, w | segment, schedule, variant | median us | text GB/s | read share | "
             "method GB/s |", "|---|---|---|---|---|---|---|---|"]
    for (s, m), idx in sorted(cells.items()):
        us = float(np.median([launch_ms[i] for i in idx])) * 1e3
        n = texts[s].size
        inf = infos[idx[0]]
        fr = read_frac[idx[0]]
        occ = float(np.median([int(cnt[i]) for i in idx]))
        mb = (fr * n + 8 * occ + inf["F"].size * inf["w"] // 8 + m) if fr is not None else None
        lc = launches[idx[0]]
        lines.append(f"| {s} | {m} | {inf['q']}, {inf['alpha']}, {inf['w']} | {lc[0]}, {lc[1]}, {lc[2]} | "
                     f"{us:.2f} | {n / us / 1e3:.1f} | {fr if fr is not None else '-'} | "
                     f"{(mb / us / 1e3) if mb is not None else float('nan'):.1f} |")
    with open(args.write_cells, "w") as f:
        f.write("\n".join(lines) + "\n")


def check_single(pats, sample, wants, cnt, handles, launches, dtexts, stream):
    """Oracle parity of the timed single-pattern launches: for each sampled
    pattern, the count its timed launch reported, and the complete list of a
    re-run with the same (q, alpha, w) and launch shape into a buffer of its
    own, compared element by element with the oracle's list."""
    import torch

    from paper_2310_15711_amd import binding as B

    dev = torch.device("cuda:0")
    equal, bad = 0, []
    for i, want in zip(sample, wants):
        s = pats[i][0]
        buf = torch.empty(int(want.size) + 16, dtype=torch.int64, device=dev)
        c1 = torch.zeros(1, dtype=torch.int64, device=dev)
        B.hc_search_async(handles[i], dtexts[s], buf, c1, launch=launches[i], stream=stream)
        torch.cuda.synchronize()
        c = int(c1.item())
        ok = int(cnt[i]) == want.size and c == want.size and \
            np.array_equal(buf[:min(c, want.size)].cpu().numpy(), want)
        equal += int(ok)
        if not ok and len(bad) < 5:
            bad.append({"sigma": s, "m": pats[i][1], "offset": int(pats[i][2]), "timed_count": int(cnt[i]),
                        "rerun_count": c, "oracle_count": int(want.size)})
    return {"checked": len(sample), "equal": equal, "exact": equal == len(sample),
            "what": "sampled patterns: timed launch's count and a re-run's complete list (same tuned "
                    "launch) vs the oracle's brute force", "mismatches": bad}


def run_batched(args):
    """Batched workload: texts with log-normal lengths in [64 KiB, 16 MiB] over
    4, 20 or 64 symbols, patterns with log-uniform lengths in [4, 1024], every
    pattern paired with every text of its alphabet, all searched by one batch
    plan (a replayed HIP graph). Compared with one hc_search_async launch per
    pair, credited with only the GPU time of its launches."""
    import torch

    from paper_2310_15711_amd import binding as B
    from paper_2310_15711_amd import workloads as W

    dev = torch.device("cuda:0")
    t0 = time.time()
    b = W.batched_config(n_texts=args.batch_texts, n_patterns=args.batch_patterns)
    sizes = np.array([t.size for t in b.texts], dtype=np.int64)
    off = np.zeros(len(b.texts) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    d_text = torch.from_numpy(np.concatenate(b.texts)).to(dev)
    pp, pt = b.pairs[:, 0].copy(), b.pairs[:, 1].copy()
    pair_bytes = int(sizes[pt].sum())
    log(f"batched inputs in {time.time() - t0:.1f}s: {len(b.texts)} texts, {int(sizes.sum())} bytes, "
        f"{len(b.patterns)} patterns, {len(pp)} pairs, {pair_bytes / 1e12:.3f} TB pattern x text")
    bparams = tuple(int(v) for v in args.batch_params.split(",")) if args.batch_params else None
    btune, btune_s = None, 0.0
    if bparams is None and not args.no_batch_tune:
        # table shape, lane segment, group size and workgroups per CU of the
        # batched kernel, timed on an evenly spaced sample of this batch's pairs
        t0 = time.time()
        btune = B.hc_batch_autotune(d_text, off, b.patterns, pp, pt, max_pairs=args.batch_tune_pairs)
        btune_s = time.time() - t0
        log(f"batched autotune in {btune_s:.1f}s: {btune}")
    t0 = time.time()
    plan = B.BatchPlan(d_text, off, b.patterns, pp, pt, params=bparams)
    plan_s = time.time() - t0
    pair_off = torch.empty(len(pp) + 1, dtype=torch.int64, device=dev)
    empty = torch.empty(0, dtype=torch.int64, device=dev)
    _, total = plan.run(empty, pair_off)
    pos = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
    for _ in range(max(args.warmup, 1)):
        plan.run(pos, pair_off)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        st, tot = plan.run(pos, pair_off)
        e1.record()
        torch.cuda.synchronize()
        assert st == B.HC_OK and tot == total
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    value = pair_bytes / (ms * 1e-3) / 1e9
    # integer work the method itself does on the plan's pairs, against the
    # chip's int32 lane-op rate (the batched kernel is bound by ALU and LDS,
    # not HBM: each staged tile serves a whole group of patterns)
    qa, aa, wa = bparams if bparams else (0, 12, 16)
    qs = [B.hc_pattern_info(B.hc_preprocess(x, (min(qa, len(x)), aa or 12, wa or 16)))["q"]
          for x in b.patterns]   # the q the plan gives each pattern
    ms_pat = np.array([len(x) for x in b.patterns], dtype=np.float64)
    per_byte = (2.0 * np.array(qs) + 6.0) / (ms_pat - np.array(qs) + 1.0)
    ops = float(np.sum(sizes[pt] * per_byte[pp]))
    roof = alu_roofline(ops, ms * 1e-3, "hc_batch_kernel + CSR kernels (one plan run)")
    # oracle parity: a seeded sample of pairs, complete lists
    from oracle import hc_oracle as O

    po_h = pair_off.cpu().numpy()
    g = np.random.default_rng([231015711, 4, 9, 0])
    sample = np.sort(g.choice(len(pp), size=min(len(pp), args.batch_oracle_pairs), replace=False))
    t1 = time.time()
    equal, bad = 0, []
    for k in sample:
        want = O.occurrences(b.patterns[int(pp[k])], b.texts[int(pt[k])])
        lo, hi = int(po_h[k]), int(po_h[k + 1])
        ok = hi - lo == want.size and np.array_equal(pos[lo:hi].cpu().numpy(), want)
        equal += int(ok)
        if not ok and len(bad) < 5:
            bad.append({"pair": int(k), "count": hi - lo, "oracle_count": int(want.size)})
    parity = {"checked": int(sample.size), "equal": equal, "exact": equal == int(sample.size),
              "what": "seeded sample of (pattern, text) pairs of the timed plan, complete lists vs the "
                      "oracle's brute force", "mismatches": bad}
    log(f"batched oracle parity in {time.time() - t1:.1f}s: {equal}/{sample.size}")
    per_pattern = None
    if not args.no_per_pattern:
        handles = [B.hc_preprocess(x) for x in b.patterns]
        po = pair_off.cpu().numpy()
        out2 = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
        cnt = torch.zeros(len(pp), dtype=torch.int64, device=dev)
        stream = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in pp]
        base = d_text.data_ptr()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for k in range(len(pp)):
            t_ = int(pt[k])
            ev[k][0].record(stream)
            c = int(po[k + 1] - po[k])
            B.hc_search_async(handles[int(pp[k])], None, out2[int(po[k]):int(po[k]) + c] if c else None,
                              cnt[k:k + 1], stream=stream, n=int(sizes[t_]), y_ptr=base + int(off[t_]))
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        busy_ms = sum(a.elapsed_time(z) for a, z in ev)
        ok = bool(torch.equal(cnt.cpu(), torch.from_numpy(np.diff(po))))
        same = ok and bool(torch.equal(out2[:total], pos[:total]))
        per_pattern = {"gbps_gpu_busy": round(pair_bytes / (busy_ms * 1e-3) / 1e9, 1),
                       "gbps_wall": round(pair_bytes / wall / 1e9, 1), "launches": len(pp),
                       "gpu_busy_ms": round(busy_ms, 2), "wall_s": round(wall, 2),
                       "same_results": same}
    rec = {
        "metric": "text GB/s per pattern (HC vs batched) + % HBM peak; p50/p99 search latency",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"batched HC: {len(b.texts)} texts ({int(sizes.sum())} bytes, log-normal "
                               f"64 KiB-16 MiB, sigma 4/20/64), {len(b.patterns)} patterns "
                               f"(m log-uniform 4..1024), {len(pp)} pairs, one plan run per step",
                   "pattern_x_text_bytes": pair_bytes, "occurrences": int(total),
                   "plan_create_s": round(plan_s, 2),
                   "autotune": ({"seconds": round(btune_s, 1), "choice": btune} if btune else None)},
        "parity": parity,
        "roofline": roof,
        "per_pattern_launches": per_pattern,
        "speedup_vs_per_pattern_gpu_busy": (round(value / per_pattern["gbps_gpu_busy"], 2)
                                            if per_pattern else None),
    }
    del plan, d_text, pos, pair_off
    torch.cuda.empty_cache()
    return rec


def run_served(args):
    """Served workload: eight resident 128 MiB texts (four iid bytes, four
    order-2 Markov walks), open-loop Poisson arrivals at each rate, every
    request a text and a pattern of log-uniform length in [4, 2048]
    (extracted with probability 1/2). Arrivals are submitted by native
    threads at their scheduled times (libhc_loadgen), completions taken by a
    native collector. Latency = observed completion minus scheduled arrival
    (p50/p99 after the first 10% of arrivals); aggregate GB/s = text bytes of
    all requests over first arrival to last completion. A seeded sample of
    requests per rate is compared with hc_search alone, and a smaller one
    with the oracle's brute force."""
    import ctypes

    import torch

    from paper_2310_15711_amd import binding as B
    from paper_2310_15711_amd import workloads as W

    dev = torch.device("cuda:0")
    t0 = time.time()
    texts = W.served_texts(n_each=args.serve_text_mib << 20)
    dtexts = [torch.from_numpy(t).to(dev) for t in texts]
    torch.cuda.synchronize()
    log(f"served inputs in {time.time() - t0:.1f}s: {len(texts)} texts x {args.serve_text_mib} MiB")
    B.lib()
    gen = ctypes.CDLL(os.path.join(ROOT, "paper_2310_15711_amd", "libhc_loadgen.so"))
    P = ctypes.c_void_p
    gen.hc_loadgen_run.restype = ctypes.c_int
    gen.hc_loadgen_run.argtypes = [P, ctypes.c_int64, P, P, P, P, P, ctypes.c_int32, ctypes.c_double,
                                   P, P, P, P, ctypes.c_int64, P]
    rates = [float(r) for r in args.serve_rates.split(",")]
    out = {}
    from oracle import hc_oracle as O

    # the server's batched kernel takes the process-wide batch knobs (table
    # shape, lane segment, group size, workgroups per CU): tuned once at
    # start-up on a sample of requests of the same kind (its own seed), as a
    # deployment would, outside every timed region
    stune = None
    if not args.no_batch_tune:
        t0 = time.time()
        sreqs = W.request_stream(texts, args.serve_tune_requests / 2.0, 2.0, sub=97)
        soff = np.zeros(len(texts) + 1, dtype=np.int64)
        soff[1:] = np.cumsum([t.size for t in texts])
        d_all = torch.cat(dtexts)
        stune = B.hc_batch_autotune(d_all, soff, [r.pattern for r in sreqs],
                                    np.arange(len(sreqs), dtype=np.int32),
                                    np.array([r.text for r in sreqs], dtype=np.int32),
                                    max_pairs=len(sreqs))
        del d_all
        torch.cuda.empty_cache()
        stune = {"seconds": round(time.time() - t0, 1), "requests": len(sreqs), "choice": stune}
        log(f"served batch knobs tuned in {stune['seconds']}s: {stune['choice']}")

    o_checked, o_equal, o_bad = 0, 0, []
    start_delay = 0.05
    for ri, rate in enumerate(rates):
        reqs = W.request_stream(texts, rate, args.serve_seconds, sub=ri)
        n = len(reqs)
        arrival = np.array([r.arrival for r in reqs], dtype=np.float64) + start_delay
        tid = np.array([r.text for r in reqs], dtype=np.int32)
        pat = np.frombuffer(b"".join(r.pattern for r in reqs), dtype=np.uint8)
        poff = np.zeros(n + 1, dtype=np.int64)
        poff[1:] = np.cumsum([len(r.pattern) for r in reqs])
        g = np.random.default_rng([231015711, 5, 9, ri])
        sample = g.choice(n, size=min(n, args.serve_check), replace=False)
        per_rate = -(-args.serve_oracle // len(rates))
        osample = sample[:min(sample.size, per_rate)]
        keep = np.zeros(n, dtype=np.uint8)
        keep[sample] = 1
        submit_s, done_s = np.zeros(n), np.zeros(n)
        count = np.zeros(n, dtype=np.int64)
        pos_cap = 1 << 25
        pos = np.zeros(pos_cap, dtype=np.int64)
        pos_off = np.zeros(n + 1, dtype=np.int64)
        srv = B.Server(dtexts, args.serve_budget_mib << 20)
        rc = gen.hc_loadgen_run(srv.handle, n, arrival.ctypes.data, tid.ctypes.data, pat.ctypes.data,
                                poff.ctypes.data, keep.ctypes.data, args.serve_threads, 600.0,
                                submit_s.ctypes.data, done_s.ctypes.data, count.ctypes.data, pos.ctypes.data,
                                pos_cap, pos_off.ctypes.data)
        if rc != B.HC_OK:
            raise RuntimeError(f"served load failed: {B.strerror(rc)} ({rc})")
        sstats = srv.stats()
        srv.close()
        lat = (done_s - arrival) * 1e3
        keep_lat = np.argsort(arrival)[n // 10:]
        text_bytes = float(sum(texts[r.text].size for r in reqs))
        makespan = float(done_s.max() - arrival.min())

        def result(i):
            o = int(pos_off[i])
            return None if o < 0 else pos[o:o + int(count[i])]

        # exact results: the sample against hc_search alone, part of it
        # against the oracle's brute force
        same, checked_alone = True, 0
        for i in sample:
            got = result(int(i))
            if got is None:
                continue
            r = reqs[int(i)]
            alone = B.find_all(B.hc_preprocess(r.pattern), dtexts[r.text]).cpu().numpy()
            checked_alone += 1
            if not np.array_equal(alone, got):
                same = False
                break
        for i in osample:
            got = result(int(i))
            r = reqs[int(i)]
            want = O.occurrences(r.pattern, texts[r.text])
            ok = got is not None and np.array_equal(want, got)
            o_equal += int(ok)
            o_checked += 1
            if not ok and len(o_bad) < 5:
                o_bad.append({"rate": rate, "request": int(i), "text": r.text, "m": len(r.pattern),
                              "count": int(count[int(i)]), "oracle_count": int(want.size)})
        out[str(int(rate))] = {
            "requests": n, "offered_rate": rate,
            "submitted_rate": round(n / float(submit_s.max() - submit_s.min() + 1e-9), 1),
            "p50_ms": round(float(np.percentile(lat[keep_lat], 50)), 3),
            "p99_ms": round(float(np.percentile(lat[keep_lat], 99)), 3),
            "agg_gbps": round(text_bytes / makespan / 1e9, 1),
            "server_busy_gbps": round(sstats["agg_gbps"], 1),
            "server_p50_ms": round(sstats["p50_us"] / 1e3, 3),
            "server_p99_ms": round(sstats["p99_us"] / 1e3, 3),
            "checked_vs_alone": checked_alone, "same_as_alone": same,
        }
        log(f"served rate {rate:.0f}/s: {out[str(int(rate))]}")
    # baseline: the same kind of requests, one hc_search_async launch each,
    # back to back on one stream (GPU-busy time counted from HIP events)
    reqs = W.request_stream(texts, 1000.0, 2.0, sub=99)
    handles = [B.hc_preprocess(r.pattern) for r in reqs]
    pos = torch.empty(1 << 24, dtype=torch.int64, device=dev)
    cnt = torch.zeros(len(reqs), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    for i in range(min(8, len(reqs))):   # warm-up
        B.hc_search_async(handles[i], dtexts[reqs[i].text], pos, cnt[i:i + 1], stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in reqs]
    w0 = time.perf_counter()
    for i, r in enumerate(reqs):
        ev[i][0].record(stream)
        B.hc_search_async(handles[i], dtexts[r.text], pos, cnt[i:i + 1], stream=stream)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    busy = sum(a.elapsed_time(b) for a, b in ev) * 1e-3
    nbytes = float(sum(texts[r.text].size for r in reqs))
    baseline = {"requests": len(reqs), "gbps_gpu_busy": round(nbytes / busy / 1e9, 1),
                "gbps_wall": round(nbytes / wall / 1e9, 1)}
    log(f"served baseline (one launch per request): {baseline}")
    del dtexts, pos
    torch.cuda.empty_cache()
    best = max(out.values(), key=lambda r: r["agg_gbps"])
    return {"workload": f"served HC: {len(texts)} resident texts x {args.serve_text_mib} MiB "
                        f"(4 iid bytes, 4 order-2 Markov), Poisson arrivals for "
                        f"{args.serve_seconds} s per rate, m log-uniform 4..2048",
            "budget_mib": args.serve_budget_mib, "batch_tuning": stune, "rates": out,
            "parity": {"checked": o_checked, "equal": o_equal, "exact": o_equal == o_checked,
                       "what": "seeded sample of served requests (spread over the rates), complete "
                               "lists vs the oracle's brute force", "mismatches": o_bad},
            "per_request_launches": baseline,
            "speedup_vs_per_request_gpu_busy": round(best["agg_gbps"] / baseline["gbps_gpu_busy"], 2)}


def time_cpu_hc(pats, infos, texts, threads):
    """The paper's sequential HC on the host: the oracle's C scan (its own
    preprocessing, then the searching phase over the whole text, with the
    line accounting the method-byte table uses), one pattern per (sigma, m)
    cell with that cell's tuned (q, alpha, w); on one core, and the same
    patterns spread over all cores; preprocessing alone timed on an empty
    text."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import hc_oracle as O

    first = {}
    for i, (s, m, _, _) in enumerate(pats):
        first.setdefault((s, m), i)
    jobs = [(pats[i][3], texts[pats[i][0]], infos[i]) for i in first.values()]

    def one(j, y=None):
        x, yy, inf = j
        return O.hc_scan(x, yy if y is None else y, inf["q"], inf["alpha"], inf["w"])

    nbytes = float(sum(y.size for _, y, _ in jobs))
    t0 = time.perf_counter()
    for j in jobs:
        one(j)
    t_one = time.perf_counter() - t0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, jobs))
    t_all = time.perf_counter() - t0
    empty = np.zeros(0, dtype=np.uint8)
    t0 = time.perf_counter()
    for j in jobs:
        one(j, empty)
    t_pre = time.perf_counter() - t0
    return {"one_core_gbps": round(nbytes / t_one / 1e9, 3),
            "one_core_search_only_gbps": round(nbytes / max(t_one - t_pre, 1e-9) / 1e9, 3),
            "all_cores_gbps": round(nbytes / t_all / 1e9, 3), "cores": threads,
            "preprocessing_ms_per_pattern": round(t_pre / len(jobs) * 1e3, 3),
            "kind": "oracle (sequential HC, hc_seq.c)",
            "sample": f"{len(jobs)} patterns (one per sigma and m, the cell's tuned q, alpha, w), each over "
                      f"its full text"}


def run_markov_leg(args):
    """The order-2 Markov workload (three 256 MiB walks over 27 symbols, m
    4..1024) in a child process of its own (it tunes its own texts), reduced
    to its value, parity and roofline."""
    import subprocess

    # the oracle leg runs on 4 patterns per cell: its lists are the parity check
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "markov", "--no-extras",
           "--cpu-sample-patterns", "4", "--steps", str(args.steps), "--warmup", str(args.warmup),
           "--per-length", str(min(args.per_length, 50))]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"markov leg failed ({r.returncode}): {r.stderr[-2000:]}")
    d = json.loads(r.stdout.strip().splitlines()[-1])
    log(f"markov leg: {d['value']} GB/s, parity {d['parity']['equal']}/{d['parity']['checked']}")
    return {"value": d["value"], "unit": d["unit"], "ms_per_step": d["ms_per_step"],
            "config": {"workload": d["config"]["workload"]}, "parity": d["parity"],
            "roofline": {k: d["roofline"][k] for k in ("achieved", "frac", "avg_launch_us", "frac_method")},
            "detail_median_text_gbps": d["detail_median_text_gbps"]}


def main():
    args = parse()
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats, args.summary_cmd)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.summary_cmd, args.per_unit, args.unit)
        return
    if args.summarize:
        summarize(*args.summarize, args.summary_cmd)
        if args.lds_dir:
            print(json.dumps(summarize_lds(args.lds_dir, args.summary_cmd)))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library searches on one GPU; sharding across GPUs is not implemented; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2310_15711_amd import binding as B
    from paper_2310_15711_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.calib_copy:
        calib_copy()
        return
    if args.workload == "batched":
        print(json.dumps(run_batched(args)), flush=True)
        return
    if args.workload == "served":
        sv = run_served(args)
        best = max(sv["rates"].values(), key=lambda r: r["agg_gbps"])
        rec = {"metric": "text GB/s per pattern (HC vs batched) + % HBM peak; p50/p99 search latency",
               "value": best["agg_gbps"], "unit": "GB/s", "n_gpus": 1, "steps": len(sv["rates"]),
               "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "u8", "data": "synthetic",
               "config": {"workload": sv["workload"]}, "served": sv}
        print(json.dumps(rec), flush=True)
        return
    dev = torch.device("cuda:0")
    B.lib()
    n = args.text_mib << 20

    # ---------------------------------------------------------------- inputs
    t0 = time.time()
    texts = {}
    if args.workload == "single":
        sigmas = [int(s) for s in args.sigmas.split(",")]
        lengths = [int(v) for v in args.lengths.split(",")] if args.lengths else list(W.SINGLE_LENGTHS)
        for s in sigmas:
            texts[s] = W.single_text(s, n)
        per = {(s, m): W.single_patterns(texts[s], s, m, args.per_length) for s in sigmas for m in lengths}
        # consecutive launches go to different texts (3 x 256 MiB do not fit
        # in the 256 MB Infinity Cache) and to different cells: the launches
        # of one cell are 29 launches apart, most of them streaming a whole
        # text, so a launch that reads only part of its text (the sparse
        # variant touches the same lines for every pattern of one length)
        # does not find them in the cache from the cell's previous launch
        pats = [(s, m) + per[(s, m)][j] for j in range(args.per_length) for m in lengths for s in sigmas]
        workload = (f"single-pattern HC: {len(sigmas)} iid texts x {args.text_mib} MiB "
                    f"(sigma {args.sigmas}), m in {lengths}, {args.per_length} patterns each")
    elif args.workload == "markov":
        lengths = [int(v) for v in args.lengths.split(",")] if args.lengths else list(W.MARKOV_LENGTHS)
        # three walks of the same chain (keys 27, 28, 29), launches
        # alternating between them and between cells as in the iid workload
        walks = (27, 28, 29)
        for k, key in enumerate(walks):
            texts[key] = W.markov_text(n, walk_sub=k)
        per = {(key, m): W.markov_patterns(texts[key], m, args.per_length) for key in walks for m in lengths}
        pats = [(key, m) + per[(key, m)][j] for j in range(args.per_length) for m in lengths for key in walks]
        workload = (f"single-pattern HC on order-2 Markov text (3 walks x {args.text_mib} MiB, 27 symbols), "
                    f"m in {lengths}, {args.per_length} patterns each")
    else:
        p = W.planted_config()
        texts[4] = p.y
        pats = [(4, 32, p.source, p.x)]
        workload = "planted: 1 MiB iid ACGT, m=32, 100 planted copies"
    log(f"inputs ready in {time.time() - t0:.1f}s: {len(pats)} patterns")

    dtexts = {s: torch.from_numpy(y).to(dev) for s, y in texts.items()}
    params = tuple(int(v) for v in args.params.split(",")) if args.params else None
    launch = (args.segment, args.schedule, args.variant, args.wg_per_cu)
    # autotuning (outside the timed region): per text, the fastest q, alpha,
    # w, schedule and segment for each pattern length, measured by the
    # library on patterns of its own choosing from that text
    tuned, tune_s = {}, 0.0
    if args.load_tuned:
        with open(args.load_tuned) as f:
            raw = json.load(f)
        tuned = {int(s_): {int(m): {"params": tuple(r["params"]), "launch": tuple(r["launch"])}
                           for m, r in d.items()} for s_, d in raw.items()}
    elif not args.no_tune and params is None and launch == (0, 0, 0, 0):
        t0 = time.time()
        for s_, yd in dtexts.items():
            ms = sorted({m for (s2, m, _, _) in pats if s2 == s_})
            tuned[s_] = {r["m"]: r for r in B.hc_autotune(yd, ms, patterns=args.tune_patterns)}
        tune_s = time.time() - t0
        B.hc_autotune_reset()
        log(f"autotuned in {tune_s:.1f}s")
        if args.save_tuned:
            with open(args.save_tuned, "w") as f:
                json.dump({str(s_): {str(m): {"params": list(r["params"]), "launch": list(r["launch"])}
                                     for m, r in d.items()} for s_, d in tuned.items()}, f, indent=1)
    handles = [B.hc_preprocess(x, tuned[s][m]["params"] if tuned else params) for (s, m, _, x) in pats]
    launches = [tuned[s][m]["launch"] if tuned else launch for (s, m, _, _) in pats]
    cap = 1 << 25
    out = torch.empty(cap, dtype=torch.int64, device=dev)
    counts = torch.zeros(len(pats), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    ev0 = [[torch.cuda.Event(enable_timing=True) for _ in pats] for _ in range(args.steps)]
    ev1 = [[torch.cuda.Event(enable_timing=True) for _ in pats] for _ in range(args.steps)]

    def step(k):
        for i, (s, m, off, x) in enumerate(pats):
            if k is not None:
                ev0[k][i].record(stream)
            B.hc_search_async(handles[i], dtexts[s], out, counts[i:i + 1], launch=launches[i],
                              stream=stream)
            if k is not None:
                ev1[k][i].record(stream)

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()

    # timed steps: back-to-back launches, events only around the whole run
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    t_wall = time.perf_counter()
    for _ in range(args.steps):
        step(None)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_total = start.elapsed_time(stop)
    ms_step = ms_total / args.steps

    # the same steps again with an event pair around every call (search +
    # emit kernels): the per-call durations of the roofline and the detail
    e_start, e_stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e_start.record(stream)
    for k in range(args.steps):
        step(k)
    e_stop.record(stream)
    torch.cuda.synchronize()
    ms_step_events = e_start.elapsed_time(e_stop) / args.steps
    per_launch = np.array([[ev0[k][i].elapsed_time(ev1[k][i]) for i in range(len(pats))]
                           for k in range(args.steps)])

    cnt = counts.cpu().numpy()
    text_bytes = sum(int(texts[s].size) for (s, _, _, _) in pats)
    value = text_bytes / (ms_step * 1e-3) / 1e9
    launch_ms = per_launch.mean(axis=0)                      # per pattern, mean over steps
    # average call duration over the timed back-to-back steps (one event pair
    # around all of them on the launch stream); the per-call events of the
    # second run add about 2 us per call and only serve the per-cell detail
    avg_launch_ms = ms_step / len(pats)
    avg_launch_ms_events = float(launch_ms.mean())
    # algorithmic bytes per launch: the text once, the positions written,
    # F and x read
    infos = [B.hc_pattern_info(h) for h in handles]
    alg_bytes = np.array([texts[s].size + 8 * int(c) + inf["F"].size * inf["w"] // 8 + m
                          for (s, m, _, _), c, inf in zip(pats, cnt, infos)], dtype=np.float64)
    achieved = float(alg_bytes.mean() / (avg_launch_ms * 1e-3) / 1e9)
    # the method's own bytes: the share of the text's 128-byte lines that the
    # sequential searching phase reads with the same (q, alpha, w), from the
    # table the oracle's scan wrote (every line for m <= 32)
    read_frac = method_read_fractions(pats, infos)
    method_bytes = None
    if all(f is not None for f in read_frac):
        method_bytes = np.array([texts[s].size * f + 8 * int(c) + inf["F"].size * inf["w"] // 8 + m
                                 for (s, m, _, _), c, inf, f in zip(pats, cnt, infos, read_frac)],
                                dtype=np.float64)
    achieved_method = (float(method_bytes.mean() / (avg_launch_ms * 1e-3) / 1e9)
                       if method_bytes is not None else None)

    detail, cells = {}, {}
    for i, (s, m, _, _) in enumerate(pats):
        detail.setdefault(f"{s}/{m}", []).append(texts[s].size / (launch_ms[i] * 1e-3) / 1e9)
        cells.setdefault((s, m), []).append(i)
    spread = {k: [round(float(np.percentile(v, q)), 1) for q in (10, 50, 90)] for k, v in detail.items()}
    detail = {k: round(float(np.median(v)), 1) for k, v in detail.items()}
    if args.detail:
        for k, v in detail.items():
            log(f"  sigma/m {k:10s} median text GB/s {v:9.1f}")
    if args.write_cells:
        write_cells(args, cells, pats, launch_ms, texts, cnt, infos, read_frac, launches, workload)

    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json))
            if tj.get("workload") == args.workload and tj.get("kernel_source") == kernel_source_hash():
                traffic = tj.get("bytes_per_launch")
        except Exception:
            traffic = None

    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "hc_search_kernel or hc_sparse_kernel, then hc_emit_kernel (one search call)",
                "avg_launch_us": round(avg_launch_ms * 1e3, 2),
                "avg_launch_us_with_call_events": round(avg_launch_ms_events * 1e3, 2),
                "alg_bytes_per_launch": round(float(alg_bytes.mean())),
                "frac_text": round(achieved / HBM_PEAK_GBPS, 4),
                "achieved_method": round(achieved_method, 1) if achieved_method else None,
                "frac_method": round(achieved_method / HBM_PEAK_GBPS, 4) if achieved_method else None,
                "method_bytes_per_launch": round(float(method_bytes.mean())) if method_bytes is not None else None,
                "method_bytes_source": "profiles/hc_method_bytes.json (share of 128-byte text lines the "
                                       "sequential searching phase reads, per sigma, m, q, alpha, w)"}

    cpu = None
    parity = None
    cpu_hc = None
    if not args.no_cpu_baseline:
        from oracle import hc_oracle as O

        th = O.default_threads()
        sample = []
        per_cell = {}
        for i, (s, m, off, x) in enumerate(pats):
            if per_cell.get((s, m), 0) < args.cpu_sample_patterns:
                per_cell[(s, m)] = per_cell.get((s, m), 0) + 1
                sample.append(i)
        t1 = time.perf_counter()
        nbytes = 0
        wants = []
        for i in sample:
            s, m, _, x = pats[i]
            wants.append(O.occurrences(x, texts[s], threads=th))
            nbytes += texts[s].size
        dt = time.perf_counter() - t1
        cpu = {"value": round(nbytes / dt / 1e9, 3), "unit": "GB/s", "cores": th, "kind": "oracle",
               "sample": f"{len(sample)} patterns ({args.cpu_sample_patterns} per sigma and m), each "
                         f"over its full {args.text_mib} MiB text, {dt:.1f} s"}
        parity = check_single(pats, sample, wants, cnt, handles, launches, dtexts, stream)
        if args.workload == "single":
            cpu_hc = time_cpu_hc(pats, infos, texts, th)

    rec = {
        "metric": "text GB/s per pattern (HC vs batched) + % HBM peak; p50/p99 search latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": workload, "launches_per_step": len(pats),
                   "text_bytes_per_step": text_bytes, "occurrences_per_step": int(cnt.sum()),
                   "wall_s": round(wall, 3),
                   "ms_per_step_with_call_events": round(ms_step_events, 3),
                   "autotune": ({"seconds": round(tune_s, 1),
                                 "choice": {f"{s_}/{m}": {"q_alpha_w": list(r["params"]),
                                                          "segment": r["launch"][0],
                                                          "schedule": r["launch"][1]}
                                            for s_, d in tuned.items() for m, r in d.items()}}
                                if tuned else None)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "detail_median_text_gbps": detail,
        "detail_p10_p50_p90_text_gbps": spread,
    }
    if cpu_hc is not None:
        rec["cpu_hc"] = cpu_hc
    if args.workload == "single" and not args.no_extras:
        del dtexts, out
        torch.cuda.empty_cache()
        bt = run_batched(args)
        rec["batched"] = {"value": bt["value"], "unit": "GB/s", "config": bt["config"],
                          "parity": bt["parity"], "roofline": bt["roofline"],
                          "per_pattern_launches": bt["per_pattern_launches"],
                          "speedup_vs_per_pattern_gpu_busy": bt["speedup_vs_per_pattern_gpu_busy"]}
        B.hc_autotune_reset()   # the served leg runs on the library's defaults
        rec["served"] = run_served(args)
        rec["markov"] = run_markov_leg(args)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
