#!/usr/bin/env python3
"""Summaries of rocprofv3 runs of bench.py, as committed under profiles/.

  python bench_profile.py stats DIR TITLE COMMAND
      per-kernel durations from the *kernel_stats.csv under DIR (a
      `rocprofv3 --kernel-trace --stats` run), as a markdown table

  python bench_profile.py counters OUT_JSON OUT_MD TITLE NOTE DIR1 CMD1 [DIR2 CMD2 ...]
      per-kernel means of every counter of several `rocprofv3 --pmc` passes,
      with read / write bytes at the L2-to-fabric interface (from the
      request-size counters), the L2 hit rate and the DRAM share of reads
      (OUT_JSON "-" writes the markdown only)
"""

import csv
import glob
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit("no *%s under %s" % (suffix, d))
    return hits


def _short(name, width=90):
    return name if len(name) <= width else name[:width]


def _dispatch_durations(d):
    """kernel name -> sorted dispatch durations in µs, from the kernel trace
    (empty when the run wrote none)."""
    per = {}
    for path in sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)):
        with open(path) as f:
            for r in csv.DictReader(f):
                per.setdefault(r["Kernel_Name"], []).append(
                    (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return {k: sorted(v) for k, v in per.items()}


def stats(d, title, command):
    rows = []
    for path in _find(d, "kernel_stats.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                rows.append(r)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    durs = _dispatch_durations(d)
    out = ["# Kernel trace: %s" % title, "", "Command (from the repository root, on one MI355X):", "", "```",
           command, "```", "", "Per-kernel durations (`--stats`; median, min and max from the dispatch trace):", "",
           "| kernel | calls | avg µs | median µs | min µs | max µs | total ms | % |",
           "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        v = durs.get(r["Name"], [])
        med, lo, hi = (("%.2f" % v[len(v) // 2], "%.2f" % v[0], "%.2f" % v[-1]) if v else ("-", "-", "-"))
        out.append("| `%s` | %s | %.2f | %s | %s | %s | %.3f | %.1f |" % (
            _short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, med, lo, hi,
            float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    print("\n".join(out))


def _all_counters(d):
    """kernel name -> ({counter: mean value per dispatch}, dispatches) over one --pmc run."""
    acc = {}
    for path in _find(d, "counter_collection.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                key = (r["Kernel_Name"], r.get("Dispatch_Id", r.get("Correlation_Id", "")), r["Counter_Name"])
                acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
    per = {}
    for (name, _, cname), v in acc.items():
        per.setdefault(name, {}).setdefault(cname, []).append(v)
    return {k: ({c: sum(v) / len(v) for c, v in cs.items()}, max(len(v) for v in cs.values()))
            for k, cs in per.items()}


def _derived(cs):
    """Bytes and rates from the raw counters of one kernel (None where a
    counter was not taken)."""
    g = cs.get
    out = {}
    if all(g(c) is not None for c in ("TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_32B_sum")):
        out["read_bytes"] = 128 * g("TCC_EA0_RDREQ_128B_sum") + 64 * g("TCC_EA0_RDREQ_64B_sum") \
            + 32 * g("TCC_EA0_RDREQ_32B_sum")
    if g("TCC_EA0_WRREQ_sum") is not None and g("TCC_EA0_WRREQ_64B_sum") is not None:
        out["write_bytes"] = 64 * g("TCC_EA0_WRREQ_64B_sum") + 32 * (g("TCC_EA0_WRREQ_sum") - g("TCC_EA0_WRREQ_64B_sum"))
    if g("TCC_HIT_sum") is not None and g("TCC_MISS_sum") is not None and g("TCC_HIT_sum") + g("TCC_MISS_sum") > 0:
        out["l2_hit_rate"] = g("TCC_HIT_sum") / (g("TCC_HIT_sum") + g("TCC_MISS_sum"))
    if g("TCC_EA0_RDREQ_DRAM_sum") is not None and g("TCC_EA0_RDREQ_sum"):
        out["dram_share_of_read_requests"] = g("TCC_EA0_RDREQ_DRAM_sum") / g("TCC_EA0_RDREQ_sum")
    return out


def counters(out_json, out_md, title, note, runs):
    """Merge several --pmc runs (DIR, COMMAND pairs) into per-kernel counter
    means and the bytes derived from them."""
    from bench import kernel_source_hash
    merged, calls = {}, {}
    for d, _ in runs:
        for k, (cs, n) in _all_counters(d).items():
            merged.setdefault(k, {}).update(cs)
            calls[k] = n
    # kernels that move at least 0.1 % of the bytes of the largest one
    def moved(k):
        d = _derived(merged[k])
        return (d.get("read_bytes", 0.0) + d.get("write_bytes", 0.0)) * calls[k]
    top = max((moved(k) for k in merged), default=0.0)
    names = sorted((k for k in merged if moved(k) >= 1e-3 * top), key=lambda k: -moved(k))
    res = {"title": title, "kernel_source_sha256_16": kernel_source_hash(), "commands": [c for _, c in runs],
           "kernels": {}}
    for k in names:
        cs = merged[k]
        res["kernels"][_short(k)] = {"dispatches": calls[k],
                                     "counters": {c: round(v, 1) for c, v in sorted(cs.items())},
                                     "derived": {c: (round(v, 4) if isinstance(v, float) else v)
                                                 for c, v in _derived(cs).items()}}
    if out_json != "-":
        with open(out_json, "w") as f:
            json.dump(res, f, indent=1)
    cols = sorted({c for cs in merged.values() for c in cs})
    md = ["# Counters: %s" % title, "", note, "", "Commands (one rocprofv3 pass each, from /tmp on one MI355X):", "",
          "```"] + [c for _, c in runs] + ["```", "",
          "Mean per dispatch. Read bytes = 128 x RDREQ_128B + 64 x RDREQ_64B + 32 x RDREQ_32B; write bytes = "
          "64 x WRREQ_64B + 32 x (WRREQ - WRREQ_64B).  These are requests from the L2 to the data fabric: the "
          "Infinity Cache (MALL) may serve a read without HBM, so they bound HBM traffic from above.", "",
          "| kernel | dispatches | GB moved, all dispatches | read bytes | write bytes | L2 hit rate | "
          "DRAM share of read requests |",
          "|---|---:|---:|---:|---:|---:|---:|"]
    for k in names:
        d = _derived(merged[k])
        md.append("| `%s` | %d | %.2f | %s | %s | %s | %s |" % (
            _short(k, 70), calls[k], moved(k) / 1e9, "%.0f" % d["read_bytes"] if "read_bytes" in d else "-",
            "%.0f" % d["write_bytes"] if "write_bytes" in d else "-",
            "%.3f" % d["l2_hit_rate"] if "l2_hit_rate" in d else "-",
            "%.3f" % d["dram_share_of_read_requests"] if "dram_share_of_read_requests" in d else "-"))
    md += ["", "Raw counters (mean per dispatch):", "", "| kernel | " + " | ".join(cols) + " |",
           "|---|" + "---:|" * len(cols)]
    for k in names:
        md.append("| `%s` | " % _short(k, 70) + " | ".join(
            "%.0f" % merged[k][c] if c in merged[k] else "-" for c in cols) + " |")
    with open(out_md, "w") as f:
        f.write("\n".join(md) + "\n")


if __name__ == "__main__":
    if len(sys.argv) >= 5 and sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif len(sys.argv) >= 8 and sys.argv[1] == "counters" and len(sys.argv) % 2 == 0:
        counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5],
                 list(zip(sys.argv[6::2], sys.argv[7::2])))
    else:
        print(__doc__, file=sys.stderr)
        sys.exit(2)
