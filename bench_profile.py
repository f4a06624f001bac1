#!/usr/bin/env python3
"""Summaries of rocprofv3 runs of bench.py, as committed under profiles/.

  python bench_profile.py stats DIR TITLE COMMAND
      per-kernel durations from the *kernel_stats.csv under DIR (a
      `rocprofv3 --kernel-trace --stats` run), as a markdown table

  python bench_profile.py traffic FETCH_DIR WRITE_DIR COPY_BYTES OUT_JSON OUT_MD CMD_FETCH CMD_WRITE
      HBM traffic per launch of the large-stripe encode and replay kernels
      from two `rocprofv3 --pmc` passes over `bench.py --mode counters`
      (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch).  Each counter is
      scaled by the bytes a plain device copy of COPY_BYTES moves over what
      the counter reports for that copy, summed over the dispatches the
      runtime splits it into.  The JSON records the hash of the
      library sources, so bench.py reports the traffic only while the kernels
      are the ones measured.
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


def stats(d, title, command):
    rows = []
    for path in _find(d, "kernel_stats.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                rows.append(r)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["# Kernel trace: %s" % title, "", "Command (from the repository root, on one MI355X):", "", "```",
           command, "```", "", "Per-kernel durations (`--stats`):", "",
           "| kernel | calls | avg µs | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        out.append("| `%s` | %s | %.2f | %.3f | %.1f |" % (
            _short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6,
            float(r["Percentage"])))
    print("\n".join(out))


def _counter(d, counter, total=False):
    """kernel name -> mean counter value per dispatch (KiB), or with total the
    sum over the kernel's dispatches."""
    acc = {}
    for path in _find(d, "counter_collection.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                key = (r["Kernel_Name"], r.get("Dispatch_Id", r.get("Correlation_Id", "")))
                acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
    per = {}
    for (name, _), v in acc.items():
        per.setdefault(name, []).append(v)
    return {k: (sum(v) if total else sum(v) / len(v)) for k, v in per.items()}


def traffic(fetch_dir, write_dir, copy_bytes, out_json, out_md, cmd_fetch, cmd_write):
    from bench import kernel_source_hash
    fetch = _counter(fetch_dir, "FETCH_SIZE")
    write = _counter(write_dir, "WRITE_SIZE")
    # the runtime splits the plain copy into several dispatches: its counters
    # are summed over all of them
    fetch_tot = _counter(fetch_dir, "FETCH_SIZE", total=True)
    write_tot = _counter(write_dir, "WRITE_SIZE", total=True)
    copy = [k for k in fetch_tot if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no plain copy kernel in the counter runs")
    ff = copy_bytes / (fetch_tot[copy[0]] * 1024.0)
    wf = copy_bytes / (write_tot[copy[0]] * 1024.0)
    res = {"workload": "large_stripe (k=4096, n=4506, t=65536)", "copy_bytes_each_way": copy_bytes,
           "fetch_factor": round(ff, 4), "write_factor": round(wf, 4),
           "kernel_source_sha256_16": kernel_source_hash(), "commands": [cmd_fetch, cmd_write]}
    for key, pat in (("encode", "gather_kernel"), ("replay", "replay_")):
        names = [k for k in fetch if pat in k and k in write]
        if not names:
            continue
        name = max(names, key=lambda k: fetch[k])
        fb, wb = fetch[name] * 1024.0 * ff, write[name] * 1024.0 * wf
        res[key] = {"kernel": _short(name), "fetch_KiB_raw": round(fetch[name], 1),
                    "write_KiB_raw": round(write[name], 1), "fetch_bytes_per_launch": int(fb),
                    "write_bytes_per_launch": int(wb), "bytes_per_launch": int(fb + wb)}
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    md = ["# HBM traffic: encode and replay kernels of the large stripe", "",
          "Commands (two passes, one counter each; bench.py --mode counters runs 5 encodes, 5 one-stream",
          "decodes and one plain device copy of the coded-block size), summarised by",
          "`python bench_profile.py traffic ...`:", "", "```", cmd_fetch, cmd_write, "```", "",
          "Scale = bytes the plain copy moves / what the counter reports for it: FETCH %.4f, WRITE %.4f." % (ff, wf),
          "", "| kernel | FETCH KiB raw | WRITE KiB raw | read bytes | write bytes | total per launch |",
          "|---|---:|---:|---:|---:|---:|"]
    for key in ("encode", "replay"):
        if key in res:
            r = res[key]
            md.append("| `%s` | %.1f | %.1f | %d | %d | %d |" % (
                r["kernel"], r["fetch_KiB_raw"], r["write_KiB_raw"], r["fetch_bytes_per_launch"],
                r["write_bytes_per_launch"], r["bytes_per_launch"]))
    md += ["", "Every kernel of the runs (raw KiB per dispatch):", ""]
    for name in sorted(fetch):
        md.append("- `%s`: FETCH %.1f, WRITE %.1f" % (_short(name), fetch[name], write.get(name, float("nan"))))
    with open(out_md, "w") as f:
        f.write("\n".join(md) + "\n")


if __name__ == "__main__":
    if len(sys.argv) >= 5 and sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif len(sys.argv) >= 9 and sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], sys.argv[6], sys.argv[7], sys.argv[8])
    else:
        print(__doc__, file=sys.stderr)
        sys.exit(2)
