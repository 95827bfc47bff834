"""Condense rocprofv3 output into the text summaries kept in this folder.

    python profiles/summarize.py stats  <kernel_stats.csv>  "<command that produced it>"
    python profiles/summarize.py pmc    <counter_collection.csv> <COUNTER> [copy_bytes]

`stats` prints per-kernel call count and average/total duration.  `pmc`
prints the per-kernel average of a byte counter (FETCH_SIZE / WRITE_SIZE are
reported in KiB per dispatch) and, when the plain copy kernel of copy_bytes
bytes is in the trace, the factor that maps the counter onto true bytes.
"""

import csv
import sys
from collections import defaultdict


def short(name):
    name = name.split("(")[0]
    for pre in ("void ", "dks::"):
        name = name.replace(pre, "")
    return name[:60]


def stats(path, cmd):
    rows = list(csv.DictReader(open(path)))
    print(f"# rocprofv3 --kernel-trace --stats\n# command: {cmd}\n")
    print(f"{'kernel':60s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        print(f"{short(r['Name']):60s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
              f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")


def pmc(path, counter, copy_bytes=None):
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", counter) != counter:
            continue
        acc[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    print(f"# rocprofv3 --pmc {counter} (KiB per dispatch, averaged)\n")
    factor = None
    if copy_bytes:
        for k, v in acc.items():
            if "copy" in k.lower() or "elementwise" in k.lower():
                kib = sum(v) / len(v)
                if kib > 0.5 * copy_bytes / 1024:
                    factor = (copy_bytes / 1024) / kib
                    print(f"# copy calibration: {k}: {kib:.0f} KiB for {copy_bytes / 1024:.0f} KiB -> factor {factor:.4f}\n")
                    break
    for k, v in sorted(acc.items(), key=lambda kv: -sum(kv[1]) / len(kv[1])):
        kib = sum(v) / len(v)
        scaled = f"{kib * factor / 1024:12.1f} MiB" if factor else ""
        print(f"{k:60s} {len(v):5d} {kib:14.0f} KiB {scaled}")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3])
    else:
        pmc(sys.argv[2], sys.argv[3], float(sys.argv[4]) if len(sys.argv) > 4 else None)
