"""Condense rocprofv3 output (its rocpd SQLite database) into the text
summaries kept in this folder.

    python profiles/summarize.py stats <results.db> "<command that produced it>"
    python profiles/summarize.py pmc   <results.db> <COUNTER> "<command>" [copy_bytes]
    python profiles/summarize.py traffic <fetch.db> <write.db> <copy_bytes> "<command>" <out.json>

`stats` prints per-kernel call count and average/total duration.  `pmc`
prints the per-kernel average of a counter per dispatch; for FETCH_SIZE and
WRITE_SIZE (KiB per dispatch) it also prints the factor that maps the counter
onto true bytes, taken from the plain device copy of copy_bytes bytes that the
profiled command ran (the torch elementwise copy kernel).
"""

import sqlite3
import sys
from collections import defaultdict


def short(name):
    name = name.split("(")[0]
    for pre in ("void ", "dks::"):
        name = name.replace(pre, "")
    return name[:64]


def stats(db, cmd):
    """Per-kernel durations from the raw dispatch records (end - start, ns)."""
    c = sqlite3.connect(db)
    acc = defaultdict(list)
    for name, dur in c.execute("select name, duration from kernels"):
        acc[short(name)].append(float(dur))
    total_all = sum(sum(v) for v in acc.values())
    print("# rocprofv3 --kernel-trace --stats")
    print(f"# command: {cmd}\n")
    print(f"{'kernel':64s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}")
    for k, v in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
        print(f"{k:64s} {len(v):6d} {sum(v) / len(v) / 1e3:10.2f} {sum(v) / 1e6:10.3f} "
              f"{100 * sum(v) / total_all:6.2f}")


def pmc(db, counter, cmd, copy_bytes=None):
    c = sqlite3.connect(db)
    cols = [r[1] for r in c.execute("pragma table_info('counters_collection')")]
    name_col = "kernel_name" if "kernel_name" in cols else "name"
    q = (f"select {name_col}, counter_name, value from counters_collection where counter_name = ?")
    acc = defaultdict(list)
    for name, _, value in c.execute(q, (counter,)):
        acc[short(name)].append(float(value))
    print(f"# rocprofv3 --pmc {counter} (value per dispatch, averaged over dispatches)")
    print(f"# command: {cmd}\n")
    factor = None
    if copy_bytes:
        # the runtime's device-to-device copy kernel (torch's tensor.copy_)
        for k, v in acc.items():
            if "copybuffer" in k.lower():
                kib = sum(v) / len(v)
                factor = (copy_bytes / 1024) / kib
                print(f"# copy calibration: {k}: {kib:.0f} KiB counted for {copy_bytes / 1024:.0f} KiB "
                      f"moved -> factor {factor:.4f}\n")
                break
    for k, v in sorted(acc.items(), key=lambda kv: -sum(kv[1]) / len(kv[1])):
        avg = sum(v) / len(v)
        scaled = f"{avg * factor / 1024:12.1f} MiB (scaled)" if factor else ""
        print(f"{k:64s} {len(v):5d} {avg:14.0f} {scaled}")


SOURCES = ("paper_1509_07685_amd/csrc/bin_kernels.hip", "paper_1509_07685_amd/csrc/fft_kernels.hip",
           "paper_1509_07685_amd/csrc/fft_engine.h", "paper_1509_07685_amd/csrc/particle_kernels.hip",
           "paper_1509_07685_amd/csrc/dks_internal.h")


def source_hashes(root):
    import hashlib
    import os
    return {f: hashlib.sha256(open(os.path.join(root, f), "rb").read()).hexdigest() for f in SOURCES}


def per_kernel(db, counter):
    c = sqlite3.connect(db)
    cols = [r[1] for r in c.execute("pragma table_info('counters_collection')")]
    name_col = "kernel_name" if "kernel_name" in cols else "name"
    acc = defaultdict(list)
    for name, value in c.execute(f"select {name_col}, value from counters_collection where counter_name = ?",
                                 (counter,)):
        acc[short(name).split("<")[0]].append(float(value))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def traffic(fetch_db, write_db, copy_bytes, cmd, out):
    """HBM bytes per dispatch of each kernel: FETCH_SIZE and WRITE_SIZE (KiB),
    each scaled by the factor that maps the same counter onto the bytes the
    runtime's device copy of copy_bytes moved.  Written as JSON with the
    hashes of the kernel sources measured, so a reader can tell whether the
    figures still describe the code."""
    import json
    import os
    f, w = per_kernel(fetch_db, "FETCH_SIZE"), per_kernel(write_db, "WRITE_SIZE")
    copy = [k for k in f if "copyBuffer" in k][0]
    ff = copy_bytes / 1024 / f[copy]
    fw = copy_bytes / 1024 / w[copy]
    kern = {k: {"fetch_bytes": f[k] * 1024 * ff, "write_bytes": w.get(k, 0.0) * 1024 * fw}
            for k in f if k.startswith("k_")}
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    doc = {"command": cmd, "copy_bytes": copy_bytes, "fetch_factor": ff, "write_factor": fw,
           "sources_sha256": source_hashes(root), "kernels": kern}
    with open(out, "w") as fh:
        json.dump(doc, fh, indent=1, sort_keys=True)
    print(json.dumps({k: {a: round(b / 2 ** 20, 1) for a, b in v.items()} for k, v in kern.items()}, indent=1))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5], sys.argv[6])
    else:
        pmc(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]) if len(sys.argv) > 5 else None)
