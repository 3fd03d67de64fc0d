"""Summarise rocprofv3 result databases into short text files under profiles/.

  python paper_2201_10132_amd/profile_summary.py stats <run_results.db> <out.md> <command>
  python paper_2201_10132_amd/profile_summary.py traffic <fetch.db> <write.db> <kernel-substring> <out.md> <command...>

The traffic summary calibrates FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
with the largest plain copy dispatch recorded in the same runs (a device copy
of known size made by profile_run.py): factor = copy bytes / counter bytes.
It also writes a one-line machine-readable record next to the summary
(<out>.txt) that bench.py reads for the roofline's "traffic" field.
"""
from __future__ import annotations

import hashlib
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("tpl_kernels.hip", "tpl_internal.h"):
        with open(os.path.join(ROOT, "paper_2201_10132_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stats(db, out, command):
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage "
                          "from top_kernels order by total_duration desc limit 15"))
    lines = ["# Kernel trace summary", "", f"Command: `{command}`", "",
             "| kernel | calls | total (ms) | average (ms) | % |", "|---|---|---|---|---|"]
    for n, calls, tot, avg, pct in rows:
        lines.append(f"| `{n[:90]}` | {calls} | {tot / 1e3:.1f} | {avg / 1e3:.3f} | {pct:.1f} |")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _per_kernel(db, counter):
    c = sqlite3.connect(db)
    q = ("select kernel_name, grid_size, value from counters_collection "
         "where counter_name = ? order by dispatch_id")
    return list(c.execute(q, (counter,)))


def traffic(fetch_db, write_db, kernel, out, command, copy_bytes=4 * 2 ** 30):
    f = _per_kernel(fetch_db, "FETCH_SIZE")
    w = _per_kernel(write_db, "WRITE_SIZE")
    cf = max(v for n, g, v in f if "copyBuffer" in n) * 1024.0
    cw = max(v for n, g, v in w if "copyBuffer" in n) * 1024.0
    kf = [v * 1024.0 for n, g, v in f if kernel in n]
    kw = [v * 1024.0 for n, g, v in w if kernel in n]
    ff, fw = copy_bytes / cf, copy_bytes / cw
    fetch = sum(kf) / len(kf) * ff
    write = sum(kw) / len(kw) * fw
    sha = kernel_source_sha()
    lines = [f"# HBM traffic of `{kernel}`", "", f"Commands: `{command}`", "",
             f"- calibration copy: {copy_bytes / 2**30:.1f} GiB read + written; FETCH_SIZE reads "
             f"{cf / 2**30:.3f} GiB (factor {ff:.3f}), WRITE_SIZE reads {cw / 2**30:.3f} GiB (factor {fw:.3f})",
             f"- dispatches measured: {len(kf)} (fetch run), {len(kw)} (write run)",
             f"- fetched per launch (calibrated): {fetch / 1e9:.3f} GB",
             f"- written per launch (calibrated): {write / 1e9:.3f} GB",
             f"- total per launch: {(fetch + write) / 1e9:.3f} GB",
             f"- kernel sources sha256[:16]: {sha}"]
    open(out, "w").write("\n".join(lines) + "\n")
    rec = os.path.splitext(out)[0] + ".txt"
    open(rec, "w").write(f"kernel {kernel}\nkernel_source_sha {sha}\n"
                         f"fetch_bytes {fetch:.0f}\nwrite_bytes {write:.0f}\n"
                         f"bytes_per_launch {fetch + write:.0f}\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], " ".join(sys.argv[6:]))
    else:
        raise SystemExit(__doc__)
