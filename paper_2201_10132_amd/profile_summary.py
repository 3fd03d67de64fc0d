"""Summarise rocprofv3 result databases into short text files under profiles/.

  python paper_2201_10132_amd/profile_summary.py stats <run_results.db> <out.md> [--bench-log <log>] [--also a,b,...] <command>
  python paper_2201_10132_amd/profile_summary.py traffic <fetch.db> <write.db> <kernel-substring> <out.md> [--last N] <command...>

--bench-log: the log of the profiled bench.py run; its HIP-event kernel time
is quoted beside the trace's average.  --also: kernels outside the 15
longest that are listed too (substrings of their names).  --last N: only the last N matching
dispatches (the steps after the launch-shape tuning of the first step).

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


def stats(db, out, command, bench_log=None, also=None):
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage "
                          "from top_kernels order by total_duration desc"))
    # the 15 longest, then any other kernel whose name holds one of `also`
    rows = rows[:15] + [r for r in rows[15:] if any(a in r[0] for a in (also or []))]
    lines = ["# Kernel trace summary", "", f"Command: `{command}`", "",
             "| kernel | calls | total (ms) | average (ms) | % |", "|---|---|---|---|---|"]
    for n, calls, tot, avg, pct in rows:
        lines.append(f"| `{n[:90]}` | {calls} | {tot / 1e3:.1f} | {avg / 1e3:.3f} | {pct:.1f} |")
    if bench_log:
        import json
        import re
        for line in open(bench_log):
            if line.startswith("{"):
                rec = json.loads(line)
                lines += ["", f"bench.py line of the same run: kernel_ms {rec.get('kernel_ms')} "
                          f"(HIP events on the library's stream), launch {rec.get('launch')}"]
            m = re.match(r"# precision=(\d) (\S+) nq=(\d+): .*?([0-9.]+) ms/step", line)
            if m:
                lines.append(f"- bench progress: precision {m.group(1)}, {m.group(2)}, nq {m.group(3)}: "
                             f"{m.group(4)} ms/step")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _per_kernel(db, counter):
    c = sqlite3.connect(db)
    q = ("select kernel_name, grid_size, value from counters_collection "
         "where counter_name = ? order by dispatch_id")
    return list(c.execute(q, (counter,)))


def traffic(fetch_db, write_db, kernel, out, command, copy_bytes=4 * 2 ** 30, last=None):
    f = _per_kernel(fetch_db, "FETCH_SIZE")
    w = _per_kernel(write_db, "WRITE_SIZE")
    cf = max(v for n, g, v in f if "copyBuffer" in n) * 1024.0
    cw = max(v for n, g, v in w if "copyBuffer" in n) * 1024.0
    mf = [(n, v) for n, g, v in f if kernel in n]
    mw = [(n, v) for n, g, v in w if kernel in n]
    if last:
        mf, mw = mf[-last:], mw[-last:]
    names = sorted({n.split("(")[0] for n, _ in mf + mw})
    kf = [v * 1024.0 for n, v in mf]
    kw = [v * 1024.0 for n, v in mw]
    ff, fw = copy_bytes / cf, copy_bytes / cw
    fetch = sum(kf) / len(kf) * ff
    write = sum(kw) / len(kw) * fw
    sha = kernel_source_sha()
    lines = [f"# HBM traffic of `{kernel}`", "", f"Commands: `{command}`", "",
             f"- calibration copy: {copy_bytes / 2**30:.1f} GiB read + written; FETCH_SIZE reads "
             f"{cf / 2**30:.3f} GiB (factor {ff:.3f}), WRITE_SIZE reads {cw / 2**30:.3f} GiB (factor {fw:.3f})",
             f"- dispatches measured: {len(kf)} (fetch run), {len(kw)} (write run) of "
             + ", ".join(f"`{n}`" for n in names),
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


def _option(args, name):
    if name in args:
        i = args.index(name)
        v = args[i + 1]
        del args[i:i + 2]
        return v
    return None


if __name__ == "__main__":
    a = sys.argv[1:]
    if not a:
        raise SystemExit(__doc__)
    if a[0] == "stats":
        log = _option(a, "--bench-log")
        also = _option(a, "--also")
        stats(a[1], a[2], " ".join(a[3:]), bench_log=log, also=also.split(",") if also else None)
    elif a[0] == "traffic":
        last = _option(a, "--last")
        traffic(a[1], a[2], a[3], a[4], " ".join(a[5:]), last=int(last) if last else None)
    else:
        raise SystemExit(__doc__)
