#!/usr/bin/env python3
"""Traffic summary of a kernel from rocprofv3 counter runs.

Reads the rocpd databases of four `rocprofv3 --pmc` runs (FETCH_SIZE and WRITE_SIZE
of the benchmark, and of a plain 256 MiB device copy for calibration) and the
kernel-trace database of the same benchmark command, and writes the JSON that
bench.py reports as `roofline.traffic` (HBM bytes per launch of the kernel) next to
the trace's average launch duration. --kernel selects the kernel: "cg_coop" (the
one-launch local CG, the step's dominant kernel) or "gemm_jobs" (the batched FP64
MFMA contractions, both tile sizes).

  python -m paper_2507_05222_amd.profile_summary --fetch F.db --write W.db \\
      --cal-fetch CF.db --cal-write CW.db --trace T.db --out profiles/....json [--kernel cg_coop]

`--table T.db [N]` prints the N largest kernels of a kernel-trace database instead.
`--overlap T.db MARKER` splits a kernel trace into calls, each starting at a launch whose
name contains MARKER (launches of one call less than 100 ms apart), and prints per call
the span of its library kernels, their summed durations and the streams they ran on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3

COPY_KIB = 262144.0      # 2^25 doubles
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_05222_amd", "csrc")
# name pattern in the trace, label, and the sources whose hash bench.py checks
KERNELS = {
    "cg_coop": ("k_cg_coop(", "k_cg_coop (one-launch local CG: FP64 MFMA products, vector updates, barriers)",
                ["solve.hip", "device_common.h"]),
    "gemm_jobs": ("k_gemm_jobs<0,", "k_gemm_jobs<0, 32|64> (FP64 MFMA batched contractions, both tile sizes)",
                  ["gemm_jobs.h", "gemm_tile.h"]),
}
KERNEL = KERNELS["gemm_jobs"][0]


def counter(db, name, pattern):
    """(dispatches, mean counter value in KiB) over kernels whose name contains pattern."""
    c = sqlite3.connect(db)
    rows = c.execute("select count(*), avg(counter_value) from pmc_events where counter_name = ? and "
                     "replace(name, ' ', '') like ?", (name, f"%{pattern.replace(' ', '')}%")).fetchone()
    return int(rows[0]), float(rows[1] or 0.0)


def trace_avg_us(db, pattern):
    c = sqlite3.connect(db)
    r = c.execute("select count(*), avg(end - start) from kernels where replace(name, ' ', '') like ?",
                  (f"%{pattern.replace(' ', '')}%",)).fetchone()
    return int(r[0]), float(r[1] or 0.0) / 1e3


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name):
    """A kernel's name without its return type, namespace and parameter list."""
    name = name.replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0][:70]


def kernel_table(db, top=25):
    """Markdown rows (name, launches, total ms, mean us, share of kernel time) of a
    kernel-trace database, largest total first."""
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), sum(end - start), avg(end - start) from kernels group by name "
                     "order by sum(end - start) desc").fetchall()
    tot = sum(r[2] for r in rows)
    lo, hi = c.execute("select min(start), max(end) from kernels").fetchone()
    out = [f"kernel time {tot / 1e6:.1f} ms over a span of {(hi - lo) / 1e6:.1f} ms, "
           f"{sum(r[1] for r in rows)} launches", "",
           "| kernel | launches | total ms | mean us | share |", "|---|---:|---:|---:|---:|"]
    for n, cnt, s, a in rows[:top]:
        out.append(f"| `{short_name(n)}` | {cnt} | {s / 1e6:.1f} | {a / 1e3:.1f} | {100 * s / tot:.1f}% |")
    return "\n".join(out)


def call_overlap(db, marker, gap_ms=100.0):
    """Per call: (launch batches, kernels, span ms, summed kernel ms, streams). A call
    starts at a launch named like `marker`; markers closer than gap_ms join the same
    call, and the call's kernels are the library's (names starting with k_) launched
    before the next call starts."""
    c = sqlite3.connect(db)
    rows = c.execute("select name, start, end, stream_id from kernels order by start").fetchall()
    marks = [r for r in rows if marker in r[0]]
    if not marks:
        return []
    groups, cur = [], [marks[0]]
    for r in marks[1:]:
        if r[1] - cur[-1][1] < gap_ms * 1e6:
            cur.append(r)
        else:
            groups.append(cur)
            cur = [r]
    groups.append(cur)
    starts = [g[0][1] for g in groups] + [rows[-1][2] + 1]
    out = []
    for i, g in enumerate(groups):
        ks = [r for r in rows if starts[i] <= r[1] < starts[i + 1] and short_name(r[0]).startswith("k_")]
        span = (max(r[2] for r in ks) - min(r[1] for r in ks)) / 1e6
        busy = sum(r[2] - r[1] for r in ks) / 1e6
        out.append((len(g), len(ks), span, busy, sorted(set(r[3] for r in ks))))
    return out


def main():
    import sys
    if len(sys.argv) >= 4 and sys.argv[1] == "--overlap":
        print("| call | launch batches | kernels | span ms | summed kernel ms | summed / span | streams |")
        print("|---:|---:|---:|---:|---:|---:|---|")
        for i, (nb, nk, span, busy, st) in enumerate(call_overlap(sys.argv[2], sys.argv[3])):
            print(f"| {i} | {nb} | {nk} | {span:.1f} | {busy:.1f} | {busy / span:.2f} | {st} |")
        return
    if len(sys.argv) >= 3 and sys.argv[1] == "--table":
        print(kernel_table(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25))
        return
    ap = argparse.ArgumentParser()
    for a in ("fetch", "write", "cal_fetch", "cal_write", "trace", "out"):
        ap.add_argument("--" + a.replace("_", "-"), required=True)
    ap.add_argument("--workload", default="cylinder O-grid 2^10x2^10, chi=64, mixed path")
    ap.add_argument("--kernel", default="cg_coop", choices=sorted(KERNELS))
    a = ap.parse_args()
    pat, label, files = KERNELS[a.kernel]
    nf, fetch = counter(a.fetch, "FETCH_SIZE", pat)
    nw, write = counter(a.write, "WRITE_SIZE", pat)
    _, cf = counter(a.cal_fetch, "FETCH_SIZE", "copyBuffer")
    _, cw = counter(a.cal_write, "WRITE_SIZE", "copyBuffer")
    nt, avg = trace_avg_us(a.trace, pat)
    out = {
        "kernel": label,
        "workload": a.workload,
        "dispatches": nf, "dispatches_write_run": nw,
        "fetch_kib_per_dispatch": round(fetch, 3), "write_kib_per_dispatch": round(write, 3),
        "copy_kib": COPY_KIB, "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_factor": round(COPY_KIB / cf, 4), "write_factor": round(COPY_KIB / cw, 4),
        "kernel_source_sha256_16": source_hash(files),
        "kernel_trace_avg_us": round(avg, 2), "kernel_trace_dispatches": nt,
    }
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
