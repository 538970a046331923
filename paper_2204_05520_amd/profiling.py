"""Summaries of rocprofv3 output databases (rocpd SQLite) for this library.

    python -m paper_2204_05520_amd.profiling stats DB [--match SUBSTR] [--tail N]
        per-kernel dispatch count, total and average duration (markdown);
        --tail N: only the last N dispatches of each kernel (the timed solves,
        after warm-up calls and the autotuner's timing launches)

    python -m paper_2204_05520_amd.profiling traffic FETCH_DB WRITE_DB --match SUBSTR
        --workload NAME --kernel NAME [--tail N] [--json OUT]
        HBM bytes per dispatch of the matching kernel from a FETCH_SIZE run and
        a WRITE_SIZE run, each scaled by what the same counter reads for the
        plain 256 MiB device copy that `bench.py --calib-copy` issues first.

The counters report KiB per dispatch; on this GPU FETCH_SIZE reads about half
of a plain copy's bytes, hence the calibration.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3
import sys

CALIB_BYTES = 256 * 1024 * 1024
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels_dev.h", "kernels.hip", "stage_inst.hip", "odp_dev.h"):
        with open(os.path.join(ROOT, "paper_2204_05520_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_stats(db: str, match: str = "", tail: int = 0):
    c = sqlite3.connect(db)
    if tail <= 0:
        rows = c.execute("select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
                         "from kernels group by name order by sum(duration) desc").fetchall()
        return [r for r in rows if match in r[0]]
    per = {}
    for name, dur in c.execute("select name, duration from kernels order by start"):
        per.setdefault(name, []).append(dur)
    rows = []
    for name, d in per.items():
        d = d[-tail:]
        rows.append((name, len(d), sum(d), sum(d) / len(d), min(d), max(d)))
    rows.sort(key=lambda r: -r[2])
    return [r for r in rows if match in r[0]]


def counter_rows(db: str, counter: str):
    c = sqlite3.connect(db)
    return c.execute("select dispatch_id, kernel_name, value, grid_size from counters_collection "
                     "where counter_name = ? order by dispatch_id", (counter,)).fetchall()


def calibration(rows):
    big = [r for r in rows if r[1] == "__amd_rocclr_copyBuffer" and r[2] * 1024 > CALIB_BYTES / 4]
    if not big:
        raise SystemExit("no calibration copy found (run bench.py with --calib-copy)")
    return CALIB_BYTES / (big[0][2] * 1024.0)


def traffic(fetch_db: str, write_db: str, match: str, tail: int = 0):
    f = counter_rows(fetch_db, "FETCH_SIZE")
    w = counter_rows(write_db, "WRITE_SIZE")
    ff, fw = calibration(f), calibration(w)
    fk = [r[2] * 1024.0 * ff for r in f if match in r[1]]
    wk = [r[2] * 1024.0 * fw for r in w if match in r[1]]
    if tail > 0:
        fk, wk = fk[-tail:], wk[-tail:]
    n = min(len(fk), len(wk))
    if n == 0:
        raise SystemExit(f"no dispatch matches {match!r}")
    fetch = sum(fk[:n]) / n
    write = sum(wk[:n]) / n
    return {"dispatches": n, "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
            "hbm_bytes_per_launch": fetch + write, "copy_factor_fetch": ff, "copy_factor_write": fw}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("db")
    a.add_argument("--match", default="")
    a.add_argument("--tail", type=int, default=0)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_db")
    b.add_argument("write_db")
    b.add_argument("--match", required=True)
    b.add_argument("--workload", required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--alg-bytes-per-launch", type=float, default=0.0)
    b.add_argument("--tail", type=int, default=0, help="only the last N matching dispatches")
    b.add_argument("--json")
    b.add_argument("--command", default="")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print("| kernel | dispatches | total ms | avg us | min us | max us |")
        print("|---|---|---|---|---|---|")
        for name, n, tot, avg, mn, mx in kernel_stats(args.db, args.match, args.tail):
            print(f"| {name.split('(')[0]} | {n} | {tot / 1e6:.3f} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} |")
        return 0
    rec = traffic(args.fetch_db, args.write_db, args.match, args.tail)
    rec.update({"kernel": args.kernel, "workload": args.workload, "match": args.match,
                "kernel_source_hash": kernel_source_hash(), "command": args.command})
    if args.alg_bytes_per_launch > 0:
        rec["alg_bytes_per_launch"] = args.alg_bytes_per_launch
        rec["overfetch"] = rec["hbm_bytes_per_launch"] / args.alg_bytes_per_launch
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(rec, fh, indent=2)
    print(json.dumps(rec, indent=2))
    return 0


if __name__ == "__main__":
    sys.exit(main())
