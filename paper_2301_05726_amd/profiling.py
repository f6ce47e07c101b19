"""Measurement helpers (not used by the library itself).

    python -m paper_2301_05726_amd.profiling copy [--mib 512] [--reps 4]
        A plain device-to-device copy of known size, run under
        `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` to calibrate what the
        counters report per byte actually moved.

    python -m paper_2301_05726_amd.profiling summarize <csv> [--top N] [--cmd "..."]
        Turn a rocprofv3 kernel_stats.csv or counter_collection.csv into a
        short text table (per-kernel calls, total and mean duration, or mean
        counter value per dispatch).
"""
from __future__ import annotations

import argparse
import csv
import sys
from collections import defaultdict


def copy_kernel(mib: int, reps: int) -> None:
    import torch
    n = mib * (1 << 20)
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps} (each copy reads {n} B and writes {n} B)", flush=True)


def _short(name: str) -> str:
    name = name.split("(")[0]
    return name.replace("void ", "")


def summarize(path: str, top: int, cmd: str | None) -> None:
    rows = list(csv.DictReader(open(path)))
    if cmd:
        print(f"# command: {cmd}")
    print(f"# source: {path.split('/')[-1]}")
    if rows and "TotalDurationNs" in rows[0]:
        rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
        tot = sum(float(r["TotalDurationNs"]) for r in rows)
        print(f"{'kernel':60s} {'calls':>8s} {'total_ms':>10s} {'avg_us':>10s} {'pct':>6s}")
        for r in rows[:top]:
            t = float(r["TotalDurationNs"])
            print(f"{_short(r['Name'])[:60]:60s} {int(r['Calls']):8d} {t / 1e6:10.3f} "
                  f"{float(r['AverageNs']) / 1e3:10.3f} {100 * t / tot:6.2f}")
        return
    # counter collection: mean counter value per dispatch and kernel
    acc = defaultdict(lambda: [0.0, 0])
    for r in rows:
        key = (_short(r.get("Kernel_Name", r.get("Kernel-Name", "?"))), r.get("Counter_Name", "?"))
        acc[key][0] += float(r.get("Counter_Value", 0.0))
        acc[key][1] += 1
    items = sorted(acc.items(), key=lambda kv: -kv[1][0])
    print(f"{'kernel':60s} {'counter':>12s} {'dispatch':>9s} {'mean/dispatch':>14s}")
    for (k, c), (s, n) in items[:top]:
        print(f"{k[:60]:60s} {c:>12s} {n:9d} {s / n:14.1f}")


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=512)
    c.add_argument("--reps", type=int, default=4)
    s = sub.add_parser("summarize")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=12)
    s.add_argument("--cmd", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        copy_kernel(a.mib, a.reps)
    else:
        summarize(a.csv, a.top, a.cmd)
    return 0


if __name__ == "__main__":
    sys.exit(main())
