"""Measurement helpers (not used by the library itself).

    python -m paper_2301_05726_amd.profiling copy [--mib 512] [--reps 4]
        A plain device-to-device copy of known size, run under
        `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` to calibrate what the
        counters report per byte actually moved.

    python -m paper_2301_05726_amd.profiling peaks [--gib 4] [--reps 5]
        Achievable device peaks to hold the kernels against: a streaming copy
        (GB/s) and a random gather of 8-byte elements over a buffer the size of
        a large hash table (elements/s), timed with HIP events on torch's own
        copy and gather kernels.

    python -m paper_2301_05726_amd.profiling summarize <csv> [--top N] [--cmd "..."]
        Turn a rocprofv3 kernel_stats.csv or counter_collection.csv into a
        short text table (per-kernel calls, total and mean duration, or mean
        counter value per dispatch).

    python -m paper_2301_05726_amd.profiling distribution <kernel_trace.csv> [--kernels k_fwd,k_rev] [--parts 8]
        Per-launch duration percentiles of the sweep kernels, and their median
        along the sweep, from a rocprofv3 --kernel-trace CSV.

    python -m paper_2301_05726_amd.profiling reduce <csv> <out.csv>
        Sum a rocprofv3 counter_collection.csv into one row per kernel and
        counter (the input of `traffic` may be either form).

    python -m paper_2301_05726_amd.profiling traffic --fetch <csv> --write <csv>
            --cal-fetch <csv> --cal-write <csv> --cal-mib M --cal-reps R [--cmd "..."]
        HBM bytes per dispatch of each kernel: FETCH_SIZE and WRITE_SIZE (KiB
        per dispatch, one rocprofv3 pass each) scaled by what the same counters
        read for the plain copy above; prints `traffic_kib <kernel> <KiB>` lines
        and the hash of the kernel sources they were measured on.
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


def peaks(gib: float, reps: int) -> None:
    import torch
    dev = torch.device("cuda")
    n8 = int(gib * (1 << 30)) // 8
    src = torch.randint(0, 1 << 62, (n8,), dtype=torch.int64, device=dev)
    dst = torch.empty_like(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            ev[0].record()
            fn()
            ev[1].record()
            torch.cuda.synchronize()
            best = min(best, ev[0].elapsed_time(ev[1]) * 1e-3)
        return best

    t = timed(lambda: dst.copy_(src))
    print(f"copy {gib:g} GiB: {2 * n8 * 8 / t / 1e9:.0f} GB/s (read + write), best of {reps}", flush=True)
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    m = min(n8 // 4, 1 << 24)
    idx = torch.randint(0, n8, (m,), dtype=torch.int64, device=dev, generator=g)
    t = timed(lambda: torch.take(src, idx))
    print(f"random gather of 8-byte elements over {gib:g} GiB: {m / t / 1e9:.2f} G elements/s, "
          f"{m * 8 / t / 1e9:.0f} GB/s useful (plus {m * 16 / t / 1e9:.0f} GB/s of index reads and "
          f"output writes, streamed)", flush=True)
    del src, dst, idx
    # the floor of a dependent chain of launches: a captured graph of tiny
    # kernels, each on one element (what a sweep step costs with no work)
    nodes = 1000
    x = torch.zeros(1, device=dev)
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        x.add_(1.0)  # warm the kernel before capture
    torch.cuda.current_stream(dev).wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(nodes):
            x.add_(1.0)
    t = timed(graph.replay)
    torch.cuda.synchronize()
    print(f"graph of {nodes} one-element kernels: {t / nodes * 1e6:.2f} us per node "
          f"(x = {x.item():.0f}, expected {1 + (1 + reps) * nodes}: every node ran)", flush=True)
    # the same chain of launches, each node reading and writing a whole
    # table-sized buffer once (2 MiB: the 20-qubit table; 8 MiB: 64 qubits)
    for mib in (2, 8):
        y = torch.zeros(mib * (1 << 20) // 4, device=dev)
        with torch.cuda.stream(side):
            y.add_(1.0)
        torch.cuda.current_stream(dev).wait_stream(side)
        gy = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gy):
            for _ in range(nodes):
                y.add_(1.0)
        t = timed(gy.replay)
        torch.cuda.synchronize()
        ok = float(y[0].item()) == 1 + (1 + reps) * nodes
        print(f"graph of {nodes} kernels each streaming {mib} MiB (read + write): {t / nodes * 1e6:.2f} us per node, "
              f"{2 * mib * (1 << 20) / (t / nodes) / 1e9:.0f} GB/s (every node ran: {ok})", flush=True)
        del gy, y


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


def _mean_per_kernel(path: str, counter: str) -> dict:
    """Mean counter value per dispatch of each kernel, from a rocprofv3
    counter_collection.csv or from its `reduce`d form."""
    acc = defaultdict(lambda: [0.0, 0])
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", counter) != counter:
            continue
        name = _short(r.get("Kernel_Name", r.get("Kernel-Name", "?")))
        key = name.replace("swc::", "").split("<")[0]
        if "Counter_Sum" in r:
            acc[key][0] += float(r["Counter_Sum"])
            acc[key][1] += int(r["Dispatches"])
        else:
            acc[key][0] += float(r.get("Counter_Value", 0.0))
            acc[key][1] += 1
    return {k: (v[0] / v[1], v[1]) for k, v in acc.items()}


def distribution(path: str, kernels: list, parts: int, cmd) -> None:
    """Per-launch durations of the named kernels from a rocprofv3
    kernel_trace.csv: percentiles over all launches, then the median of each
    of `parts` equal runs of consecutive launches (how the duration moves
    along a sweep as the state grows)."""
    import numpy as np
    dur = defaultdict(list)
    for r in csv.DictReader(open(path)):
        name = _short(r.get("Kernel_Name", "?")).replace("swc::", "").split("<")[0]
        if name in kernels:
            dur[name].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    if cmd:
        for c in cmd:
            print(f"# command: {c}")
    for k in kernels:
        if not dur[k]:
            continue
        d = np.array([x[1] for x in sorted(dur[k])], dtype=np.float64) / 1e3  # launch order, us
        q = np.percentile(d, [1, 10, 50, 90, 99, 99.9])
        print(f"{k}: {d.size} launches, mean {d.mean():.3f} us; percentiles 1/10/50/90/99/99.9: "
              + " / ".join(f"{v:.2f}" for v in q) + f"; max {d.max():.2f} us")
        meds = [np.median(c) for c in np.array_split(d, parts)]
        print(f"  median per 1/{parts} of the launches in order: " + " ".join(f"{v:.2f}" for v in meds))


def reduce_counters(path: str, out: str) -> None:
    """Sum a counter_collection.csv (one row per dispatch and counter) into
    one row per kernel and counter, so a run of many dispatches keeps a
    small file."""
    acc = defaultdict(lambda: [0.0, 0])
    for r in csv.DictReader(open(path)):
        key = (r.get("Kernel_Name", r.get("Kernel-Name", "?")), r.get("Counter_Name", "?"))
        acc[key][0] += float(r.get("Counter_Value", 0.0))
        acc[key][1] += 1
    with open(out, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Sum", "Dispatches"])
        for (k, c), (v, n) in sorted(acc.items()):
            w.writerow([k, c, repr(v), n])
    print(f"{path}: {sum(n for _, n in acc.values())} rows -> {len(acc)} kernels/counters in {out}")


def sources_sha() -> str:
    import hashlib
    import os
    h = hashlib.sha256()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for f in ("swc_kernels.hip", "swc_api.hip", "swc_internal.h", "swc_noalloc.hip"):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def traffic(a) -> None:
    fetch, write = _mean_per_kernel(a.fetch, "FETCH_SIZE"), _mean_per_kernel(a.write, "WRITE_SIZE")
    cf, cw = _mean_per_kernel(a.cal_fetch, "FETCH_SIZE"), _mean_per_kernel(a.cal_write, "WRITE_SIZE")
    moved_kib = a.cal_mib * 1024.0  # per copy: read this much and write this much
    # the copy kernel is the one dispatch of the calibration run with the most traffic
    cfk = max(cf.values(), key=lambda x: x[0])[0]
    cwk = max(cw.values(), key=lambda x: x[0])[0]
    ff, fw = moved_kib / cfk, moved_kib / cwk
    if a.cmd:
        for c in a.cmd:
            print(f"# command: {c}")
    print(f"# calibration: {a.cal_mib} MiB device copy: FETCH_SIZE {cfk:.1f} KiB -> factor {ff:.3f}; "
          f"WRITE_SIZE {cwk:.1f} KiB -> factor {fw:.3f}")
    print(f"# kernel sources sha256[:16]: {sources_sha()}")
    print(f"{'kernel':28s} {'dispatches':>10s} {'FETCH_KiB':>12s} {'WRITE_KiB':>12s} {'traffic_KiB':>12s}")
    rows = []
    for k in sorted(set(fetch) | set(write), key=lambda k: -(fetch.get(k, (0, 0))[0] + write.get(k, (0, 0))[0])):
        fv, n = fetch.get(k, (0.0, 0))
        wv, _ = write.get(k, (0.0, 0))
        t = fv * ff + wv * fw
        rows.append((k, t))
        print(f"{k:28s} {n:10d} {fv:12.1f} {wv:12.1f} {t:12.1f}")
    # the one-factor steps over all their builds (the plain ones, the forward's
    # high-occupancy build on large indexes, those probing through the
    # presence filter), weighted by dispatches: what bench.py's k_fwd and
    # k_rev lines average over
    for step, builds in (("k_fwd_step", ("k_fwd", "k_fwd_ho", "k_fwd_pf", "k_fwd_ho_pf")),
                         ("k_rev_step", ("k_rev", "k_rev_pf"))):
        parts = [k for k in builds if k in fetch and k in write]
        if not parts:
            continue
        n = sum(fetch[k][1] for k in parts)
        t = sum((fetch[k][0] * ff + write[k][0] * fw) * fetch[k][1] for k in parts) / n
        rows.append((step, t))
        print(f"{step + ' (all builds)':28s} {n:10d} {'':12s} {'':12s} {t:12.1f}")
    print("# per dispatch, calibrated (read by bench.py while the sources are unchanged):")
    for k, t in rows:
        print(f"traffic_kib {k} {t:.1f}")
    print(f"sources_sha {sources_sha()}")


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="sub", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=512)
    c.add_argument("--reps", type=int, default=4)
    s = sub.add_parser("summarize")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=12)
    s.add_argument("--cmd", default=None)
    pk = sub.add_parser("peaks")
    pk.add_argument("--gib", type=float, default=4.0)
    pk.add_argument("--reps", type=int, default=5)
    t = sub.add_parser("traffic")
    for f in ("--fetch", "--write", "--cal-fetch", "--cal-write"):
        t.add_argument(f, required=True)
    t.add_argument("--cal-mib", type=int, default=512)
    t.add_argument("--cmd", action="append")
    ds = sub.add_parser("distribution")
    ds.add_argument("csv")
    ds.add_argument("--kernels", default="k_fwd,k_rev")
    ds.add_argument("--parts", type=int, default=8)
    ds.add_argument("--cmd", action="append")
    rd = sub.add_parser("reduce")
    rd.add_argument("csv")
    rd.add_argument("out")
    a = ap.parse_args(argv)
    if a.sub == "copy":
        copy_kernel(a.mib, a.reps)
    elif a.sub == "peaks":
        peaks(a.gib, a.reps)
    elif a.sub == "traffic":
        traffic(a)
    elif a.sub == "reduce":
        reduce_counters(a.csv, a.out)
    elif a.sub == "distribution":
        distribution(a.csv, a.kernels.split(","), a.parts, a.cmd)
    else:
        summarize(a.csv, a.top, a.cmd)
    return 0


if __name__ == "__main__":
    sys.exit(main())
