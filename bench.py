#!/usr/bin/env python3
"""Benchmark of the sparse wavefunction UCC circuit on one MI355X.

One step = one energy_and_grad call: forward sweep of all UCC factors with
truncation, sigma = H psi and E, and the adjoint sweep giving dE/dtheta,
for one theta vector of the workload, inputs already resident in HBM.

    python bench.py [--steps K] [--warmup W] [--workload q64] [--prec fp64]

The default workload is the 64-qubit one (32 electrons, all 94,848 factors of
spin-conserving UCCSD, threshold 1e-4, hash capacity 2^28, checkpoints every
4096 factors) with FP64 amplitudes: the largest configuration, whose energy
the FP64 path gives within 1e-6 Ha.

Prints one JSON line.  Besides the step rate it reports the forward
det-update rate, the same-GPU FP64 forward + central finite-difference
gradient rate (extrapolated from sampled parameters), the roofline figures
of the dominant kernel from HIP events, the FP32-amplitude path's rate and
its difference from the timed path, parity against the CPU oracle (the whole
circuit up to 20 qubits, a prefix of it above), and the CPU oracle timed on
the host.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("det-updates/s (UCC forward); E+∇E evals/s adjoint vs FD, 1 MI355X, ΔE≤1e-6")
HBM_PEAK_GBS = 8000.0


def rotate_bytes(st: dict, tsz: int) -> float:
    """Algorithmic bytes of one forward sweep's rotate kernels: 8 B key per
    visited determinant; per rotated pair the own amplitude read+write and
    an 8 B partner-key probe; partner amplitude read+write when it exists;
    key + amplitude per inserted determinant."""
    return (8.0 * st["det_updates"] + st["pair_updates"] * (2 * tsz + 8) + st["partner_hits"] * 2 * tsz
            + st["inserts"] * (8 + tsz))




def measured_traffic(workload: str, prec: str) -> dict:
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (calibrated against a copy kernel), only while the kernel sources
    are the ones that were profiled; otherwise empty (traffic reported null)."""
    from paper_2301_05726_amd.profiling import sources_sha
    path = os.path.join(ROOT, "profiles", f"sweep_kernels_{workload}_{prec}_traffic.txt")
    if not os.path.exists(path):
        return {}
    vals, sha = {}, None
    for line in open(path):
        parts = line.split()
        if len(parts) == 3 and parts[0] == "traffic_kib":
            vals[parts[1]] = float(parts[2]) * 1024.0
        elif len(parts) == 2 and parts[0] == "sources_sha":
            sha = parts[1]
    return vals if sha == sources_sha() else {}


def state_difference(s64, s32, theta, exc, thr, h1, h2) -> dict:
    """Final states (member 0) of the FP64 and FP32 paths after the same
    forward sweep: the determinants only one of them kept (truncation
    decisions that rounding moved across the cut, and their descendants),
    the amplitude differences on the determinants both kept, and the energy
    difference split exactly into those two parts.  With X|c the state X
    restricted to the common determinants, every energy evaluated by the FP64
    path (build_state + energy):
        E(32) - E(64) = [E(32) - E(32|c)] - [E(64) - E(64|c)]   (decisions)
                      + [E(32|c) - E(64|c)]                      (rounding)"""
    import numpy as np
    out = {}
    for name, s in (("fp64", s64), ("fp32", s32)):
        s.apply_ucc(theta, exc, thr)
        out[name] = s.get_state(0)
        s.build_state()
    (d64, a64), (d32, a32) = out["fp64"], out["fp32"]
    both, i64, i32 = np.intersect1d(d64, d32, assume_unique=True, return_indices=True)
    diff = np.abs(a64[i64] - a32[i32])
    only64 = np.setdiff1d(np.arange(d64.size), i64)
    only32 = np.setdiff1d(np.arange(d32.size), i32)

    def energy(d, a):
        s64.build_state(d, a)
        return float(s64.energy(h1, h2)[0].item())

    E64, E32 = energy(d64, a64), energy(d32, a32)
    E64c, E32c = energy(both, a64[i64]), energy(both, a32[i32])
    s64.build_state()
    return {
        "dE": E32 - E64,
        "dE_decisions": (E32 - E32c) - (E64 - E64c),
        "dE_rounding": E32c - E64c,
        "n_fp64": int(d64.size), "n_fp32": int(d32.size),
        "only_fp64": int(only64.size), "only_fp32": int(only32.size),
        "max_abs_amp_only": float(max(np.max(np.abs(a64[only64]), initial=0.0),
                                      np.max(np.abs(a32[only32]), initial=0.0))),
        "weight_only": float(np.sum(a64[only64] ** 2) + np.sum(a32[only32] ** 2)),
        "max_abs_amp_diff_common": float(np.max(diff, initial=0.0)),
        "rms_amp_diff_common": float(np.sqrt(np.mean(diff ** 2))) if diff.size else 0.0,
    }


def random_read_rate(dev, gib: float = 1.0, reps: int = 3) -> float:
    """Random reads the device serves per second (G/s): torch's gather of
    8-byte elements at uniformly random positions of a `gib` GiB buffer (best
    of `reps`, HIP events).  The index reads and the output writes are
    streamed, so this is a slightly conservative ceiling for kernels whose
    accesses land at random places of a table this size."""
    import torch
    n = int(gib * (1 << 30)) // 8
    src = torch.zeros(n, dtype=torch.int64, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    m = 1 << 24
    idx = torch.randint(0, n, (m,), dtype=torch.int64, device=dev, generator=g)
    torch.take(src, idx)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best = float("inf")
    for _ in range(reps):
        ev[0].record()
        torch.take(src, idx)
        ev[1].record()
        torch.cuda.synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]) * 1e-3)
    del src, idx
    return m / best / 1e9


def graph_node_floor_us(dev, nodes: int = 1000, reps: int = 5) -> float:
    """Mean time per node of a captured graph of `nodes` one-element kernels
    (best of `reps` replays), measured with HIP events."""
    import torch
    x = torch.zeros(1, device=dev)
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        x.add_(1.0)  # the kernel loaded before the capture
    torch.cuda.current_stream(dev).wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(nodes):
            x.add_(1.0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best = float("inf")
    for _ in range(reps):
        ev[0].record()
        graph.replay()
        ev[1].record()
        torch.cuda.synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]) * 1e3 / nodes)
    del graph
    return best


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def reverse_bytes(st: dict, tsz: int) -> float:
    """Algorithmic bytes of one reverse sweep, counted on the forward's
    pairs (the reverse visits the same pairs): 8 B key per visited
    determinant; per pair the own amplitude and adjoint read+write and an
    8 B partner-key probe; partner amplitude and adjoint read+write when it
    exists; created entries are removed (one 4 B state write)."""
    return (8.0 * st["det_updates"] + st["pair_updates"] * (4 * tsz + 8) + st["partner_hits"] * 4 * tsz
            + st["inserts"] * 4)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="q64")
    ap.add_argument("--prec", default="fp64", choices=["fp32", "fp64"])
    ap.add_argument("--fd-params", type=int, default=32)
    ap.add_argument("--no-fd", action="store_true")
    ap.add_argument("--fd-max-s", type=float, default=90.0,
                    help="time budget of the sampled finite-difference parameters (at least two are timed)")
    ap.add_argument("--fd-full-max-s", type=float, default=60.0,
                    help="run the finite differences over every parameter when the sampled estimate is below this")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--factors", type=int, default=0, help="keep only the first K factors (0: all)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="beyond 20 qubits the CPU oracle evaluates E+grad on ever longer prefixes of the circuit "
                         "(x2 factors each) until one takes at least this long; the GPU is compared with it there")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the FP32-amplitude rate and accuracy reported beside an FP64 run")
    ap.add_argument("--batch", type=int, default=1, help="theta vectors per call")
    ap.add_argument("--capacity-log2", type=int, default=0, help="hash capacity 2^c (0: the workload's)")
    ap.add_argument("--log-capacity-log2", type=int, default=0, help="truncation-log records 2^c (0: capacity)")
    ap.add_argument("--topk", default="", help="N_MAX,N_CUT truncation after every factor (paper's rule)")
    ap.add_argument("--entropy", action="store_true", help="track the entropy (Eq. 6) after every factor")
    ap.add_argument("--threshold", type=float, default=-1.0,
                    help="truncation threshold (default: the workload's)")
    ap.add_argument("--sigma-scratch-gib", type=float, default=-1.0,
                    help="device scratch for sigma by pairing (0: hash probes)")
    ap.add_argument("--sigma-mode", type=int, default=0, help="pairing: 0 auto, 1 always, 2 never")
    ap.add_argument("--fp64-check", action="store_true",
                    help="also run one FP64 energy_and_grad and report its differences from the timed path")
    ap.add_argument("--checkpoint-interval", type=int, default=-1,
                    help="snapshot psi every K factors of the gradient sweep (0: off; -1: 4096 at 64 qubits, "
                         "else off)")
    ap.add_argument("--checkpoint-entries-log2", type=int, default=24,
                    help="live determinants per snapshot the checkpoint buffer holds, 2^c")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(batch members and finite-difference parameters would shard across GPUs with only a gather "
              "of E and g); run it with --gpus 1", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    from paper_2301_05726_amd import swc, synth

    wl = synth.WORKLOADS[args.workload]
    if args.threshold >= 0.0:
        wl = dataclasses.replace(wl, threshold=args.threshold)
    if args.checkpoint_interval < 0:
        args.checkpoint_interval = 4096 if wl.name == "q64" else 0
    p = synth.make_problem(wl, batch=args.batch, n_factors=args.factors or None)
    B = args.batch
    cap = (1 << args.capacity_log2) if args.capacity_log2 else wl.capacity
    if args.sigma_scratch_gib < 0:
        # large states: the doubles of sigma by pairing (32 GiB of scratch);
        # small ones: by probes, which cost less there
        args.sigma_scratch_gib = 32.0 if cap >= (1 << 26) else 0.0
    nq, M = wl.n_qubits, p.M
    prec = swc.FP32 if args.prec == "fp32" else swc.FP64
    tsz = 4 if prec == swc.FP32 else 8
    dev = torch.device("cuda:0")
    theta = torch.tensor(p.theta, dtype=torch.float64, device=dev)
    h1 = torch.tensor(p.h1, dtype=torch.float64, device=dev)
    h2 = torch.tensor(p.h2, dtype=torch.float64, device=dev)

    logcap = (1 << args.log_capacity_log2) if args.log_capacity_log2 else 0
    s = swc.Solver(nq, wl.n_occ, wl.n_occ, cap, prec=prec, batch=B, max_factors=M, log_capacity=logcap, device=dev)
    topk = tuple(int(x) for x in args.topk.split(",")) if args.topk else None
    if topk:
        s.set_topk(*topk)
    if args.entropy:
        s.track_entropy(True)
    if args.sigma_scratch_gib > 0:
        s.set_sigma_scratch(int(args.sigma_scratch_gib * (1 << 30)), mode=args.sigma_mode)
    if args.checkpoint_interval > 0:
        s.set_checkpoints(args.checkpoint_interval, 1 << args.checkpoint_entries_log2)
    s.build_state()

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    tw = time.perf_counter()
    for i in range(args.warmup):
        s.energy_and_grad(theta, p.exc, wl.threshold, h1, h2)
        torch.cuda.synchronize()
        progress(f"warmup {i + 1}/{args.warmup} done, {time.perf_counter() - tw:.1f} s")
    torch.cuda.synchronize()
    # HIP events recorded by the library on its stream bracket each sweep
    # (forward, reverse) and the sigma kernel inside every timed step; the
    # library sums them over its calls, read before and after the timed steps
    st0 = s.stats()
    t0 = time.perf_counter()
    t_said = t0
    for i in range(args.steps):
        E, g = s.energy_and_grad(theta, p.exc, wl.threshold, h1, h2)
        # a line per step only when steps are slow (the host print would
        # otherwise sit between the steps of the timed region)
        now = time.perf_counter()
        if now - t_said > 5.0 or i + 1 == args.steps:
            progress(f"step {i + 1}/{args.steps} done")
            t_said = now
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    st = s.stats()
    assert st["grad_calls"] - st0["grad_calls"] == args.steps
    fwd_ms = st["fwd_ms_total"] - st0["fwd_ms_total"]
    rev_ms = st["rev_ms_total"] - st0["rev_ms_total"]
    sig_ms = st["sigma_kernel_ms_total"] - st0["sigma_kernel_ms_total"]
    n_fwd, n_rev = st["rotate_launches"], st["reverse_launches"]
    log_records = st["log_records"]
    ck_taken = st["checkpoints"]
    scans = {"forward": st["fwd_slots_scanned"], "reverse": st["rev_slots_scanned"], "index_growths": st["rehashes"]}
    value = args.steps * B / elapsed  # theta vectors evaluated per second
    E0 = float(E[0].item())
    g0 = g.cpu().numpy()[0]

    # forward sweep statistics of one step (identical every step), with the
    # live count of every step
    s.track_live(True)
    s.apply_ucc(theta, p.exc, wl.threshold)
    st = s.stats()
    progress("statistics sweep done")
    n_live = st["n_live"]
    traj = s.live_counts(0)  # live determinants before each factor, then after the last
    marks = sorted({int(round(M * q / 8)) for q in range(9)})
    live_traj = {"factor": marks, "n_live": [int(traj[k]) for k in marks], "max": int(traj.max())}
    det_updates = st["det_updates"]
    s.build_state()

    # sweep kernels run back to back on the stream (one or, at threshold 0,
    # two factors per launch), so the mean launch duration is the bracketed
    # sweep time / launches
    per_step = {"forward_sweep": fwd_ms / args.steps, "reverse_sweep": rev_ms / args.steps,
                "sigma": sig_ms / args.steps}
    two = wl.threshold == 0.0 and n_fwd < M
    kern = {
        ("k_fwd2" if two else "k_fwd"): (
            rotate_bytes(st, tsz) / n_fwd, fwd_ms / args.steps / n_fwd,
            f"forward: pair rotation + truncation, {M} factors in {n_fwd} launches"),
        ("k_rev2" if two else "k_rev"): (
            reverse_bytes(st, tsz) / n_rev, rev_ms / args.steps / n_rev,
            f"reverse: exact inverse + adjoint rotation + gradient dot, {M} factors in {n_rev} launches"),
    }
    traffic = measured_traffic(args.workload, args.prec)
    # index probes: every scanned member of a rotated pair looks its partner
    # up once (the pair's owner, and the upper member of a pair whose lower
    # member is present, which owns it), so a sweep makes pairs + partner
    # hits probes; set against the random reads the device serves
    probes = st["pair_updates"] + st["partner_hits"]
    rr = random_read_rate(dev)
    lines = {}
    for name, (bpl, ms, what) in kern.items():
        ach = bpl / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        n_l = n_fwd if name.startswith("k_fwd") else n_rev
        ppl = probes / n_l
        prate = ppl / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        lines[name] = {"kernel": name, "what": what, "bound": "hbm", "achieved": round(ach, 2),
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5),
                       "traffic": traffic.get(name + "_step", traffic.get(name)), "bytes_per_launch": round(bpl, 1),
                       "avg_launch_us": round(ms * 1e3, 3),
                       # (a two-factor launch probes for up to three partners per
                       # member: its probes are not these)
                       "probes": None if two else {
                           "per_launch": round(ppl, 1), "achieved_G_per_s": round(prate, 3),
                           "device_random_reads_G_per_s": round(rr, 3),
                           "frac": round(prate / rr, 4) if rr > 0 else None}}
    dom = max(lines, key=lambda n: kern[n][1])
    roofline = dict(lines[dom])
    roofline["kernel_ms_per_step"] = {k: round(v, 4) for k, v in per_step.items()}
    # the floor of a chain of dependent launches on this device: a captured
    # graph of one-element kernels (what a sweep step would cost with no work)
    floor = graph_node_floor_us(dev)
    roofline["launch_floor_us"] = round(floor, 3)
    roofline["other"] = {n: l for n, l in lines.items() if n != dom}
    for l in [roofline] + list(roofline["other"].values()):
        l["launch_over_floor"] = round(l["avg_launch_us"] / floor, 2)

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "E+grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == swc.FP32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{wl.name}: {nq} qubits, {2 * wl.n_occ} electrons, "
                         + (f"first {M} factors of spin-conserving UCCSD" if args.factors
                            else f"full spin-conserving UCCSD ({M} factors)")
                         + f", theta~N(0,{wl.theta_sigma}), threshold {wl.threshold}, "
                         f"capacity 2^{int(np.log2(cap))}" + (f", batch {B}" if B > 1 else "")
                         + (f", N_MAX/N_CUT {topk[0]}/{topk[1]}" if topk else "")
                         + (", entropy tracked" if args.entropy else "")
                         + (f", checkpoints every {args.checkpoint_interval} factors"
                            if args.checkpoint_interval > 0 else "")),
            "amplitudes": args.prec, "reductions": "f64 (exact fixed point)",
            "n_det_final": n_live,
        },
        "det_updates_per_step": det_updates,
        "pair_updates_per_step": st["pair_updates"],
        "partner_hits_per_step": st["partner_hits"],
        "inserts_per_step": st["inserts"],
        "pruned_per_step": st["pruned"],
        "truncation_log_records": log_records,
        "sigma_partitions": st["sigma_partitions"],
        "table_slots_final": st["table_slots"],
        "live_trajectory": live_traj,
        "entry_positions_scanned_per_step": scans,
        "checkpoints_per_step": ck_taken,
        "det_updates_per_s_forward": round(det_updates / (fwd_ms / args.steps * 1e-3), 1) if fwd_ms else None,
        "energy": E0,
        **({"entropy_final": float(s.entropy(0)[-1])} if args.entropy else {}),
        "roofline": roofline,
    }

    if args.fp64_check and prec == swc.FP32:
        # the same evaluation with FP64 amplitudes: the FP32 path's error at this depth
        s.close()
        s = swc.Solver(nq, wl.n_occ, wl.n_occ, cap, prec=swc.FP64, batch=B, max_factors=M, log_capacity=logcap,
                       device=dev)
        if args.sigma_scratch_gib > 0:
            s.set_sigma_scratch(int(args.sigma_scratch_gib * (1 << 30)), mode=args.sigma_mode)
        s.build_state()
        c0 = time.perf_counter()
        E64, g64 = s.energy_and_grad(theta, p.exc, wl.threshold, h1, h2)
        torch.cuda.synchronize()
        c1 = time.perf_counter()
        progress("FP64 evaluation done")
        E64, g64 = E64.cpu().numpy(), g64.cpu().numpy()
        out["fp64_check"] = {
            "seconds": round(c1 - c0, 3),
            "max_abs_dE": float(np.max(np.abs(E.cpu().numpy() - E64))),
            "max_abs_dg": float(np.max(np.abs(g.cpu().numpy() - g64))),
            "rms_dg": float(np.sqrt(np.mean((g.cpu().numpy() - g64) ** 2))),
            "max_abs_g": float(np.max(np.abs(g64))),
        }

    if not args.no_fd:
        # same-GPU FP64 forward + central finite differences (h = 1e-5)
        sf = swc.Solver(nq, wl.n_occ, wl.n_occ, cap, prec=swc.FP64, batch=1, max_factors=M, device=dev)
        if args.sigma_scratch_gib > 0:  # the same sigma method as the adjoint run
            sf.set_sigma_scratch(int(args.sigma_scratch_gib * (1 << 30)), mode=args.sigma_mode)
        sf.build_state()
        h = 1e-5
        tp = theta[0:1].clone()
        w0 = time.perf_counter()
        sf.apply_ucc(tp, p.exc, wl.threshold)
        sf.energy(h1, h2)
        sf.build_state()
        torch.cuda.synchronize()
        t_eval = time.perf_counter() - w0
        # as many sampled parameters as fit the time budget (at least two)
        n_fd = max(2, min(args.fd_params, int(args.fd_max_s / (2.0 * t_eval))))
        idx = synth.fd_subset(M, n_fd, 3000 + wl.cfg)
        progress(f"finite differences: warm-up evaluation done ({t_eval:.2f} s), {n_fd} parameters sampled")
        fd = np.empty(len(idx))
        f0 = time.perf_counter()
        for q, k in enumerate(idx):
            ev = []
            for sgn in (1.0, -1.0):
                tp.copy_(theta[0:1])
                tp[0, k] += sgn * h
                sf.build_state()
                sf.apply_ucc(tp, p.exc, wl.threshold)
                ev.append(sf.energy(h1, h2).item())
                progress(f"finite differences: parameter {q + 1}/{len(idx)}, sign {sgn:+.0f} done")
            fd[q] = (ev[0] - ev[1]) / (2 * h)
        torch.cuda.synchronize()
        f1 = time.perf_counter()
        t_full = (f1 - f0) / len(idx) * M
        extrapolated = True
        if t_full <= args.fd_full_max_s and len(idx) < M:
            # cheap enough: every parameter, timed as a whole
            idx = np.arange(M)
            fd = np.empty(M)
            f0 = time.perf_counter()
            for q, k in enumerate(idx):
                ev = []
                for sgn in (1.0, -1.0):
                    tp.copy_(theta[0:1])
                    tp[0, k] += sgn * h
                    sf.build_state()
                    sf.apply_ucc(tp, p.exc, wl.threshold)
                    ev.append(sf.energy(h1, h2).item())
                fd[q] = (ev[0] - ev[1]) / (2 * h)
            torch.cuda.synchronize()
            t_full = time.perf_counter() - f0
            extrapolated = False
            progress(f"finite differences over all {M} parameters done, {t_full:.1f} s")
        out["fd_baseline"] = {
            "what": "same GPU, FP64 amplitudes: E(theta +- h e_p) by forward sweep + energy, h=1e-5",
            "params_timed": int(len(idx)),
            "extrapolated": extrapolated,
            "seconds_per_full_gradient": round(t_full, 4),
            "evals_per_s": round(1.0 / t_full, 6),
            "adjoint_speedup": round(value * t_full, 2),
            "max_abs_grad_diff_vs_adjoint": float(np.max(np.abs(fd - g0[idx]))),
        }
        sf.close()

    if prec == swc.FP64 and not args.no_fp32:
        # the FP32-amplitude path (FP64 reductions) on the same workload: its
        # rate and its distance from the FP64 result timed above
        s32 = swc.Solver(nq, wl.n_occ, wl.n_occ, cap, prec=swc.FP32, batch=B, max_factors=M, log_capacity=logcap,
                         device=dev)
        if args.sigma_scratch_gib > 0:
            s32.set_sigma_scratch(int(args.sigma_scratch_gib * (1 << 30)), mode=args.sigma_mode)
        if args.checkpoint_interval > 0:
            s32.set_checkpoints(args.checkpoint_interval, 1 << args.checkpoint_entries_log2)
        s32.build_state()
        s32.energy_and_grad(theta, p.exc, wl.threshold, h1, h2)
        torch.cuda.synchronize()
        n32 = 2
        c0 = time.perf_counter()
        for _ in range(n32):
            E32, g32 = s32.energy_and_grad(theta, p.exc, wl.threshold, h1, h2)
        torch.cuda.synchronize()
        c1 = time.perf_counter()
        out["fp32"] = {
            "what": "FP32 amplitudes and rotations, FP64 reductions; same workload, same theta",
            "evals_per_s": round(n32 * B / (c1 - c0), 4),
            "abs_dE_vs_fp64": float(np.max(np.abs(E32.cpu().numpy() - E.cpu().numpy()))),
            "max_abs_dg_vs_fp64": float(np.max(np.abs(g32.cpu().numpy() - g.cpu().numpy()))),
            "final_states": state_difference(s, s32, theta, p.exc, wl.threshold, h1, h2),
        }
        s32.close()
        progress("FP32 evaluations done")

    if not args.no_cpu_baseline:
        import oracle
        if topk:
            oracle.set_topk(*topk)
        if wl.name in ("q8", "q20"):
            # the whole evaluation fits the CPU budget (about 10 s at 20 qubits)
            c0 = time.perf_counter()
            E_ref, g_ref, _ = oracle.energy_and_grad(nq, [p.hf], [1.0], p.exc, p.theta[0], wl.threshold, p.h1, p.h2)
            c1 = time.perf_counter()
            out["cpu_baseline"] = {
                "value": round(1.0 / (c1 - c0), 6),
                "unit": "E+grad evals/s",
                "cores": 1,
                "kind": "oracle",
                "sample": f"one full E+grad evaluation of {wl.name} ({M} factors), single-threaded std::map FP64",
                "seconds": round(c1 - c0, 3),
                "host_cpus": os.cpu_count(),
                "host_cpu_model": cpu_model(),
            }
            out["parity_vs_oracle"] = {"abs_dE": abs(E0 - E_ref), "max_abs_dg": float(np.max(np.abs(g0 - g_ref)))}
        else:
            # The oracle's E+grad over prefixes of the circuit twice as long
            # each time, until one takes cpu-seconds; that evaluation is the
            # CPU sample and the parity reference of the GPU on the prefix.
            K = 256
            while True:
                K = min(M, 2 * K)
                c0 = time.perf_counter()
                E_ref, g_ref, nc = oracle.energy_and_grad(nq, [p.hf], [1.0], p.exc[:K], p.theta[0, :K], wl.threshold,
                                                          p.h1, p.h2)
                t_eg = time.perf_counter() - c0
                if t_eg >= args.cpu_seconds or K == M:
                    break
            progress(f"oracle E+grad of the first {K} factors: {t_eg:.1f} s")
            par = {"factors": K, "oracle_near_cut_events": nc}
            for name, pr in (("fp64", swc.FP64), ("fp32", swc.FP32)):
                sp_ = swc.Solver(nq, wl.n_occ, wl.n_occ, 1 << 20, prec=pr, batch=1, max_factors=K, device=dev)
                sp_.build_state()
                Ep, gp = sp_.energy_and_grad(theta[0:1, :K], p.exc[:K], wl.threshold, h1, h2)
                par[f"abs_dE_{name}"] = abs(float(Ep[0].item()) - E_ref)
                par[f"max_abs_dg_{name}"] = float(np.max(np.abs(gp.cpu().numpy()[0] - g_ref)))
                sp_.close()
            out["parity_vs_oracle"] = par
            # Scaled to the whole circuit: the sweeps' time grows with the
            # determinants visited (det-updates), the energy's with the final
            # determinants (each probes the same number of connections).
            dK, aK, _, _ = oracle.apply_ucc(nq, [p.hf], [1.0], p.exc[:K], p.theta[0, :K], wl.threshold)
            c0 = time.perf_counter()
            oracle.energy(nq // 2, p.h1, p.h2, dK, aK)
            t_E = time.perf_counter() - c0
            du_c = int(np.sum(oracle.live_trajectory(nq, [p.hf], [1.0], p.exc[:K], p.theta[0, :K],
                                                     wl.threshold)[:-1]))
            t_sw = max(t_eg - t_E, 0.0)
            t_full_cpu = t_sw * det_updates / max(du_c, 1) + t_E * n_live / len(dK)
            out["cpu_baseline"] = {
                "value": round(1.0 / t_full_cpu, 9),
                "unit": "E+grad evals/s",
                "cores": 1,
                "kind": "oracle",
                "sample": f"one E+grad evaluation of the first {K} factors of {wl.name} ({t_eg:.1f} s: sweeps "
                          f"{t_sw:.1f} s over {du_c} det-updates, energy {t_E:.1f} s over {len(dK)} determinants), "
                          "single-threaded std::map FP64; scaled to the whole circuit (sweeps by its "
                          f"{det_updates} det-updates, energy by its {n_live} final determinants)",
                "extrapolated": K < M,
                "seconds": round(t_eg + t_E, 3),
                "host_cpus": os.cpu_count(),
                "host_cpu_model": cpu_model(),
            }

    s.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
