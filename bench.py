#!/usr/bin/env python3
"""Benchmark: list ranking and connected components on one MI355X.

One step = one full solve through the C ABI.  The headline workload is the
uniform random list of n = 2^26 nodes ranked by the random-splitter (ruling
set) path, inputs resident in HBM.  Extra workloads (Wyllie, other layouts,
the 2^20 list, components on 2^22 vertices / 2^25 pairs, the batched 4096-list
set against per-list launches) are reported under "extras".

Prints progress on stderr and ONE JSON line on stdout.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

METRIC = "list-rank nodes/s & CC edges/s at 1 GPU; batched vs plain speedup; p99 lat"
HBM_PEAK_GBS = 8000.0
LR_BYTES_PER_NODE = 8   # algorithmic: succ read once + rank written once
CC_BYTES_PER_PAIR = 8   # algorithmic: both ends read once
CC_BYTES_PER_VERTEX = 4  # algorithmic: label written once
PROFILE_DIR = os.path.join(ROOT, "profiles")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def require(ok, what):
    """Every timed result is checked; a wrong one ends the run with an error."""
    if not ok:
        log(f"MISMATCH: {what}")
        raise SystemExit(f"wrong result: {what}")
    return True


def closed_form_ok(torch, rank, d_order):
    """rank[order[k]] == k: the k-th node of the generator's list order has
    rank k (the closed form of every generated list)."""
    n = d_order.numel()
    return bool(torch.equal(rank[d_order], torch.arange(n, dtype=torch.int32,
                                                        device=rank.device)))


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1002_4482_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(name, src_files):
    """HBM bytes per launch from a committed counter summary, if the kernel
    source it was taken from is unchanged; else None."""
    path = os.path.join(PROFILE_DIR, name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash(*src_files):
        return None
    return rec.get("hbm_bytes_per_launch")


def timed(torch, fn, steps, warmup, per_step=None):
    """Mean ms per step over `steps` back-to-back calls on the current stream
    (events between steps, one synchronisation at the end).  If `per_step`
    is a list, the individual step times are appended to it."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    if per_step is not None:
        per_step.extend(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    return ev[0].elapsed_time(ev[steps]) / steps


def random_access_ceiling(torch, dev, d_succ, d_order, hops, reps=5):
    """The level-0 walk's access pattern alone (libpjprobe.so): lanes chase
    disjoint segments of `hops` nodes that together cover the list, reading a
    random successor per step, and (rmw) storing to the word just read, as
    the walk overwrites each successor with the node's packed state.
    Returns the mean device ms of each variant (the list is visited once per
    run; the stores write back the values read)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1002_4482_amd", "libpjprobe.so"))
    lib.pjp_chase.restype = ctypes.c_int
    lib.pjp_chase.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                              ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                              ctypes.POINTER(ctypes.c_float),
                              ctypes.POINTER(ctypes.c_ulonglong), ctypes.c_void_p]
    a = d_succ.clone()
    starts = d_order[::hops].to(torch.int32).contiguous()
    scratch = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = {}
    for name, write in (("read", 0), ("rmw", 1)):
        times = []
        for _ in range(reps + 1):
            ms = ctypes.c_float(0.0)
            vis = ctypes.c_ulonglong(0)
            rc = lib.pjp_chase(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(starts.data_ptr()),
                               starts.numel(), hops, write, 0, ctypes.c_void_p(scratch.data_ptr()),
                               ctypes.byref(ms), ctypes.byref(vis), stream)
            require(rc == 0 and vis.value == d_succ.numel(), f"ceiling probe ({name})")
            times.append(ms.value)
        out[name] = float(np.mean(times[1:]))
    require(bool(torch.equal(a, d_succ)), "ceiling probe left the list unchanged")
    del a, starts, scratch
    return out


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_peak_gbs(torch, dev):
    """Achievable HBM rate of a plain 256 MiB device copy (read + write bytes)."""
    a = torch.empty(1 << 26, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    ms = timed(torch, lambda: b.copy_(a), 10, 3)
    del a, b
    return 2 * (1 << 28) / (ms * 1e-3) / 1e9


def phase_means(stats_list):
    acc = {}
    for st in stats_list:
        for name, ms in st["phase_list"]:
            acc.setdefault(name, []).append(ms)
    return {k: float(np.mean(v)) for k, v in acc.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--log2n", type=int, default=26)
    ap.add_argument("--workload", default="list_uniform",
                    choices=["list_uniform", "list_sequential", "list_blocked",
                             "list_uniform_wyllie", "list_uniform_2p20", "cc_uniform",
                             "cc_planted", "lists_batched_4096", "list_sweep"],
                    help="list_uniform (default) is the headline; the others time one workload "
                         "alone (for profiling) and print its own JSON line")
    ap.add_argument("--serve-requests", type=int, default=5000,
                    help="requests per load point of the serving sweep")
    ap.add_argument("--serve-warmup", type=int, default=500,
                    help="serving warm-up requests (not timed, not checked)")
    ap.add_argument("--sweep-sizes", type=lambda v: [int(x) for x in v.split(",")],
                    default=[22, 24, 26, 28],
                    help="log2 list sizes of the packing / Wyllie size sweep (comma-separated)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy a 256 MiB int32 tensor three times (a kernel of known "
                         "traffic, to scale HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "one GPU per process: --gpus must be 1 (the library has no "
                                   "multi-GPU path)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    import paper_1002_4482_amd as pj

    pj.load()
    dev = torch.device("cuda:0")
    n = 1 << args.log2n
    if args.calibrate_copy:
        a = torch.arange(1 << 26, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 256 MiB")
        del a, b
    if args.workload != "list_uniform":
        print(json.dumps(single_workload(torch, pj, dev, args)), flush=True)
        return

    log(f"generating uniform random list n=2^{args.log2n}")
    succ, order = W.random_list_with_order(n, W.SEED_BASE + 2)
    d_succ = torch.from_numpy(succ).to(dev)
    d_rank = torch.empty_like(d_succ)

    def step():
        pj.list_rank(d_succ, d_rank, algo="ruling_set")

    log(f"timing ruling set: warmup {args.warmup}, steps {args.steps}")
    step_ms = []
    ms = timed(torch, step, args.steps, args.warmup, step_ms)
    # correctness of what was timed: closed form rank[order[k]] = k
    d_order = torch.from_numpy(order).to(dev).long()
    ok = require(closed_form_ok(torch, d_rank, d_order), "the headline list")
    log(f"ruling set {ms:.3f} ms/step, correct={ok}")

    # per-phase device times: HIP events the library records on its stream
    # around each phase, over as many stats-enabled steps right after the
    # timed ones (reading them back needs a synchronisation per step, which
    # is kept out of the timed region)
    stats = []
    for _ in range(max(3, min(args.steps, 10))):
        _, st = pj.list_rank(d_succ, d_rank, algo="ruling_set", return_stats=True)
        stats.append(st)
    phases = phase_means(stats)
    walk_ms = phases.get("walk0", float("nan"))
    achieved = LR_BYTES_PER_NODE * n / (walk_ms * 1e-3) / 1e9
    traffic = traffic_from_profile("walk0_u26_traffic.json", ["list_rank.hip"])
    copy_gbs = copy_peak_gbs(torch, dev)
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": "lr_walk level 0 (sublist walks)",
        "kernel_ms": round(walk_ms, 4),
        "bytes_per_node": LR_BYTES_PER_NODE,
        "copy_peak": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4),
        "traffic_per_node": round(traffic / n, 1) if traffic else None,
        "amplification": round(traffic / (LR_BYTES_PER_NODE * n), 1) if traffic else None,
        "traffic_rate": round(traffic / (walk_ms * 1e-3) / 1e9, 1) if traffic else None,
    }
    # the walk against the same access pattern alone, on this chip
    hops = max(1, n // max(1, stats[-1]["sublists0"]))
    ceil = random_access_ceiling(torch, dev, d_succ, d_order, hops)
    roofline.update({
        "random_ceiling_kernel": f"dependent random read + store to the same word, "
                                 f"{hops}-node segments covering the list (libpjprobe.so)",
        "random_ceiling_ms": round(ceil["rmw"], 4),
        "random_read_only_ms": round(ceil["read"], 4),
        "frac_of_random_ceiling": round(ceil["rmw"] / walk_ms, 4),
    })
    log(f"random-access ceiling {ceil}, walk {walk_ms:.3f} ms")
    path_gbs = LR_BYTES_PER_NODE * n / (ms * 1e-3) / 1e9
    log(f"phases {phases}")

    extras = {
        "step_ms": {"mean": round(float(np.mean(step_ms)), 4), "sd": round(float(np.std(step_ms)), 4),
                    "median": round(float(np.median(step_ms)), 4)},
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "levels": stats[-1]["levels"],
        "level_nodes": stats[-1]["level_nodes"],
        "path_frac_of_hbm": round(path_gbs / HBM_PEAK_GBS, 4),
    }
    if not args.no_extras:
        extras.update(run_extras(torch, pj, dev, d_succ, d_rank, d_order, n, args))
    del d_succ, d_rank, d_order
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        import cpu_baseline
        import oracle
        log("timing the CPU oracle on the same list (one run, 1 thread)")
        t = time.perf_counter()
        ref = oracle.list_rank(succ)
        dt = time.perf_counter() - t
        assert np.array_equal(ref[order], np.arange(n, dtype=np.int32))
        cpu = {"value": round(n / dt, 1), "unit": "nodes/s", "cores": 1, "kind": "oracle",
               "sample": f"one sequential walk over the whole 2^{args.log2n}-node uniform list "
                         f"with validation ({dt:.2f} s)"}
        # the paper's multi-core comparison: random splitters on POSIX threads
        threads = min(16, os.cpu_count() or 1)
        best = None
        for _ in range(3):
            t = time.perf_counter()
            rc, mt = cpu_baseline.ruling_set(succ, 64, threads)
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        assert rc == 0 and np.array_equal(mt, ref)
        extras["cpu_ruling_set_threads"] = {
            "value": round(n / best, 1), "unit": "nodes/s", "cores": threads,
            "ms": round(best * 1e3, 1),
            "sample": f"the same list, spacing 64, best of 3 runs"}
        log(f"CPU ruling set on {threads} threads: {best * 1e3:.1f} ms")
        # the components oracle on the 2^22-vertex, 2^25-pair uniform graph
        nv, m = 1 << 22, 1 << 25
        src, dst = W.random_graph(nv, m, W.SEED_BASE + 3)
        t = time.perf_counter()
        oracle.connected_components(src, dst, nv)
        dt = time.perf_counter() - t
        extras["cpu_oracle_cc_2p22_uniform"] = {
            "value": round(m / dt, 1), "unit": "pairs/s", "cores": 1, "ms": round(dt * 1e3, 1),
            "sample": "sequential union-find over the whole graph, one run"}
        log(f"CPU components oracle: {dt * 1e3:.1f} ms")
        extras["host_cpu"] = {"model": host_cpu_model(), "threads": os.cpu_count()}
    extras["environment"] = {"hip": getattr(torch.version, "hip", None), "torch": torch.__version__,
                             "device": torch.cuda.get_device_name(0), "seed_base": W.SEED_BASE}

    out = {
        "metric": METRIC,
        "value": round(n / (ms * 1e-3), 1),
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": f"list ranking, one uniform random list, n=2^{args.log2n} int32 "
                        "successors, ruling set (random splitters, recursive)",
            "n": n,
            "layout": "uniform random permutation",
            "algo": "ruling_set",
            "seed": W.SEED_BASE + 2,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


def single_workload(torch, pj, dev, args):
    """Time one workload alone; returns its JSON record (phases included)."""
    wl = args.workload
    rec = {"workload": wl, "steps": args.steps, "warmup": args.warmup}
    if wl == "list_sweep":
        rec["sizes"] = list_sweep(torch, pj, dev, args)
    elif wl.startswith("list_"):
        n = 1 << (20 if wl == "list_uniform_2p20" else args.log2n)
        if wl == "list_sequential":
            s, order = W.sequential_list(n), np.arange(n)
        elif wl == "list_blocked":
            s, order = W.blocked_list_with_order(n, 4096, W.SEED_BASE + 2)
        else:
            s, order = W.random_list_with_order(
                n, W.SEED_BASE + (1 if wl == "list_uniform_2p20" else 2))
        algo = "wyllie" if wl == "list_uniform_wyllie" else "ruling_set"
        ds = torch.from_numpy(s).to(dev)
        dr = torch.empty_like(ds)
        ms = timed(torch, lambda: pj.list_rank(ds, dr, algo=algo), args.steps, args.warmup)
        require(closed_form_ok(torch, dr, torch.from_numpy(order).to(dev).long()), wl)
        _, st = pj.list_rank(ds, dr, algo=algo, return_stats=True)
        rec.update(n=n, algo=algo, ms=round(ms, 4), nodes_per_s=round(n / (ms * 1e-3), 1),
                   phases=st["phases"], levels=st["levels"], level_nodes=st["level_nodes"])
    elif wl in ("cc_uniform", "cc_planted"):
        nv, m = 1 << 22, 1 << 25
        if wl == "cc_uniform":
            src, dst = W.random_graph(nv, m, W.SEED_BASE + 3)
        else:
            src, dst, _ = W.planted_graph(nv, m, 1024, W.SEED_BASE + 3)
        ds, dd = torch.from_numpy(src).to(dev), torch.from_numpy(dst).to(dev)
        lab = torch.empty(nv, dtype=torch.int32, device=dev)
        ms = timed(torch, lambda: pj.connected_components(ds, dd, nv, lab), args.steps,
                   args.warmup)
        import oracle
        require(np.array_equal(lab.cpu().numpy(), oracle.connected_components(src, dst, nv)),
                wl)
        _, st = pj.connected_components(ds, dd, nv, lab, return_stats=True)
        rec.update(n=nv, m=m, ms=round(ms, 4), edges_per_s=round(m / (ms * 1e-3), 1),
                   rounds=st["rounds"], phases=st["phases"])
    else:  # lists_batched_4096
        bs, boff = W.batched_lists(4096, 6, 20, W.SEED_BASE + 4)
        dbs, dboff = torch.from_numpy(bs).to(dev), torch.from_numpy(boff).to(dev)
        dbr = torch.empty_like(dbs)
        ms = timed(torch, lambda: pj.list_rank_batched(dbs, dboff, dbr, h_offsets=boff),
                   args.steps, args.warmup)
        import oracle
        require(np.array_equal(dbr.cpu().numpy(), oracle.list_rank_batched(bs, boff)[1]), wl)
        _, st = pj.list_rank_batched(dbs, dboff, dbr, h_offsets=boff, return_stats=True)
        rec.update(total_nodes=int(boff[-1]), ms=round(ms, 4),
                   nodes_per_s=round(int(boff[-1]) / (ms * 1e-3), 1), phases=st["phases"],
                   levels=st["levels"], level_nodes=st["level_nodes"])
    log(json.dumps(rec))
    return rec


def list_sweep(torch, pj, dev, args):
    """Uniform random lists from 2^20 to 2^28 nodes: where the rate bends as
    the list outgrows the 256 MiB last-level cache."""
    rows = []
    for lg in (20, 22, 24, 25, 26, 27, 28):
        n = 1 << lg
        log(f"sweep: generating a uniform list of 2^{lg} nodes")
        s, order = W.random_list_with_order(n, W.SEED_BASE + 2)
        ds = torch.from_numpy(s).to(dev)
        dr = torch.empty_like(ds)
        del s
        steps = max(3, min(args.steps, 20 if lg <= 24 else 8))
        row = {"log2n": lg}
        do = torch.from_numpy(order).to(dev).long()
        want = torch.arange(n, dtype=torch.int32, device=dev)
        del order
        for algo in ("ruling_set", "wyllie"):
            ms = timed(torch, lambda: pj.list_rank(ds, dr, algo=algo), steps, 1)
            _, st = pj.list_rank(ds, dr, algo=algo, return_stats=True)
            row[f"{algo}_ms"] = round(ms, 4)
            row[f"{algo}_nodes_per_s"] = round(n / (ms * 1e-3), 1)
            if algo == "ruling_set":
                row["walk0_ms"] = round(st["phases"].get("walk0", 0.0), 4)
                row["expand0_ms"] = round(st["phases"].get("expand0", 0.0), 4)
            # closed form: the k-th node of the list order has rank k
            row[f"{algo}_correct"] = bool(torch.equal(dr[do], want))
        del do, want
        log(f"sweep 2^{lg}: {row}")
        rows.append(row)
        del ds, dr
        torch.cuda.empty_cache()
    return rows


def run_extras(torch, pj, dev, d_succ, d_rank, d_order, n, args):
    ex = {}
    steps = max(3, min(args.steps, 10))

    # the serving loop first, in a process that has not yet run the large
    # single solves (their cached device memory and pinned pages made the
    # loop measurably slower when it ran last)
    ex.update(run_serving(torch, pj, args))

    # Wyllie on the same list
    ms = timed(torch, lambda: pj.list_rank(d_succ, d_rank, algo="wyllie"), steps, 1)
    ok = require(closed_form_ok(torch, d_rank, d_order), "Wyllie on the headline list")
    ex[f"list_2p{args.log2n}_uniform_wyllie"] = {
        "ms": round(ms, 3), "nodes_per_s": round(n / (ms * 1e-3), 1), "correct": ok}
    log(f"wyllie uniform {ms:.3f} ms")

    # weighted ranks on the same list (separate state, weights beside succ);
    # closed form: the exclusive prefix of the weights along the list order.
    # The library's sums are int32, so the weights are drawn small enough
    # that the list's total fits (below 16 per node: under 2^30 at 2^26)
    wts = torch.from_numpy(np.random.default_rng(W.SEED_BASE + 7).integers(
        0, 16, n).astype(np.int32)).to(dev)
    assert 15 * n < 2**31
    ms = timed(torch, lambda: pj.list_rank_weighted(d_succ, wts, d_rank), steps, 1)
    wo = wts[d_order].to(torch.int64)
    ok = require(bool(torch.equal(d_rank[d_order].to(torch.int64), torch.cumsum(wo, 0) - wo)),
                 "weighted ranks on the headline list")
    ex[f"list_2p{args.log2n}_uniform_weighted"] = {
        "ms": round(ms, 3), "nodes_per_s": round(n / (ms * 1e-3), 1), "correct": ok}
    log(f"weighted uniform {ms:.3f} ms")
    del wts, wo

    # other layouts
    for name in ("sequential", "blocked"):
        if name == "sequential":
            s, order = W.sequential_list(n), None
        else:
            s, order = W.blocked_list_with_order(n, 4096, W.SEED_BASE + 2)
        ds = torch.from_numpy(s).to(dev)
        do = (torch.from_numpy(order).to(dev).long() if order is not None
              else torch.arange(n, device=dev))
        for algo in ("ruling_set", "wyllie"):
            ms = timed(torch, lambda: pj.list_rank(ds, d_rank, algo=algo), steps, 1)
            ok = require(closed_form_ok(torch, d_rank, do), f"{name} list, {algo}")
            ex[f"list_2p{args.log2n}_{name}_{algo}"] = {
                "ms": round(ms, 3), "nodes_per_s": round(n / (ms * 1e-3), 1),
                "frac_of_hbm": round(LR_BYTES_PER_NODE * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "correct": ok}
            log(f"{name} {algo} {ms:.3f} ms")
        del ds, do

    # 2^20 list
    n1 = 1 << 20
    s1, o1 = W.random_list_with_order(n1, W.SEED_BASE + 1)
    s1 = torch.from_numpy(s1).to(dev)
    o1 = torch.from_numpy(o1).to(dev).long()
    r1 = torch.empty_like(s1)
    for algo in ("ruling_set", "wyllie"):
        ms = timed(torch, lambda: pj.list_rank(s1, r1, algo=algo), 20, 3)
        ok = require(closed_form_ok(torch, r1, o1), f"2^20 list, {algo}")
        ex[f"list_2p20_uniform_{algo}"] = {
            "ms": round(ms, 4), "nodes_per_s": round(n1 / (ms * 1e-3), 1),
            "frac_of_hbm": round(LR_BYTES_PER_NODE * n1 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "correct": ok}
        log(f"2^20 uniform {algo} {ms:.4f} ms")

    ex.update(splitter_ablation(torch, pj, dev, d_succ, d_rank, d_order, n, steps))

    # components, checked against the union-find oracle
    import oracle
    nv, m = 1 << 22, 1 << 25
    for kind in ("uniform", "planted"):
        if kind == "uniform":
            src, dst = W.random_graph(nv, m, W.SEED_BASE + 3)
        else:
            src, dst, _ = W.planted_graph(nv, m, 1024, W.SEED_BASE + 3)
        ds, dd = torch.from_numpy(src).to(dev), torch.from_numpy(dst).to(dev)
        lab = torch.empty(nv, dtype=torch.int32, device=dev)
        ms = timed(torch, lambda: pj.connected_components(ds, dd, nv, lab), steps, 1)
        ok = require(np.array_equal(lab.cpu().numpy(), oracle.connected_components(src, dst, nv)),
                     f"components, {kind} graph")
        _, st = pj.connected_components(ds, dd, nv, lab, return_stats=True)
        ex[f"cc_2p22_{kind}"] = {
            "ms": round(ms, 3), "edges_per_s": round(m / (ms * 1e-3), 1), "rounds": st["rounds"],
            "frac_of_hbm": round((CC_BYTES_PER_PAIR * m + CC_BYTES_PER_VERTEX * nv)
                                 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "phases_ms": {k: round(v, 3) for k, v in st["phases"].items()}, "correct": ok}
        log(f"cc {kind} {ms:.3f} ms rounds {st['rounds']}")
        del ds, dd, lab

    ex.update(cc_families(torch, pj, dev, steps))

    ex.update(cc_batched(torch, pj, dev, steps))

    ex.update(batched_lists(torch, pj, dev, steps))

    ex.update(packing_sweep(torch, pj, dev, args))
    return ex


def batched_lists(torch, pj, dev, steps):
    """4096 lists of 2^6..2^20 nodes: one batched call (eager, replayed graph,
    tuned) against one plain call per list, every form checked by the closed
    form of each list."""
    log("generating 4096 lists, sizes log-uniform in [2^6, 2^20]")
    bs, boff, orders = W.batched_lists(4096, 6, 20, W.SEED_BASE + 4, return_orders=True)
    total = int(boff[-1])
    dbs = torch.from_numpy(bs).to(dev)
    dboff = torch.from_numpy(boff).to(dev)
    dbr = torch.empty_like(dbs)
    sizes = torch.from_numpy(np.diff(boff)).to(dev)
    base = torch.repeat_interleave(dboff[:-1], sizes)
    pos = torch.from_numpy(np.concatenate(orders)).to(dev).long() + base
    kk = (torch.arange(total, device=dev) - base).int()
    del base, orders

    def check(what):
        ok = bool(torch.equal(dbr[pos], kk))
        return require(ok, f"4096-list batch, {what}")

    views = [(dbs[boff[i]:boff[i + 1]], dbr[boff[i]:boff[i + 1]]) for i in range(4096)]

    def plain():
        for s, r in views:
            pj.list_rank(s, r)

    def batched():
        pj.list_rank_batched(dbs, dboff, dbr, h_offsets=boff)

    def graphed():
        pj.list_rank_batched(dbs, dboff, dbr, h_offsets=boff, use_graph=True)

    dbr.fill_(-1)
    ms_b = timed(torch, batched, steps, 1)
    check("eager")
    dbr.fill_(-1)
    ms_p = timed(torch, plain, 2, 1)
    check("one call per list")
    # the first graphed call captures and instantiates the graph: its cost is
    # reported on its own and kept out of the replay timing
    pj.graph_cache_clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    graphed()
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    dbr.fill_(-1)
    ms_g = timed(torch, graphed, steps, 1)
    check("graph replay")
    # tuned parameters for this size class, then eager and the graph replay again
    best, _ = pj.tune_list_rank(dbs, dboff, h_offsets=boff)
    pj.graph_cache_clear()
    dbr.fill_(-1)
    ms_te = timed(torch, batched, steps, 1)
    check("tuned, eager")
    dbr.fill_(-1)
    ms_t = timed(torch, graphed, steps, 1)
    ok = check("tuned, graph replay")
    pj.graph_cache_clear()
    pj.tune_clear()
    best_ms = min(ms_b, ms_g, ms_te, ms_t)
    log(f"batched {ms_b:.3f} ms graph {ms_g:.3f} ms tuned {ms_te:.3f} / {ms_t:.3f} ms {best} "
        f"plain {ms_p:.3f} ms")
    del dbs, dboff, dbr, views, pos, kk
    torch.cuda.empty_cache()
    return {"batch_4096_lists": {
        "total_nodes": total, "batched_ms": round(ms_b, 3),
        "graph_capture_first_call_ms": round(build_ms, 3), "batched_graph_ms": round(ms_g, 3),
        "tuned_ms": round(ms_te, 3), "tuned_graph_ms": round(ms_t, 3), "tuned": best,
        "plain_ms": round(ms_p, 3), "batched_nodes_per_s": round(total / (best_ms * 1e-3), 1),
        "speedup_batched_vs_plain": round(ms_p / best_ms, 3), "correct": ok}}


def splitter_ablation(torch, pj, dev, d_succ, d_rank, d_order, n, steps, spacing=64):
    """Random against evenly spaced splitters (Section 3.2, Table 3): the
    same number of level-0 splitters (n / spacing) chosen uniformly at random
    or every spacing-th node in list order, walked by the same kernel; the
    library's hashed splitters (one per block of ids) beside them."""
    r = n // spacing
    rng = np.random.default_rng(W.SEED_BASE + 9)
    rand = torch.from_numpy(rng.choice(n, r, replace=False).astype(np.int32)).to(dev)
    even = d_order[::spacing].to(torch.int32).contiguous()
    out = {}
    # expected longest sublist of r random splitters: lengths are nearly
    # geometric with mean n / r, so the longest is about (n / r) (ln r + 0.5772)
    expect_max_random = (n / r) * (np.log(r) + 0.5772)
    for name, kw in (("random", {"splitters": rand}), ("even", {"splitters": even}),
                     ("hashed", {"spacing": spacing})):
        ms = timed(torch, lambda: pj.list_rank(d_succ, d_rank, max_walk=4096, **kw), steps, 1)
        ok = require(closed_form_ok(torch, d_rank, d_order), f"{name} splitters")
        sts = [pj.list_rank(d_succ, d_rank, max_walk=4096, return_stats=True, **kw)[1]
               for _ in range(3)]
        walk = float(np.mean([st["phases"].get("walk0", 0.0) for st in sts]))
        st = sts[-1]
        out[name] = {"ms": round(ms, 3), "walk0_ms": round(walk, 3),
                     "sublists": st["sublists0"], "mean_sublist": round(n / st["sublists0"], 2),
                     "max_sublist": st["max_sublist0"], "cuts": st["cuts0"], "correct": ok}
        log(f"splitters {name}: {out[name]}")
    out["expected"] = {"mean_sublist": spacing, "max_sublist_even": spacing,
                       "max_sublist_random": round(expect_max_random, 1)}
    del rand, even
    return {f"splitters_2p{int(np.log2(n))}_spacing{spacing}": out}


def packing_sweep(torch, pj, dev, args):
    """Level-0 state packed into the output word against a separate 8-byte
    state (the question Section 3.2 asks of its 48- and 64-bit layouts), and
    the ruling set against Wyllie, over list sizes around the last-level
    cache (Section 3.3's inflection point); every result checked by the
    closed form."""
    rows = []
    sizes = args.sweep_sizes
    for lg in sizes:
        nn = 1 << lg
        log(f"sweep: generating a uniform list of 2^{lg} nodes")
        s, order = W.random_list_with_order(nn, W.SEED_BASE + 2)
        ds = torch.from_numpy(s).to(dev)
        dr = torch.empty_like(ds)
        do = torch.from_numpy(order).to(dev).long()
        del s, order
        st_steps = max(3, min(args.steps, 10 if lg <= 24 else 5))
        row = {"log2n": lg}
        for name, kw in (("packed", dict(algo="ruling_set")),
                         ("separate", dict(algo="ruling_set", level0_state="separate")),
                         ("wyllie", dict(algo="wyllie"))):
            ms = timed(torch, lambda: pj.list_rank(ds, dr, **kw), st_steps, 1)
            ok = require(closed_form_ok(torch, dr, do), f"sweep 2^{lg} {name}")
            row[name] = {"ms": round(ms, 4), "nodes_per_s": round(nn / (ms * 1e-3), 1),
                         "correct": ok}
            if name != "wyllie":
                _, st = pj.list_rank(ds, dr, return_stats=True, **kw)
                row[name]["walk0_ms"] = round(st["phases"].get("walk0", 0.0), 4)
                row[name]["expand0_ms"] = round(st["phases"].get("expand0", 0.0), 4)
        log(f"sweep 2^{lg}: {row}")
        rows.append(row)
        del ds, dr, do
        torch.cuda.empty_cache()
    return {"size_sweep": rows}


def cc_batched(torch, pj, dev, steps, G=1024, seed=W.SEED_BASE + 8):
    """G graphs of the serving mix's shape (n = 2^U, U ~ U[8, 16], degree
    ~ U[2, 16], uniform pairs) solved by one batched call and by one call per
    graph; local ids and offset tables as the batched call takes them."""
    rng = np.random.default_rng(seed)
    ns = np.floor(2.0 ** rng.uniform(8, 16, G)).astype(np.int64)
    ms = np.round(ns * rng.uniform(2, 16, G) / 2).astype(np.int64)
    srcs, dsts = [], []
    for i in range(G):
        a, b = W.random_graph(int(ns[i]), int(ms[i]), seed + 1 + i)
        srcs.append(a)
        dsts.append(b)
    voff = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    eoff = np.concatenate([[0], np.cumsum(ms)]).astype(np.int64)
    src, dst = np.concatenate(srcs), np.concatenate(dsts)
    ds, dd = torch.from_numpy(src).to(dev), torch.from_numpy(dst).to(dev)
    dv, de = torch.from_numpy(voff).to(dev), torch.from_numpy(eoff).to(dev)
    lab = torch.empty(int(voff[-1]), dtype=torch.int32, device=dev)
    views = [(ds[eoff[i]:eoff[i + 1]], dd[eoff[i]:eoff[i + 1]], int(ns[i]),
              lab[voff[i]:voff[i + 1]]) for i in range(G)]

    def batched():
        pj.connected_components_batched(ds, dd, dv, de, lab, h_vtx_off=voff, h_edge_off=eoff)

    def plain():
        for a, b, n, out in views:
            pj.connected_components(a, b, n, out)

    import oracle
    want = torch.from_numpy(oracle.connected_components_batched(src, dst, voff, eoff)).to(dev)
    lab.fill_(-1)
    ms_b = timed(torch, batched, steps, 1)
    require(bool(torch.equal(lab, want)), f"batched components of {G} graphs")
    # one captured graph (the rounds it holds return at once after
    # convergence); its first call captures and is timed on its own
    def graphed():
        pj.connected_components_batched(ds, dd, dv, de, lab, h_vtx_off=voff, h_edge_off=eoff,
                                        use_graph=True)

    pj.graph_cache_clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    graphed()
    torch.cuda.synchronize()
    cap_ms = (time.perf_counter() - t0) * 1e3
    lab.fill_(-1)
    ms_g = timed(torch, graphed, steps, 1)
    require(bool(torch.equal(lab, want)), f"batched components of {G} graphs, graph replay")
    pj.graph_cache_clear()
    lab.fill_(-1)
    ms_p = timed(torch, plain, 2, 1)
    ok = require(bool(torch.equal(lab, want)), f"components of {G} graphs, one call per graph")
    best = min(ms_b, ms_g)
    log(f"cc batched {G} graphs ({int(voff[-1])} vertices, {int(eoff[-1])} pairs): "
        f"{ms_b:.3f} ms, graph {ms_g:.3f} ms, one call per graph {ms_p:.3f} ms")
    return {f"cc_batched_{G}_graphs": {
        "vertices": int(voff[-1]), "pairs": int(eoff[-1]), "batched_ms": round(ms_b, 3),
        "batched_graph_ms": round(ms_g, 3), "graph_capture_first_call_ms": round(cap_ms, 3),
        "plain_ms": round(ms_p, 3), "pairs_per_s": round(int(eoff[-1]) / (best * 1e-3), 1),
        "speedup_vs_plain": round(ms_p / best, 3), "correct": ok}}


def cc_families(torch, pj, dev, steps, m=8_000_000, comps=64):
    """The paper's graph families at m = 8M pairs: collections of random lists
    (degree 1), random k-ary trees, and random components of edge density d.
    Rounds, time, and device time per round of each step of a round."""
    fams = [("lists", None)] + [(f"trees_k{k}", k) for k in (2, 3, 4, 6, 8, 12, 16, 20)] + \
           [(f"components_d{d}", d) for d in (0.001, 0.01)]
    out = []
    for i, (name, par) in enumerate(fams):
        seed = W.SEED_BASE + 6 + i
        if name == "lists":
            src, dst, grp = W.list_graph(m + comps, comps, seed, with_groups=True)
        elif name.startswith("trees"):
            src, dst, grp = W.random_tree_graph(m + comps, par, comps, seed, with_groups=True)
        else:
            src, dst, grp = W.component_density_graph(m, par, comps, seed)
        nv = grp.shape[0]
        # expected labels from the construction: the smallest id of each group
        gmin = np.full(comps, nv, dtype=np.int64)
        np.minimum.at(gmin, grp.astype(np.int64), np.arange(nv))
        want = torch.from_numpy(gmin[grp].astype(np.int32)).to(dev)
        ds, dd = torch.from_numpy(src).to(dev), torch.from_numpy(dst).to(dev)
        lab = torch.empty(nv, dtype=torch.int32, device=dev)
        ms = timed(torch, lambda: pj.connected_components(ds, dd, nv, lab), steps, 1)
        ok = bool(torch.equal(lab, want))
        _, st = pj.connected_components(ds, dd, nv, lab, return_stats=True)
        r = max(1, st["rounds"])
        per_round = {k: round(v / r, 4) for k, v in st["phases"].items()
                     if k.startswith("sv") and k != "sv0_init" or k in ("compact", "flag_check")}
        out.append({"family": name, "n": nv, "m": int(src.shape[0]), "rounds": st["rounds"],
                    "ms": round(ms, 3), "edges_per_s": round(src.shape[0] / (ms * 1e-3), 1),
                    "ms_per_round": per_round, "correct": ok})
        log(f"cc family {name}: n {nv} m {src.shape[0]} rounds {st['rounds']} {ms:.3f} ms "
            f"correct {ok}")
        if not ok:
            raise SystemExit(f"components mismatch on the {name} family")
        del ds, dd, lab, want
    return {"cc_families_m8M": out}


def serving_pool(seed, lists=24, graphs=12):
    """Distinct inputs drawn from the serving mix, with their oracle results."""
    import oracle
    rng = np.random.default_rng(seed)
    pool = {"lr": [], "cc": []}
    for i in range(lists):
        n = int(np.floor(2 ** rng.uniform(10, 24)))
        s = W.random_list(n, seed + i)
        pool["lr"].append((s, oracle.list_rank(s)))
    for i in range(graphs):
        n = int(np.floor(2 ** rng.uniform(10, 22)))
        m = int(round(n * rng.uniform(2, 16) / 2))
        src, dst = W.random_graph(n, m, seed + 100 + i)
        pool["cc"].append((src, dst, n, oracle.connected_components(src, dst, n)))
    return pool


def serve_run(torch, S, pool, count, rate, seed, budget, check=True, keep=0):
    """Submit `count` requests (70% lists) with Poisson arrivals at `rate`
    per second (rate None: all at once); returns the server's stats, with the
    first `keep` results under "kept" as (kind, pool index, output)."""
    import threading
    rng = np.random.default_rng(seed)
    picks = [("lr", int(rng.integers(len(pool["lr"])))) if rng.random() < 0.7 else
             ("cc", int(rng.integers(len(pool["cc"])))) for _ in range(count)]
    gaps = rng.exponential(1.0 / rate, count) if rate else np.zeros(count)
    ids = [None] * count
    with S.Server(hbm_budget=budget, max_inflight=3, max_batch=64) as srv:
        def producer():
            t0 = time.perf_counter()
            due = 0.0
            for i, (kind, j) in enumerate(picks):
                due += gaps[i]
                delay = t0 + due - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                if kind == "lr":
                    ids[i] = srv.submit_list_rank(pool["lr"][j][0])
                else:
                    src, dst, n, _ = pool["cc"][j]
                    ids[i] = srv.submit_cc(src, dst, n)

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        srv.drain()
        bad = []
        kept = []
        for i, (rid, (kind, j)) in enumerate(zip(ids, picks)):
            st, _, out = srv.wait(rid)
            if i < keep:
                kept.append((kind, j, np.array(out, copy=True)))
            want = pool["lr"][j][1] if kind == "lr" else pool["cc"][j][3]
            wrong = int((out != want).sum()) if check and st == 0 else 0
            if st != 0 or wrong:
                bad.append({"request": i, "kind": kind, "input": j, "status": int(st),
                            "size": int(len(want)), "wrong": wrong})
        stats = srv.stats()
    for b in bad:
        log(f"serving mismatch {b}")
    stats["mismatches"] = len(bad)
    stats["kept"] = kept
    return stats


def run_serving(torch, pj, args):
    from paper_1002_4482_amd import serve as S
    log("serving: building the request pool")
    pool = serving_pool(W.SEED_BASE + 5)
    # pinned host copies keep the server's copies asynchronous
    pool["lr"] = [(torch.from_numpy(s).pin_memory(), r) for s, r in pool["lr"]]
    pool["cc"] = [(torch.from_numpy(a).pin_memory(), torch.from_numpy(b).pin_memory(), n, r)
                  for a, b, n, r in pool["cc"]]
    ex = {}
    serve_run(torch, S, pool, args.serve_warmup, None, 1, 16 << 30, check=False)  # warm-up
    # a burst long enough to reach steady state (short bursts overstate it)
    sat = serve_run(torch, S, pool, 1500, None, 2, 16 << 30)
    ex["serving_saturation_req_per_s"] = round(sat["req_per_s"], 1)
    log(f"serving saturation {sat['req_per_s']:.1f} req/s")
    # open-loop Poisson arrivals at fractions of the saturation rate; 0.75 is
    # the headline point
    sweep = {}
    for frac in (0.25, 0.5, 0.75, 0.9):
        lam = frac * sat["req_per_s"]
        st = serve_run(torch, S, pool, args.serve_requests, lam, 3, 16 << 30,
                       keep=12 if frac == 0.75 else 0)
        sweep[frac] = (lam, st)
        log(f"serving at {frac:.2f} x saturation ({lam:.1f} req/s): p50 {st['p50_ms']:.2f} ms "
            f"p99 {st['p99_ms']:.2f} ms {st['req_per_s']:.1f} req/s "
            f"mismatches {st['mismatches']}")
    ex["serving_sweep"] = [
        {"load": frac, "rate_req_per_s": round(lam, 1), "p50_ms": round(st["p50_ms"], 3),
         "p99_ms": round(st["p99_ms"], 3), "req_per_s": round(st["req_per_s"], 1),
         "completed": st["completed"], "mismatches": st["mismatches"]}
        for frac, (lam, st) in sweep.items()]
    lam, run = sweep[0.75]
    # a sample of served results re-run alone through the plain calls
    rerun_bad = 0
    for kind, j, out in run["kept"]:
        if kind == "lr":
            d = pool["lr"][j][0].cuda()
            alone = pj.list_rank(d).cpu().numpy()
        else:
            src, dst, n, _ = pool["cc"][j]
            alone = pj.connected_components(src.cuda(), dst.cuda(), n).cpu().numpy()
        rerun_bad += int(not np.array_equal(alone, out))
    ex["serving_rerun_sample"] = len(run["kept"])
    ex["serving_rerun_mismatches"] = rerun_bad
    # a burst under a 512 MiB budget: admission must wait for memory
    small = serve_run(torch, S, pool, 300, None, 4, 512 << 20)
    ex["serving_rate_req_per_s"] = round(lam, 1)
    for tag, st in (("serving", run), ("serving_512MiB", small)):
        ex[f"{tag}_p50_ms"] = round(st["p50_ms"], 3)
        ex[f"{tag}_p99_ms"] = round(st["p99_ms"], 3)
        ex[f"{tag}_req_per_s"] = round(st["req_per_s"], 1)
        ex[f"{tag}_items_per_s"] = round(st["items_per_s"], 1)
        ex[f"{tag}_completed"] = st["completed"]
        ex[f"{tag}_mismatches"] = st["mismatches"]
        ex[f"{tag}_ticks"] = st["ticks"]
        ex[f"{tag}_inflight_peak"] = st["inflight_peak"]
        ex[f"{tag}_budget_waits"] = st["budget_waits"]
        ex[f"{tag}_bytes_peak"] = st["bytes_peak"]
        log(f"{tag}: p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms "
            f"{st['req_per_s']:.1f} req/s mismatches {st['mismatches']}")
    log(f"serving re-run sample: {rerun_bad} of {len(run['kept'])} differ")
    bad = sum(st["mismatches"] for _, st in sweep.values()) + small["mismatches"] + \
        sat["mismatches"] + rerun_bad
    ex["serving_correct"] = require(bad == 0, f"serving: {bad} wrong or failed responses")
    return ex


if __name__ == "__main__":
    main()
