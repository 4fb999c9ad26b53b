#!/usr/bin/env python3
"""Benchmark of the robust multilevel sample sort on one MI355X.

Default workload: plain sort of n = 2^28 uint64 keys with two levels of 256
buckets, over the five input families Uniform, Gaussian, Zero, DeterDupl and
Reverse (one step = one sort of one 2^28-key array; the timed steps cycle
through the five).  Inputs are generated on the host from fixed seeds and are
resident in HBM before timing starts.

Prints ONE JSON line with the metric, the roofline of the dominant kernel
(algorithmic bytes per launch / its average event-timed duration), the
per-pass rooflines, and the CPU oracle timed on a bounded sample.

Other workloads (--workload): "batched" (segmented sort of many uneven
arrays vs one plain sort per array), "small" (many equal small arrays by
RFIS / RQuick / merge sort), "serving" (Poisson request stream through the
sort server, p50/p99 latency).
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

HBM_PEAK_GBS = 8000.0
DISTS = ["uniform", "gaussian", "zero", "deterdupl", "reverse"]


def src_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1606_08766_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM traffic per kernel measured with rocprofv3 counters (committed under
    profiles/); ignored when the kernel sources changed since."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("src_hash") != src_hash():
        return None
    return t


def kernel_class(name: str) -> str:
    """Map a launch tag to the pass it implements."""
    if "k_count" in name:
        return "count_l1" if "F32, true" in name else "count_l2"
    if "k_scatter" in name:
        return "scatter_l1" if "F32, true" in name else "scatter_l2"
    if any(s in name for s in ("k_local_sort", "k_rfis", "k_rquick", "k_oversize")):
        return "local_sort"
    if "k_splitters" in name:
        return "splitters"
    if "k_scan" in name:
        return "scan"
    return "other"


def pass_bytes_per_key(ks: int):
    """Algorithmic HBM bytes per key of each pass (read + write), u64 keys,
    u32 positions: see the design doc."""
    return {
        "count_l1": ks,                 # read keys
        "scatter_l1": ks + ks + 4,      # read keys; write key + position
        "count_l2": ks + 4,             # read key + position
        "scatter_l2": 2 * (ks + 4),     # read and write key + position
        "local_sort": 2 * (ks + 4),     # read key + position; write key + perm
    }


def cpu_baseline(n_log2: int, budget_s: float = 20.0):
    """The oracle (std::sort of (key, position) records, multi-threaded) on a
    bounded sample of the same workload."""
    from gen import gen
    from oracle import oracle as O

    threads = max(1, min(os.cpu_count() or 1, 16))
    m = 1 << min(n_log2, 24)
    tot_keys, tot_t = 0, 0.0
    for d in DISTS:
        x = gen.keys("u64", d, m, seed=1)
        t0 = time.perf_counter()
        O.sort(x, threads=threads)
        tot_t += time.perf_counter() - t0
        tot_keys += m
        if tot_t > budget_s:
            break
    return {"value": round(tot_keys / tot_t / 1e9, 4), "unit": "Gkeys/s", "cores": threads, "kind": "oracle",
            "sample": "2^%d u64 keys per distribution over %s, std::sort of (key, position) records on %d "
                      "threads with a pairwise merge tree" % (min(n_log2, 24), "/".join(DISTS), threads)}


def bench_plain(args, R, torch):
    from gen import gen

    n = 1 << args.n_log2
    ks = 8
    inputs = []
    for d in DISTS:
        x = gen.keys("u64", d, n, seed=1)
        inputs.append(torch.from_numpy(x).cuda())
        del x
    ko = torch.empty_like(inputs[0])
    po = torch.empty(n, dtype=torch.uint32, device="cuda")
    ws = torch.empty(R.plain_workspace_bytes(R.U64, n), dtype=torch.uint8, device="cuda")
    for s in range(args.warmup):
        R.sort(inputs[s % len(DISTS)], workspace=ws, out=(ko, po))
    torch.cuda.synchronize()
    # per-distribution time (events around each step; reported, not the metric)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    R.timing_begin()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record()
        R.sort(inputs[s % len(DISTS)], workspace=ws, out=(ko, po))
        ev[s][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = R.timing_end()
    per_dist = {}
    for s in range(args.steps):
        per_dist.setdefault(DISTS[s % len(DISTS)], []).append(ev[s][0].elapsed_time(ev[s][1]))
    per_dist = {d: round(n / (sum(v) / len(v) / 1e3) / 1e9, 3) for d, v in per_dist.items()}
    st = R.stats(ws)
    if st["status"] != 0:
        raise RuntimeError("device status %d" % st["status"])
    elapsed = t1 - t0
    # per-pass rooflines from the event timing
    bpk = pass_bytes_per_key(ks)
    agg = {}
    for name, (cnt, ms) in timing.items():
        c = kernel_class(name)
        a = agg.setdefault(c, {"launches": 0, "ms": 0.0, "kernels": []})
        a["launches"] += cnt
        a["ms"] += ms
        a["kernels"].append(name)
    passes = {}
    for c, a in agg.items():
        e = {"ms_per_sort": round(a["ms"] / args.steps, 4)}
        if c in bpk:
            gbs = bpk[c] * n / (a["ms"] / args.steps / 1e3) / 1e9
            e["GB_s"] = round(gbs, 1)
            e["frac"] = round(gbs / HBM_PEAK_GBS, 4)
        passes[c] = e
    # dominant single kernel (by total time)
    dom_name, (dom_cnt, dom_ms) = max(timing.items(), key=lambda kv: kv[1][1])
    dom_class = kernel_class(dom_name)
    traffic = load_traffic()
    roof = None
    if dom_class in bpk:
        # launches of this kernel per sort, and the keys one launch processes
        launches_per_sort = dom_cnt / args.steps
        keys_per_launch = n / launches_per_sort if dom_class != "local_sort" else None
        if keys_per_launch is None:
            # a local-sort class kernel processes the keys of its size class
            keys_per_launch = n * (dom_ms / agg["local_sort"]["ms"]) / launches_per_sort
        alg = bpk[dom_class] * keys_per_launch
        avg_s = dom_ms / dom_cnt / 1e3
        achieved = alg / avg_s / 1e9
        tr = None
        if traffic and dom_name in traffic.get("kernels", {}):
            tr = traffic["kernels"][dom_name]["bytes_per_launch"]
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr, "kernel": dom_name,
                "alg_bytes_per_launch": int(alg)}
    value = args.steps * n / elapsed / 1e9
    out = {
        "metric": "Gkeys/s (plain multilevel sample sort, 2^%d u64 keys)" % args.n_log2,
        "value": round(value, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "plain sort of 2^%d uint64 keys, 2 levels x 256 buckets, distributions %s (steps "
                               "cycle through them)" % (args.n_log2, "/".join(DISTS)),
                   "n": n, "levels": int(st["levels"]), "key_bytes": ks, "perm": True},
        "roofline": roof,
        "passes": passes,
        "gkeys_per_s_by_distribution": per_dist,
        "hbm_bytes_per_key_algorithmic": sum(bpk.values()),
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-log2", type=int, default=28)
    ap.add_argument("--workload", default="plain", choices=["plain", "batched", "small", "serving"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this sort's multi-GPU path is a design, not a build "
              "(see DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1606_08766_amd import rsort as R

    if args.workload == "plain":
        out = bench_plain(args, R, torch)
    else:
        from paper_1606_08766_amd import workloads

        out = workloads.run(args.workload, args, R, torch)
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        out["cpu_baseline"] = cpu_baseline(args.n_log2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
