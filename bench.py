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


def kernel_key(name: str) -> str:
    """Normalise a launch tag "(k_count<K, F32, true, 256, 16>)" or a profiler
    name "rs::k_count<unsigned long, false, true, 256, 16>(rs::Work, ...)" to
    "k_count/l1/256/16" (count/scatter carry their level) or
    "k_local_sort/768/8"."""
    import re

    m = re.search(r"(k_[a-z_0-9]+)\s*<([^>]*)>", name)
    if not m:
        m2 = re.search(r"(k_[a-z_0-9]+)", name)
        return m2.group(1) if m2 else name
    base, args = m.group(1), [a.strip() for a in m.group(2).split(",")]
    nums = [a for a in args if a.isdigit()]
    parts = [base]
    if base in ("k_count", "k_scatter", "k_splitters") and len(args) > 2:
        parts.append("l1" if args[2] == "true" else "l2")
    return "/".join(parts + nums)


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
    if args.calib_copy_mib:
        # a plain device copy of known size, so that profiler byte counters
        # can be scaled by what they read for it
        cb = args.calib_copy_mib << 20
        src = torch.empty(cb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
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
        if traffic and kernel_key(dom_name) in traffic.get("kernels", {}):
            tr = traffic["kernels"][kernel_key(dom_name)]["hbm_bytes_per_launch"]
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


def _read_pmc(path, counter):
    """Per normalised kernel: (dispatches, mean counter value) from a rocprofv3
    counter_collection.csv."""
    import csv

    acc = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = kernel_key(r["Kernel_Name"]) if "rs::" in r["Kernel_Name"] else r["Kernel_Name"].split("(")[0]
        d = acc.setdefault(k, {})
        d[r["Dispatch_Id"]] = d.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return {k: (len(v), sum(v.values()) / len(v)) for k, v in acc.items()}


def pmc_summary(fetch_csv, write_csv, copy_mib, command, out_dir):
    """Scale FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by what they read for a
    plain copy of copy_mib MiB and write profiles/traffic.json + a text table."""
    f = _read_pmc(fetch_csv, "FETCH_SIZE")
    w = _read_pmc(write_csv, "WRITE_SIZE")
    copy = [k for k in f if "copyBuffer" in k or "copy" in k.lower()]
    if not copy:
        raise SystemExit("no copy kernel found for calibration")
    ck = max(copy, key=lambda k: f[k][1])
    cb = copy_mib << 20
    fr = cb / (f[ck][1] * 1024.0)
    fw = cb / (w[ck][1] * 1024.0) if ck in w and w[ck][1] > 0 else 1.0
    kern = {}
    for k in sorted(set(f) | set(w)):
        if not k.startswith("k_"):
            continue
        fb = f.get(k, (0, 0.0))[1] * 1024.0 * fr
        wb = w.get(k, (0, 0.0))[1] * 1024.0 * fw
        kern[k] = {"dispatches": f.get(k, w.get(k))[0], "fetch_bytes_per_launch": int(fb),
                   "write_bytes_per_launch": int(wb), "hbm_bytes_per_launch": int(fb + wb)}
    res = {"src_hash": src_hash(), "command": command,
           "calibration": {"copy_kernel": ck, "copy_bytes": cb, "fetch_kib": f[ck][1],
                           "write_kib": w.get(ck, (0, 0))[1], "fetch_scale": fr, "write_scale": fw},
           "kernels": kern}
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, "traffic.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    lines = ["HBM traffic per kernel launch from rocprofv3 FETCH_SIZE and WRITE_SIZE (two separate runs),",
             "scaled by the counters of a plain %d MiB device copy (%s): read x%.3f, write x%.3f." % (
                 copy_mib, ck, fr, fw),
             "command: " + command, "source hash: " + res["src_hash"], "",
             "%-28s %10s %14s %14s %14s" % ("kernel", "dispatches", "fetch MB", "write MB", "total MB")]
    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["hbm_bytes_per_launch"]):
        lines.append("%-28s %10d %14.2f %14.2f %14.2f" % (k, v["dispatches"], v["fetch_bytes_per_launch"] / 1e6,
                                                          v["write_bytes_per_launch"] / 1e6,
                                                          v["hbm_bytes_per_launch"] / 1e6))
    with open(os.path.join(out_dir, "hbm_traffic_plain_2p28_u64.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def trace_summary(stats_csv, command, out_path, title):
    """Short text table from a rocprofv3 --stats kernel_stats.csv."""
    import csv

    rows = list(csv.DictReader(open(stats_csv)))
    lines = [title, "command: " + command, "source hash: " + src_hash(), "",
             "%-34s %7s %12s %12s %7s" % ("kernel", "calls", "total ms", "avg us", "%")]
    for r in rows:
        nm = r.get("Name") or r.get("KernelName") or ""
        key = kernel_key(nm) if "rs::" in nm else nm[:34]
        lines.append("%-34s %7s %12.3f %12.1f %7.2f" % (key[:34], r.get("Calls"), float(r.get("TotalDurationNs", 0)) / 1e6,
                                                       float(r.get("AverageNs", 0)) / 1e3,
                                                       float(r.get("Percentage", 0))))
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a plain device copy of this size before timing (profiler calibration)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc runs into profiles/ (no GPU needed)")
    ap.add_argument("--trace-summary", metavar="KERNEL_STATS_CSV",
                    help="summarise a rocprofv3 --stats run into profiles/ (no GPU needed)")
    ap.add_argument("--profile-command", default="", help="command recorded in the summaries")
    ap.add_argument("--profile-name", default="kernel_trace_plain_2p28_u64.txt")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-log2", type=int, default=28)
    ap.add_argument("--workload", default="plain", choices=["plain", "batched", "small", "serving"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.calib_copy_mib or 1024, args.profile_command,
                    os.path.join(ROOT, "profiles"))
        return
    if args.trace_summary:
        trace_summary(args.trace_summary, args.profile_command, os.path.join(ROOT, "profiles", args.profile_name),
                      "rocprofv3 --kernel-trace --stats summary")
        return
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
