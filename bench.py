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
import collections
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


def load_traffic(name: str = "traffic.json"):
    """HBM traffic per kernel measured with rocprofv3 counters (committed under
    profiles/); ignored when the kernel sources changed since."""
    p = os.path.join(ROOT, "profiles", name)
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
    if any(s in name for s in ("k_local_sort", "k_local_words", "k_rfis", "k_rquick", "k_oversize")):
        return "local_sort"
    if "k_splitters" in name:
        return "splitters"
    if "k_scan" in name:
        return "scan"
    return "other"


def pass_bytes_per_key(ks: int):
    """Algorithmic HBM bytes per key of each pass (read + write) for keys of
    ks bytes and u32 positions: every byte a pass must move, counted once.
    The second level's count needs only the key (plus the position of a key
    that ties a splitter key, not counted here); the bytes a record layout
    or a bucket-id array adds on top show up in the measured traffic ratio."""
    return {
        "count_l1": ks,                 # read keys
        "scatter_l1": ks + ks + 4,      # read keys; write (key, position)
        "count_l2": ks,                 # read keys
        "scatter_l2": 2 * (ks + 4),     # read and write (key, position)
        "local_sort": 2 * (ks + 4),     # read (key, position); write key + perm
    }


def cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(n_log2: int, budget_s: float = 25.0):
    """The oracle (std::sort of (key, position) records) on a bounded sample
    of the same workload: all host threads (chunk sorts + pairwise merges),
    then one thread, over the five distributions."""
    from gen import gen
    from oracle import oracle as O

    model, nproc = cpu_info()
    m = 1 << min(n_log2, 24)
    xs = [gen.keys("u64", d, m, seed=1) for d in DISTS]
    res = {}
    for name, threads in (("all", nproc), ("one", 1)):
        tot_keys, tot_t = 0, 0.0
        for x in xs:
            t0 = time.perf_counter()
            O.sort(x, threads=threads)
            tot_t += time.perf_counter() - t0
            tot_keys += m
            if tot_t > budget_s / 2:
                break
        res[name] = (tot_keys / tot_t / 1e9, tot_keys)
    return {"value": round(res["all"][0], 4), "unit": "Gkeys/s", "cores": nproc, "kind": "oracle",
            "sample": "2^%d u64 keys per distribution over %s (%d keys with all threads, %d with one), std::sort "
                      "of (key, position) records, chunk sorts + pairwise merge tree on %d threads"
                      % (min(n_log2, 24), "/".join(DISTS), res["all"][1], res["one"][1], nproc),
            "single_thread_value": round(res["one"][0], 4), "cpu_model": model, "host_threads": nproc}


def bandwidth_ceilings(R, torch, nbytes: int = 2 << 30, reps: int = 5):
    """Rates of the library's own read-only and copy kernels over nbytes
    (practical ceilings of a read pass and of a read + write pass)."""
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for kind, moved in (("read", nbytes), ("copy", 2 * nbytes)):
        for _ in range(2):
            R.bandwidth_probe(kind, src, dst, nbytes)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            R.bandwidth_probe(kind, src, dst, nbytes)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b) / reps
        gbs = moved / (ms / 1e3) / 1e9
        out[kind] = {"GB_s": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes": moved,
                     "ms": round(ms, 4)}
    del src, dst
    return out


def calib_copy(args, R, torch):
    """One run of the library's copy probe over calib_copy_mib MiB (reads and
    writes that many bytes), so that profiler byte counters can be scaled by
    what they read for a copy of known size."""
    cb = args.calib_copy_mib << 20
    src = torch.ones(cb // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    R.bandwidth_probe("copy", src, dst, cb)
    torch.cuda.synchronize()
    del src, dst


def bench_plain(args, R, torch):
    from gen import gen

    n = 1 << args.n_log2
    kt_name = args.key_type
    kt = {"u64": R.U64, "u32": R.U32, "f32": R.F32}[kt_name]
    ks = 8 if kt_name == "u64" else 4
    inputs = []
    for d in DISTS:
        x = gen.keys(kt_name, d, n, seed=1)
        inputs.append(torch.from_numpy(x).cuda())
        del x
    ko = torch.empty_like(inputs[0])
    po = torch.empty(n, dtype=torch.uint32, device="cuda")
    ws = torch.empty(R.plain_workspace_bytes(kt, n), dtype=torch.uint8, device="cuda")
    if args.calib_copy_mib:
        calib_copy(args, R, torch)
    for s in range(args.warmup):
        R.sort(inputs[s % len(DISTS)], workspace=ws, out=(ko, po))
    torch.cuda.synchronize()
    # per-distribution time (events around each step; reported, not the metric)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record()
        R.sort(inputs[s % len(DISTS)], workspace=ws, out=(ko, po))
        ev[s][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the same steps again with an event pair around every kernel launch, for
    # the per-pass figures (kept out of the timed region above)
    R.timing_begin()
    for s in range(args.steps):
        R.sort(inputs[s % len(DISTS)], workspace=ws, out=(ko, po))
    torch.cuda.synchronize()
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
    traffic = load_traffic() if kt_name == "u64" and args.n_log2 == 28 else None
    passes = {}
    for c, a in agg.items():
        e = {"ms_per_sort": round(a["ms"] / args.steps, 4)}
        if c in bpk:
            gbs = bpk[c] * n / (a["ms"] / args.steps / 1e3) / 1e9
            e["alg_bytes_per_key"] = bpk[c]
            e["GB_s"] = round(gbs, 1)
            e["frac"] = round(gbs / HBM_PEAK_GBS, 4)
            if traffic:
                # measured HBM bytes per sort (rocprofv3 FETCH_SIZE + WRITE_SIZE of
                # every kernel of the pass) over the pass's algorithmic bytes
                meas = 0.0
                for k in a["kernels"]:
                    kk = kernel_key(k)
                    if kk in traffic["kernels"]:
                        meas += traffic["kernels"][kk]["hbm_bytes_per_launch"] * timing[k][0] / args.steps
                e["traffic_ratio"] = round(meas / (bpk[c] * n), 3) if meas else None
        passes[c] = e
    # dominant single kernel (by total time)
    dom_name, (dom_cnt, dom_ms) = max(timing.items(), key=lambda kv: kv[1][1])
    dom_class = kernel_class(dom_name)
    roof = None
    if dom_class in bpk:
        # launches of this kernel per sort, and the keys one launch processes
        launches_per_sort = dom_cnt / args.steps
        if dom_class != "local_sort":
            keys_per_launch = n / launches_per_sort
        else:
            # a local-sort kernel sorts the keys of one size class: exact count
            # per distribution from the device statistics, averaged over the mix
            import re

            nums = [int(v) for v in re.findall(r"\b(\d+)\b", dom_name)]
            if "k_rfis" in dom_name:
                caps = {nums[-1]}
            elif "k_rquick" in dom_name:
                caps = {nums[-2]} if nums[-2] <= 2048 else {3072, 4096}
            else:
                caps = {nums[-2] * nums[-1]}
            ks_sum = 0
            for s in range(args.steps):
                R.sort(inputs[s % len(DISTS)], workspace=ws, out=(ko, po))
                for cmax, _, keys in R.class_stats(ws):
                    if cmax in caps:
                        ks_sum += keys
            keys_per_launch = ks_sum / args.steps / launches_per_sort
        alg = bpk[dom_class] * keys_per_launch
        avg_s = dom_ms / dom_cnt / 1e3
        achieved = alg / avg_s / 1e9
        tr = None
        # the committed counters were taken on the 2^28 u64 sort
        if traffic and kernel_key(dom_name) in traffic.get("kernels", {}):
            tr = traffic["kernels"][kernel_key(dom_name)]["hbm_bytes_per_launch"]
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr, "kernel": dom_name,
                "alg_bytes_per_launch": int(alg)}
    value = args.steps * n / elapsed / 1e9
    out = {
        "metric": "Gkeys/s (plain multilevel sample sort, 2^%d %s keys)" % (args.n_log2, kt_name),
        "value": round(value, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": kt_name,
        "data": "synthetic",
        "config": {"workload": "plain sort of 2^%d %s keys, %d levels, distributions %s (steps "
                               "cycle through them)" % (args.n_log2, kt_name, int(st["levels"]), "/".join(DISTS)),
                   "n": n, "levels": int(st["levels"]), "key_bytes": ks, "perm": True},
        "roofline": roof,
        "passes": passes,
        "gkeys_per_s_by_distribution": per_dist,
        "hbm_bytes_per_key_algorithmic": sum(bpk.values()),
    }
    return out


def _timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def bench_batched(args, R, torch):
    """Config 4: 100k segments with log-uniform sizes, u64 keys + u32 payload,
    Uniform / Zero / DeterDupl per segment.  One rsort_segmented call against
    rsort_plain per segment (keys + perm only, back to back on one stream)."""
    from gen import gen

    count = 100_000
    hi = 18 if args.batched_variant == "literal" else 13
    sizes = gen.log_uniform_sizes(count, 0, hi, seed=1)
    dists = gen.pick_dists(count, ["uniform", "zero", "deterdupl"], seed=2)
    keys, pay, off = gen.segmented("u64", sizes, dists, seed=3)
    n = keys.size
    dk, dp, do = torch.from_numpy(keys).cuda(), torch.from_numpy(pay).cuda(), torch.from_numpy(off).cuda()
    del keys, pay
    ko, po, plo = torch.empty_like(dk), torch.empty(n, dtype=torch.uint32, device="cuda"), torch.empty_like(dp)
    ws = torch.empty(R.segmented_workspace_bytes(R.U64, n, count, True), dtype=torch.uint8, device="cuda")
    if args.calib_copy_mib:
        calib_copy(args, R, torch)
    t_b = _timed(torch, lambda: R.segmented_sort(dk, do, dp, workspace=ws, out=(ko, po, plo)), args.steps, args.warmup)
    # per-pass figures from a separate, instrumented run
    R.timing_begin()
    for _ in range(args.steps):
        R.segmented_sort(dk, do, dp, workspace=ws, out=(ko, po, plo))
    torch.cuda.synchronize()
    timing = R.timing_end()
    if R.workspace_status(ws) != 0:
        raise RuntimeError("segmented sort reported an error")
    # plain baseline on the first segments (enough for a stable rate)
    m = 4000
    offh = off[:m + 1]
    npl = int(offh[-1])
    wsp = torch.empty(max(R.plain_workspace_bytes(R.U64, int(sizes[:m].max())), 256), dtype=torch.uint8,
                      device="cuda")

    def plain_loop():
        for s in range(m):
            a, b = int(offh[s]), int(offh[s + 1])
            if b > a:
                R.sort(dk[a:b], workspace=wsp, out=(ko[a:b], po[a:b]))

    t_p = _timed(torch, plain_loop, 1, 1)
    batched = n / t_b / 1e9
    plain = npl / t_p / 1e9
    per = {}
    calls = args.steps
    for name, (cnt, ms) in timing.items():
        c = kernel_class(name)
        per[c] = round(per.get(c, 0.0) + ms / calls, 4)
    # algorithmic bytes per pass: keys of segments longer than the LDS
    # capacity of a payload call (8192) take sample-sort levels
    cap = 8192
    n_lv = int(sizes[sizes > cap].sum())
    n_in = n - n_lv
    pass_bytes = {"count_l1": 8 * n_lv,                        # keys
                  "scatter_l1": (8 + 4 + 12 + 4) * n_lv,       # key + payload in; record + payload out
                  "local_sort": (8 + 4 + 16) * n_in + (12 + 4 + 16) * n_lv}  # in; key + payload + perm out
    traffic = load_traffic("traffic_batched_1gib.json") if args.batched_variant == "1gib" else None
    passes = {}
    for c, ms in per.items():
        e = {"ms_per_call": ms}
        if c in pass_bytes and ms > 0 and pass_bytes[c]:
            gbs = pass_bytes[c] / (ms / 1e3) / 1e9
            e.update({"alg_bytes": pass_bytes[c], "GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
            if traffic:
                # measured HBM bytes per call of the pass's kernels (rocprofv3
                # FETCH_SIZE + WRITE_SIZE) over its algorithmic bytes
                meas = sum(traffic["kernels"][kernel_key(k)]["hbm_bytes_per_launch"] * timing[k][0] / calls
                           for k in timing if kernel_class(k) == c and kernel_key(k) in traffic["kernels"])
                e["traffic_ratio"] = round(meas / pass_bytes[c], 3) if meas else None
        passes[c] = e
    return {
        "metric": "Gkeys/s (batched segmented sort, %d segments)" % count,
        "value": round(batched, 3), "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_b * 1e3, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "100k segments, sizes log-uniform in [1, 2^%d], u64 keys + u32 payload, "
                               "Uniform/Zero/DeterDupl per segment" % hi, "n": n, "segments": count},
        "plain_per_segment_gkeys_s": round(plain, 3), "batched_over_plain": round(batched / plain, 2),
        "plain_sample": "rsort_plain on the first %d segments (%d keys), keys + perm only" % (m, npl),
        "passes": passes, "keys_in_levels": n_lv,
    }


def bench_latency(args, R, torch):
    """Config 1: one plain sort of 2^20 uniform u64 keys (seed 1), single
    level of 256 buckets then the local sorts; keys + permutation.  Each sort
    is timed alone with events on the stream it runs on."""
    import numpy as np

    from gen import gen

    n = 1 << 20
    x = torch.from_numpy(gen.keys("u64", "uniform", n, seed=1)).cuda()
    ko = torch.empty_like(x)
    po = torch.empty(n, dtype=torch.uint32, device="cuda")
    us = []
    with R.tuned(target=4096):  # one level of 256 buckets of about 4096 keys
        ws = torch.empty(R.plain_workspace_bytes(R.U64, n), dtype=torch.uint8, device="cuda")
        for _ in range(max(args.warmup, 3)):
            R.sort(x, workspace=ws, out=(ko, po))
        torch.cuda.synchronize()
        st = R.stats(ws)
        for _ in range(max(args.steps, 20)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            R.sort(x, workspace=ws, out=(ko, po))
            b.record()
            b.synchronize()
            us.append(a.elapsed_time(b) * 1e3)
    us = np.array(us)
    mean = float(us.mean())
    return {"metric": "us per plain sort of 2^20 u64 keys (latency)", "value": round(mean, 2), "unit": "us",
            "n_gpus": 1, "steps": int(us.size), "warmup": max(args.warmup, 3), "ms_per_step": round(mean / 1e3, 4),
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
            "data": "synthetic",
            "config": {"workload": "plain sort of 2^20 uniform uint64 keys (seed 1), single level of 256 buckets",
                       "n": n, "levels": int(st["levels"]), "buckets": int(st["k"])},
            "p50_us": round(float(np.percentile(us, 50)), 2), "min_us": round(float(us.min()), 2),
            "gkeys_per_s": round(n / mean / 1e3, 3)}


def bench_small(args, R, torch):
    """Config 3: 2^14 independent arrays of n in {64, 256, 1024, 4096} u32 keys
    (uniform, 8 distinct values) by RFIS, RQuick and the LDS merge sort."""
    from gen import gen

    arrays = 1 << 14
    rows = []
    algos = {"rfis": dict(rfis_max=1024, rquick_max=1), "rquick": dict(rfis_max=1, rquick_max=4096),
             "merge": dict(rfis_max=1, rquick_max=1)}
    for n in (64, 256, 1024, 4096):
        if args.small_n and n != args.small_n:
            continue
        for dist in ("uniform", "dup8"):
            x = gen.keys("u32", "uniform" if dist == "uniform" else "topbits", arrays * n, seed=1,
                         param=0 if dist == "uniform" else 3)
            off = torch.arange(0, arrays * n + 1, n, dtype=torch.int64).cuda()
            dx = torch.from_numpy(x).cuda()
            ko, po = torch.empty_like(dx), torch.empty(dx.numel(), dtype=torch.uint32, device="cuda")
            ws = torch.empty(R.segmented_workspace_bytes(R.U32, dx.numel(), arrays, False), dtype=torch.uint8,
                             device="cuda")
            for a, tune in algos.items():
                if args.small_algo and a != args.small_algo:
                    continue
                if a == "rfis" and n > 1024:
                    continue
                if a == "rquick" and n < 2048:
                    continue
                with R.tuned(**tune):
                    t = _timed(torch, lambda: R.segmented_sort(dx, off, workspace=ws, out=(ko, po, None)), args.steps,
                               args.warmup)
                row = {"n": n, "dist": dist, "algo": a, "ms": round(t * 1e3, 4), "arrays_per_s": round(arrays / t),
                       "gkeys_s": round(arrays * n / t / 1e9, 3)}
                if a == "rfis":
                    row["compares_per_s"] = float("%.4g" % (arrays * n * n / t))
                rows.append(row)
    best = max([r["gkeys_s"] for r in rows if r["n"] == 4096] or [0.0])
    return {"metric": "Gkeys/s (2^14 small arrays, best algorithm at n = 4096)", "value": best, "unit": "Gkeys/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": "2^14 arrays x n in {64, 256, 1024, 4096}, u32 uniform / 8 distinct values"},
            "rows": rows}


def bench_rquick_mw(args, R, torch):
    """Robust hypercube quicksort over 2^log2_p workgroups (exchanges through
    HBM) against the sample sort on the same single array: u32 keys, uniform
    and all-equal, split by (key, position), by key only, and by the paper's
    local choice among copies of the splitter key.  Reports the largest PE
    part after the last exchange (load balance) next to the times."""
    from gen import gen

    rows = []
    for n, lp in ((1 << 13, 2), (1 << 15, 3), (1 << 16, 4), (1 << 18, 5), (1 << 18, 6), (1 << 18, 8), (1 << 21, 8)):
        for dist in ("uniform", "zero"):
            x = torch.from_numpy(gen.keys("u32", dist, n, seed=1)).cuda()
            ws = torch.empty(R.rquick_mw_workspace_bytes(n, lp), dtype=torch.uint8, device="cuda")
            wsp = torch.empty(R.plain_workspace_bytes(R.U32, n), dtype=torch.uint8, device="cuda")
            row = {"n": n, "log2_p": lp, "dist": dist}
            for name, tb in (("rquick_tb", 1), ("rquick_ntb", 0), ("rquick_local", 2)):
                t = _timed(torch, lambda: R.rquick_mw(x, lp, tie_break=tb, workspace=ws), args.steps, args.warmup)
                row[name + "_us"] = round(t * 1e6, 1)
                row[name + "_max_part"] = int(R.rquick_mw(x, lp, tie_break=tb, workspace=ws)[2][-1].item())
            row["sample_sort_us"] = round(_timed(torch, lambda: R.sort(x, workspace=wsp), args.steps,
                                                 args.warmup) * 1e6, 1)
            row["n_over_p"] = n >> lp
            rows.append(row)
    ref = [r for r in rows if r["n"] == 1 << 18 and r["log2_p"] == 5 and r["dist"] == "uniform"][0]
    return {"metric": "us per hypercube-quicksort of 2^18 u32 keys over 32 workgroups", "value": ref["rquick_tb_us"],
            "unit": "us", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": "one array of 2^13..2^21 u32 keys, uniform / all equal, 4..256 workgroups"},
            "rows": rows}


def bench_serving(args, R, torch):
    """Config 5: Poisson stream of sort requests through the sort server at
    0.5x and 0.8x of its measured closed-loop rate; sizes log-uniform in
    [2^8, 2^26], key type and distribution drawn per request; 64 GiB budget."""
    import numpy as np

    from gen import gen

    pool_n = 1 << 26
    kts = [("u32", R.U32), ("u64", R.U64), ("f32", R.F32)]
    pool = {}
    for kname, kt in kts:
        for d in DISTS:
            pool[(kname, d)] = torch.from_numpy(gen.keys(kname, d, pool_n, seed=5)).cuda()
    rng = np.random.default_rng(1)
    total = args.requests + args.serve_warmup
    sizes = np.floor(2.0 ** rng.uniform(8, 26, total)).astype(np.int64)
    kinds = [(kts[rng.integers(3)], DISTS[rng.integers(5)]) for _ in range(total)]
    offs = [int(rng.integers(0, pool_n - s + 1)) for s in sizes]
    # every request writes to its own region of one output arena, so the
    # client never waits for a buffer: latency is the server's alone
    # output ring of 2^32 keys (+ perm): a request takes the next region that
    # no pending request holds (regions are freed oldest first), so a client
    # waits for a buffer only when 2^32 keys are pending
    ring = 1 << 32
    arena_k = torch.empty(ring, dtype=torch.uint64, device="cuda")
    arena_p = torch.empty(ring, dtype=torch.uint32, device="cuda")
    budget = 64 << 30
    inflight = args.serve_slots

    def run(qps):
        lat, keys, starts, ends = [], 0, [], []
        live = collections.OrderedDict()  # ticket -> region start, in allocation order
        head = 0

        def place(n):
            lo = next(iter(live.values())) if live else None
            for pos in ((head,) if head + n <= ring else ()) + (0,):
                if pos + n > ring:
                    continue
                if lo is None or (lo < head and (pos >= head or pos + n <= lo)) or (head <= lo and pos >= head
                                                                                  and pos + n <= lo):
                    return pos
            return None

        with R.Server(device=0, hbm_budget_bytes=budget, max_inflight=inflight) as s:
            t0 = time.monotonic_ns()
            gaps = rng.exponential(1.0 / qps, total) if qps else np.zeros(total)
            arrive = t0 + np.cumsum(gaps * 1e9).astype(np.int64)
            pending = {}
            i = 0
            while i < total or pending:
                now = time.monotonic_ns()
                while i < total and arrive[i] <= now:
                    (kname, kt), d = kinds[i]
                    src = pool[(kname, d)]
                    n = int(sizes[i])
                    pos = place(n)
                    if pos is None:
                        break
                    tk = s.submit(kt, src.data_ptr() + offs[i] * src.element_size(), n,
                                  arena_k.data_ptr() + 8 * pos, arena_p.data_ptr() + 4 * pos)
                    live[tk] = pos
                    head = pos + n
                    pending[tk] = (i, int(arrive[i]))
                    i += 1
                done = []
                for tk, (j, arr) in pending.items():
                    rc, r = s.poll(tk)
                    if rc != R.PENDING:
                        if rc != R.OK:
                            raise RuntimeError("request failed: %d" % rc)
                        done.append(tk)
                        if j >= args.serve_warmup:
                            lat.append((r.t_done_ns - arr) / 1e6)
                            keys += int(sizes[j])
                            starts.append(r.t_start_ns)
                            ends.append(r.t_done_ns)
                for tk in done:
                    del pending[tk]
                    del live[tk]
                    s.release(tk)
                if not done:
                    time.sleep(20e-6)
        span = (max(ends) - min(starts)) / 1e9
        # busy fraction: share of the span with at least one request on the GPU
        busy, cur_s, cur_e = 0, None, None
        for a, b in sorted(zip(starts, ends)):
            if cur_e is None or a > cur_e:
                if cur_e is not None:
                    busy += cur_e - cur_s
                cur_s, cur_e = a, b
            else:
                cur_e = max(cur_e, b)
        busy += cur_e - cur_s
        lat = np.array(lat)
        return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "gkeys_s": round(keys / span / 1e9, 3), "requests": int(lat.size),
                "gpu_busy_frac": round(busy / 1e9 / span, 3)}

    closed = run(0)  # all requests released at once: closed-loop saturation
    sat_qps = closed["requests"] / ((closed["requests"] * np.mean(sizes)) / (closed["gkeys_s"] * 1e9))
    res = {"closed_loop": closed, "saturation_qps": round(float(sat_qps), 1)}
    for f in (0.5, 0.8):
        res["qps_%.1fx" % f] = dict(run(f * sat_qps), qps=round(float(f * sat_qps), 1))
    return {"metric": "p50/p99 sort-request latency (ms) at 0.5x / 0.8x saturation QPS",
            "value": res["qps_0.8x"]["p99_ms"], "unit": "ms (p99 at 0.8x saturation)", "n_gpus": 1,
            "steps": total, "warmup": args.serve_warmup, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32/u64/f32", "data": "synthetic",
            "config": {"workload": "Poisson sort requests, sizes log-uniform [2^8, 2^26], key type uniform over "
                                   "u32/u64/f32, 5 distributions, 64 GiB budget, %d streams" % inflight},
            "serving": res}


def run_extras(args, R, torch):
    """The other configurations, run after the headline and reported as extra
    keys of the same JSON line: 2^20-key latency, 2^14 small arrays, the
    batched segmented sort (1 GiB and literal variants, each against one
    plain sort per segment) and the serving loop (p50/p99 at 0.5x and 0.8x of
    its saturation rate).  Progress goes to stderr."""
    extras = {}

    def step(name, fn):
        t0 = time.perf_counter()
        sys.stderr.write("[bench] %s ...\n" % name)
        sys.stderr.flush()
        r = fn()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        sys.stderr.write("[bench] %s done in %.1f s\n" % (name, time.perf_counter() - t0))
        sys.stderr.flush()
        return r

    lat = step("config 1 latency", lambda: bench_latency(args, R, torch))
    extras["config1_latency"] = {"us_mean": lat["value"], "p50_us": lat["p50_us"], "min_us": lat["min_us"],
                                 "gkeys_s": lat["gkeys_per_s"], "sorts": lat["steps"], "config": lat["config"]}
    sm = step("config 3 small arrays", lambda: bench_small(args, R, torch))
    extras["config3_small"] = {"rows": sm["rows"], "best_gkeys_s_n4096": sm["value"], "config": sm["config"]}
    b4 = {}
    for variant in ("1gib", "literal"):
        a = argparse.Namespace(**vars(args))
        a.batched_variant = variant
        r = step("config 4 batched (%s)" % variant, lambda: bench_batched(a, R, torch))
        b4[variant] = {"gkeys_s": r["value"], "ms_per_call": r["ms_per_step"],
                       "plain_per_segment_gkeys_s": r["plain_per_segment_gkeys_s"],
                       "batched_over_plain": r["batched_over_plain"], "plain_sample": r["plain_sample"],
                       "passes": r["passes"], "config": r["config"]}
    extras["config4_batched"] = b4
    sv = step("config 5 serving", lambda: bench_serving(args, R, torch))
    extras["config5_serving"] = dict(sv["serving"], slots=args.serve_slots, config=sv["config"])
    return extras


def _read_pmc(path, counter):
    """Per normalised kernel: (dispatches, mean counter value) from a rocprofv3
    counter_collection.csv."""
    import csv

    acc = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = kernel_key(r["Kernel_Name"]) if "rs::k_" in r["Kernel_Name"] else r["Kernel_Name"].split("(")[0]
        d = acc.setdefault(k, {})
        d[r["Dispatch_Id"]] = d.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return {k: (len(v), sum(v.values()) / len(v)) for k, v in acc.items()}


def pmc_summary(fetch_csv, write_csv, copy_mib, command, out_dir, name="hbm_traffic_plain_2p28_u64.txt",
                json_name="traffic.json"):
    """Scale FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by what they read for a
    plain copy of copy_mib MiB and write profiles/traffic.json + a text table."""
    f = _read_pmc(fetch_csv, "FETCH_SIZE")
    w = _read_pmc(write_csv, "WRITE_SIZE")
    copy = [k for k in f if "k_probe_copy" in k]
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
    with open(os.path.join(out_dir, json_name), "w") as fh:
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
    with open(os.path.join(out_dir, name), "w") as fh:
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


def counter_table(csv_paths, command, out_path, title):
    """Per-kernel means of any rocprofv3 --pmc counters (one or more
    counter_collection.csv files, e.g. one per pass) as a short text table."""
    import csv
    from collections import defaultdict

    agg = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(lambda: defaultdict(set))
    for path in csv_paths:
        for r in csv.DictReader(open(path)):
            k = kernel_key(r["Kernel_Name"])
            agg[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[k][r["Counter_Name"]].add(r["Dispatch_Id"])
    names = sorted({c for v in agg.values() for c in v})
    lines = [title, "command: " + command, "source hash: " + src_hash(),
             "values: mean per dispatch", "",
             "%-28s " % "kernel" + " ".join("%16s" % c[:16] for c in names)]
    order = sorted(agg, key=lambda k: -max(agg[k].values()))
    for k in order[:16]:
        vals = []
        for c in names:
            n = len(disp[k][c])
            vals.append("%16.4g" % (agg[k][c] / n) if n else "%16s" % "-")
        lines.append("%-28s " % k[:28] + " ".join(vals))
    ratios = [("LDS bank-conflict cycles / LDS active cycles", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE"),
              ("wave cycles waiting on anything / wave cycles", "SQ_WAIT_ANY", "SQ_WAVE_CYCLES")]
    for label, a, b in ratios:
        if a in names and b in names:
            lines += ["", label]
            for k in order[:16]:
                if agg[k][b] > 0:
                    lines.append("  %-28s %6.3f" % (k[:28], agg[k][a] / agg[k][b]))
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
    ap.add_argument("--counter-table", nargs="+", metavar="COUNTER_CSV",
                    help="summarise rocprofv3 --pmc runs (any counters) into profiles/ (no GPU needed)")
    ap.add_argument("--profile-command", default="", help="command recorded in the summaries")
    ap.add_argument("--profile-name", default="")
    ap.add_argument("--traffic-json", default="traffic.json", help="--pmc-summary: name of the JSON written")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-log2", type=int, default=28)
    ap.add_argument("--workload", default="plain", choices=["plain", "latency", "batched", "small", "serving",
                                                             "rquick_mw"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--key-type", default="u64", choices=["u64", "u32", "f32"], help="plain workload key type")
    ap.add_argument("--batched-variant", default="1gib", choices=["1gib", "literal"])
    ap.add_argument("--small-n", type=int, default=0, help="small workload: only this array size")
    ap.add_argument("--small-algo", default="", choices=["", "rfis", "rquick", "merge"],
                    help="small workload: only this algorithm")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--serve-slots", type=int, default=8,
                    help="server slots, one stream each (the process has 4 hardware queues by default; more slots "
                         "than queues keep each queue fed when a request ends)")
    ap.add_argument("--no-extras", action="store_true",
                    help="plain workload only: skip the ceilings and the other configurations")
    ap.add_argument("--serve-warmup", type=int, default=200)
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.calib_copy_mib or 1024, args.profile_command,
                    os.path.join(ROOT, "profiles"), args.profile_name or "hbm_traffic_plain_2p28_u64.txt",
                    args.traffic_json)
        return
    if args.counter_table:
        counter_table(args.counter_table, args.profile_command,
                      os.path.join(ROOT, "profiles", args.profile_name or "sq_counters_plain_2p28_u64.txt"),
                      "rocprofv3 --pmc counter summary")
        return
    if args.trace_summary:
        trace_summary(args.trace_summary, args.profile_command,
                      os.path.join(ROOT, "profiles", args.profile_name or "kernel_trace_plain_2p28_u64.txt"),
                      "rocprofv3 --kernel-trace --stats summary")
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the sort is built and measured on a single GPU and its "
              "sharding over several GPUs is described, not implemented; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1606_08766_amd import rsort as R

    if args.workload == "plain":
        out = bench_plain(args, R, torch)
    elif args.workload == "latency":
        out = bench_latency(args, R, torch)
    elif args.workload == "batched":
        out = bench_batched(args, R, torch)
    elif args.workload == "small":
        out = bench_small(args, R, torch)
    elif args.workload == "rquick_mw":
        out = bench_rquick_mw(args, R, torch)
    else:
        out = bench_serving(args, R, torch)
    if args.workload == "plain" and not args.no_extras:
        torch.cuda.empty_cache()
        out["ceilings"] = bandwidth_ceilings(R, torch)
        cp = out["ceilings"]["copy"]["GB_s"]
        rd = out["ceilings"]["read"]["GB_s"]
        for c, e in out["passes"].items():
            if "GB_s" in e:
                e["frac_of_ceiling"] = round(e["GB_s"] / (rd if c.startswith("count") else cp), 4)
        out.update(run_extras(args, R, torch))
    if (args.workload == "plain" and args.key_type == "u64" and not args.no_cpu_baseline
            and int(os.environ.get("RANK", "0")) == 0):
        out["cpu_baseline"] = cpu_baseline(args.n_log2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
