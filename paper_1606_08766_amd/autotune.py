"""Autotuner for librsort: per-size-class algorithm choice and tile shapes.

The paper's family has several algorithms that are each fastest for a range
of input sizes (Section 4, Section 7.1); on one GPU the same holds for the
final buckets of a sort and for the segments of a batched sort.  This module
times the candidates on the current GPU and sets the library's tuning:

* per final-size class, RFIS, RQuick or the LDS merge sort, timed on many
  equal segments that fall in that class; the choice is expressed through
  the two thresholds the library understands (classes with upper bound
  <= rfis_max use RFIS, classes <= rquick_max use RQuick, larger ones the
  merge sort), picked to minimise the summed per-key time over the classes;
* per final-size class from 1024 to 4096 keys, the word sort's workgroup
  shape (the default, or twice the threads with half the keys per thread),
  expressed as the class_shape bit mask;
* tile size, oversampling, target bucket size and the number of sample-sort
  levels (the fewest that reach the target, or one more) of a plain sort.

Results are plain JSON (``save``/``load``); ``apply`` installs them with
``rsort_set_tuning``.  Tuning changes speed only: every setting produces the
same output.
"""
from __future__ import annotations

import argparse
import itertools
import json

# upper bounds of the final-size classes (the last, oversize class is never
# tuned) and the algorithms each class can use
CLASS_BOUNDS = (64, 256, 1024, 2048, 3072, 4096, 6144, 8192, 12288)
RFIS_BOUNDS = (64, 256, 1024)
RQUICK_BOUNDS = (2048, 3072, 4096)
ALGOS = ("rfis", "rquick", "merge")
ALT_SHAPE_BOUNDS = (1024, 2048, 3072, 4096)  # classes with an alternative word-sort shape
SHAPE_ON = 0x80000000  # class_shape is taken only with bit 31 set


def algo_for(bound: int, rfis_max: int, rquick_max: int) -> str:
    """The algorithm the library runs for the class with this upper bound
    (a class an algorithm has no kernel for takes the merge sort)."""
    if bound <= rfis_max and bound in RFIS_BOUNDS:
        return "rfis"
    if bound <= rquick_max and bound in RQUICK_BOUNDS:
        return "rquick"
    return "merge"


def choose_thresholds(ns_per_key: dict) -> tuple[int, int, float]:
    """Given measured times ns_per_key[(bound, algo)], return the (rfis_max,
    rquick_max) pair expressible by the library that minimises the summed
    time over the measured classes, and that sum.  A threshold of 1 turns
    an algorithm off."""
    bounds = sorted({b for b, _ in ns_per_key})
    best = None
    for rf in (1,) + RFIS_BOUNDS:
        for rq in (1,) + RQUICK_BOUNDS:
            if rq != 1 and rq <= rf:
                continue
            total = 0.0
            for b in bounds:
                a = algo_for(b, rf, rq)
                t = ns_per_key.get((b, a))
                if t is None:
                    total = float("inf")
                    break
                total += t
            if best is None or total < best[2]:
                best = (rf, rq, total)
    return best


def _time_ms(torch, fn, iters: int) -> float:
    fn()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(iters):
        fn()
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / iters


def tune(kt: str = "u64", quick: bool = False, seg_keys: int = 1 << 22, n_plain: int = 1 << 26,
         iters: int = 3, apply_result: bool = True) -> dict:
    """Measure on the current GPU and return (and by default apply) a tuning."""
    import torch

    from gen import gen
    from paper_1606_08766_amd import rsort as R

    ktc = {"u32": R.U32, "u64": R.U64, "f32": R.F32}[kt]
    base = R.get_tuning()
    keep = {f: getattr(base, f) for f, _ in R.Tuning._fields_}
    if quick:
        seg_keys, n_plain, iters = 1 << 18, 1 << 22, 1
    times = {}
    try:
        # --- per-class algorithm choice on equal segments of each class
        for bound in CLASS_BOUNDS:
            size = max(2, bound - bound // 8)  # inside (previous bound, bound]
            count = max(16, seg_keys // size)
            keys = gen.keys(kt, "uniform", size * count, seed=bound)
            offs = torch.arange(0, size * count + 1, size, dtype=torch.int64).cuda()
            dk = torch.from_numpy(keys).cuda()
            ws = torch.empty(R.segmented_workspace_bytes(ktc, dk.numel(), count, False), dtype=torch.uint8,
                             device="cuda")
            out = (torch.empty_like(dk), torch.empty(dk.numel(), dtype=torch.uint32, device="cuda"), None)
            for algo in ALGOS + ("merge_alt",):
                if algo == "rfis" and bound not in RFIS_BOUNDS:
                    continue
                if algo == "rquick" and bound not in RQUICK_BOUNDS:
                    continue
                if algo == "merge_alt" and bound not in ALT_SHAPE_BOUNDS:
                    continue
                rf = bound if algo == "rfis" else 1
                rq = bound if algo == "rquick" else 1
                cs = SHAPE_ON | ((1 << CLASS_BOUNDS.index(bound)) if algo == "merge_alt" else 0)
                R.set_tuning(**dict(keep, rfis_max=rf, rquick_max=rq, class_shape=cs))
                ms = _time_ms(torch, lambda: R.segmented_sort(dk, offs, workspace=ws, out=out), iters)
                times[(bound, algo)] = ms * 1e6 / dk.numel()
            del dk, ws, out
        # the word sort of a class takes its faster shape
        shape = 0
        for b in ALT_SHAPE_BOUNDS:
            if times.get((b, "merge_alt"), float("inf")) < times.get((b, "merge"), float("inf")):
                shape |= 1 << CLASS_BOUNDS.index(b)
                times[(b, "merge")] = times[(b, "merge_alt")]
        rf, rq, _ = choose_thresholds({k: v for k, v in times.items() if k[1] != "merge_alt"})
        # --- sample-sort levels on a plain sort
        x = torch.from_numpy(gen.keys(kt, "uniform", n_plain, seed=7)).cuda()
        ws = torch.empty(R.plain_workspace_bytes(ktc, n_plain), dtype=torch.uint8, device="cuda")
        out = (torch.empty_like(x), torch.empty(n_plain, dtype=torch.uint32, device="cuda"))
        grid = list(itertools.product((12, 13), (16, 32), (4096, 5120, 6144), (0, 1)))
        if quick:
            grid = grid[:3]
        level = {}
        for tl, a, tg, ex in grid:
            R.set_tuning(**dict(keep, rfis_max=rf, rquick_max=rq, tile_log2=tl, oversample=a, target=tg,
                                extra_levels=ex + 1, class_shape=SHAPE_ON | shape))
            wsb = R.plain_workspace_bytes(ktc, n_plain)
            if wsb > ws.numel():
                ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
            level[(tl, a, tg, ex)] = _time_ms(torch, lambda: R.sort(x, workspace=ws, out=out), iters)
        tl, a, tg, ex = min(level, key=level.get)
    finally:
        R.set_tuning(**keep)
    result = {
        "key_type": kt,
        "rfis_max": rf, "rquick_max": rq, "tile_log2": tl, "oversample": a, "target": tg,
        "extra_levels": ex, "class_shape": shape,
        "class_ns_per_key": {"%d/%s" % k: round(v, 4) for k, v in sorted(times.items())},
        "plain_ms": {"%d/%d/%d/%d" % k: round(v, 4) for k, v in sorted(level.items())},
        "n_plain": n_plain,
    }
    if apply_result:
        apply(result)
    return result


def apply(result: dict) -> None:
    """Install a tuning produced by tune() (fields not present are kept)."""
    from paper_1606_08766_amd import rsort as R

    cur = R.get_tuning()
    fields = {f: getattr(cur, f) for f, _ in R.Tuning._fields_}
    for f in ("rfis_max", "rquick_max", "tile_log2", "oversample", "target"):
        if f in result:
            fields[f] = int(result[f])
    if "extra_levels" in result:
        fields["extra_levels"] = int(result["extra_levels"]) + 1
    if "class_shape" in result:
        fields["class_shape"] = SHAPE_ON | int(result["class_shape"])
    R.set_tuning(**fields)


def save(result: dict, path: str) -> None:
    with open(path, "w") as fh:
        json.dump(result, fh, indent=1, sort_keys=True)


def load(path: str, apply_result: bool = True) -> dict:
    with open(path) as fh:
        result = json.load(fh)
    if apply_result:
        apply(result)
    return result


def main() -> None:
    ap = argparse.ArgumentParser(description="time librsort's candidates on this GPU and write a tuning file")
    ap.add_argument("--out", required=True)
    ap.add_argument("--key-type", default="u64", choices=("u32", "u64", "f32"))
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    res = tune(args.key_type, quick=args.quick, apply_result=False)
    save(res, args.out)
    print(json.dumps({k: res[k] for k in ("rfis_max", "rquick_max", "tile_log2", "oversample", "target",
                                          "extra_levels", "class_shape")}))


if __name__ == "__main__":
    main()
