"""Parity of rsort_segmented (size-class dispatch: RFIS, RQuick, LDS merge
sort, sample-sort levels) against the oracle's per-segment sort."""
import functools

import numpy as np
import pytest

from gen import gen
from oracle import oracle as O
from paper_1606_08766_amd import rsort as R
from tests.gpu_util import banner, dev, gpu_segmented, host, same_bits

pytestmark = pytest.mark.gpu

ALGOS = {
    "default": dict(rfis_max=1024, rquick_max=4096),
    "merge_only": dict(rfis_max=1, rquick_max=1),
    "rquick_wide": dict(rfis_max=64, rquick_max=4096),
}

# Small-input regime at its own size: 2^14 independent arrays per call, so
# every class kernel's workgroup sorts many arrays in turn (its grid is capped
# at a few workgroups per CU) and LDS is reused from array to array.
CONFIG3_ALGOS = {
    "rfis": dict(rfis_max=1024, rquick_max=1),      # RFIS for n <= 1024
    "rquick": dict(rfis_max=1, rquick_max=4096),    # RQuick for every class up to 4096
    "words": dict(rfis_max=1, rquick_max=1),        # the LDS word sort everywhere
    "production": {},                               # the library's default routing
}


def check_against_oracle(keys, off, payload=None):
    ko, po, plo, _ = gpu_segmented(keys, off, payload)
    ek, ep, epl = O.segmented(keys, off, payload)
    assert same_bits(ko, ek)
    assert np.array_equal(po, ep)
    if payload is not None:
        assert np.array_equal(plo, epl)


@functools.lru_cache(maxsize=1)
def _config3_case(n, dist):
    """2^14 arrays of n u32 keys (uniform, or 8 distinct values) and the
    oracle's per-array sort of them, computed once per (n, dist)."""
    count = 1 << 14
    if dist == "uniform":
        keys = gen.keys("u32", "uniform", count * n, seed=1)
    else:
        keys = gen.keys("u32", "topbits", count * n, seed=1, param=3)
    off = np.arange(0, count * n + 1, n, dtype=np.uint64)
    ek, ep, _ = O.segmented(keys, off)
    return keys, off, ek, ep


@pytest.mark.parametrize("algo", list(CONFIG3_ALGOS))
@pytest.mark.parametrize("dist", ["uniform", "dup8"])
@pytest.mark.parametrize("n", [64, 256, 1024, 4096])
def test_config3_small_arrays(algo, dist, n):
    """Config 3 at full size: 2^14 independent arrays of n u32 keys (uniform or
    8 distinct values), each class routed to RFIS (Section 5, Appendix F),
    RQuick (Section 6, Algorithm 2) or the word sort; bit-exact against the
    oracle's per-array sort."""
    keys, off, ek, ep = _config3_case(n, dist)
    with R.tuned(**CONFIG3_ALGOS[algo]):
        ko, po, _, _ = gpu_segmented(keys, off)
    assert same_bits(ko, ek)
    assert np.array_equal(po, ep)


RAGGED = [0, 1, 2, 3, 0, 63, 64, 65, 100, 255, 256, 257, 1000, 1024, 1025, 2048, 2049, 3000, 4096, 4097, 8192,
          8193, 12288, 12289, 20000, 70000, 0, 300001, 5, 1]


@pytest.mark.parametrize("algo", list(ALGOS))
@pytest.mark.parametrize("kt", ["u64", "u32", "f32"])
@pytest.mark.parametrize("with_payload", [False, True])
def test_ragged_segments(algo, kt, with_payload):
    sizes = np.array(RAGGED, dtype=np.uint64)
    dists = gen.pick_dists(sizes.size, ["uniform", "zero", "deterdupl", "reverse", "gaussian"], seed=5)
    keys, pay, off = gen.segmented(kt, sizes, dists, seed=11, with_payload=with_payload)
    with R.tuned(**ALGOS[algo]):
        check_against_oracle(keys, off, pay)


def test_config4_reduced_mix():
    """Log-uniform sizes in [1, 2^18], Uniform / Zero / DeterDupl per segment,
    u64 keys with a random u32 payload."""
    count = 3000
    sizes = gen.log_uniform_sizes(count, 0, 18, seed=1)
    dists = gen.pick_dists(count, ["uniform", "zero", "deterdupl"], seed=2)
    keys, pay, off = gen.segmented("u64", sizes, dists, seed=3)
    check_against_oracle(keys, off, pay)


def test_config4_one_gib_variant():
    """100k segments, log-uniform [1, 2^13] (about 1 GiB of keys + payload + outputs)."""
    count = 100_000
    sizes = gen.log_uniform_sizes(count, 0, 13, seed=1)
    dists = gen.pick_dists(count, ["uniform", "zero", "deterdupl"], seed=2)
    keys, pay, off = gen.segmented("u64", sizes, dists, seed=3)
    check_against_oracle(keys, off, pay)


def test_config4_literal_100k_segments_up_to_2p18():
    """Config 4 as stated: 100k segments of log-uniform sizes in [1, 2^18]
    (2.11e9 keys, about 17 GiB of u64 keys) with a random u32 payload,
    Uniform / Zero / DeterDupl per segment, in one segmented call.  Too large
    for the oracle as a whole: every segment is checked on the device for the
    characterising properties (bijection onto its own positions, gather of
    keys and payload, strictly increasing (key, position)), and 24 sampled
    segments, including the largest, are compared element by element with
    the oracle's sort of that segment alone."""
    import torch

    from tests.checks import check_sorted_segmented_device

    count = 100_000
    sizes = gen.log_uniform_sizes(count, 0, 18, seed=1)
    dists = gen.pick_dists(count, ["uniform", "zero", "deterdupl"], seed=2)
    keys, pay, off = gen.segmented("u64", sizes, dists, seed=3)
    n = keys.size
    banner("config 4 literal: %d segments, %d keys, with payload" % (count, n))
    dk, dp = dev(keys), dev(pay)
    ws = torch.empty(R.segmented_workspace_bytes(R.U64, n, count, True), dtype=torch.uint8, device="cuda")
    ko, po, plo = R.segmented_sort(dk, dev(off.astype(np.uint64)), dp, workspace=ws)
    assert R.workspace_status(ws) == R.OK
    del ws
    torch.cuda.synchronize()
    check_sorted_segmented_device(dk, off, ko, po, dp, plo)
    rng = np.random.default_rng(17)
    pick = set(rng.choice(count, 23, replace=False).tolist()) | {int(np.argmax(sizes))}
    for s in sorted(pick):
        a, b = int(off[s]), int(off[s + 1])
        ek, ep, epl = O.sort(keys[a:b], pay[a:b])
        assert np.array_equal(host(ko[a:b]), ek), s
        assert np.array_equal(host(po[a:b]), ep), s
        assert np.array_equal(host(plo[a:b]), epl), s


def test_single_big_segment_with_payload():
    keys, pay, off = gen.segmented("u64", np.array([3_000_000], np.uint64), ["gaussian"], seed=4)
    check_against_oracle(keys, off, pay)


@pytest.mark.parametrize("dist", ["deterdupl", "zero"])
def test_one_split_segment_of_tied_keys_among_small_ones(dist):
    """A keys-only call whose one segment above the LDS capacity (4M keys of
    few distinct values, starting at an offset that is not a multiple of
    anything) is split over two levels: its first level stores bucket ids at
    the segment's own place in the id buffer.  Every segment equals the
    oracle's."""
    sizes = np.array([5, 700, 4_000_003, 64, 3000, 0, 1], np.uint64)
    keys, _, off = gen.segmented("u64", sizes, ["uniform", "gaussian", dist, "uniform", "zero", "uniform", "reverse"],
                                 seed=12)
    check_against_oracle(keys, off)


def test_all_empty_and_one_element():
    keys = np.array([7], dtype=np.uint64)
    off = np.array([0, 0, 0, 1, 1], dtype=np.uint64)
    check_against_oracle(keys, off)


def test_decreasing_offsets_reported():
    keys = gen.keys("u64", "uniform", 100, seed=1)
    off = np.array([0, 60, 40, 100], dtype=np.uint64)
    _, _, _, st = gpu_segmented(keys, off, check_status=False)
    assert st == R.EINVAL


@pytest.mark.parametrize("kt", ["u64", "u32"])
def test_forced_fallback_path(kt):
    """Every final bucket above 64 elements takes the global-memory fallback."""
    sizes = np.array([100, 5000, 50000, 1 << 20, 7], dtype=np.uint64)
    keys, pay, off = gen.segmented(kt, sizes, ["uniform", "zero", "deterdupl", "uniform", "uniform"], seed=8)
    with R.tuned(force_fallback=1):
        check_against_oracle(keys, off, pay)


@pytest.mark.parametrize("kt", ["u64", "u32"])
@pytest.mark.parametrize("with_payload", [False, True])
def test_clustered_segments_take_the_merge_path(kt, with_payload):
    """Segments whose keys form two clusters far apart: the bins by the top
    key bits put about half of each segment into one bin, so the ranking cost
    exceeds its budget and the merge instance after the classes sorts them.
    Mixed with a segment large enough for sample-sort levels, so that both
    the input-segment and the buffer-segment instances run."""
    rng = np.random.default_rng(21)
    dt = np.uint64 if kt == "u64" else np.uint32
    hi = dt(1) << dt(60 if kt == "u64" else 28)
    sizes = [1500, 3000, 5000, 8000, 100000, 2500]
    parts = []
    for n in sizes:
        a = rng.integers(0, 1000, n).astype(dt)
        a[rng.random(n) < 0.5] += hi
        parts.append(a)
    keys = np.concatenate(parts)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    pay = rng.integers(0, 1 << 32, keys.size, dtype=np.uint64).astype(np.uint32) if with_payload else None
    check_against_oracle(keys, off, pay)
