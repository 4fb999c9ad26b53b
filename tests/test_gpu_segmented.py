"""Parity of rsort_segmented (size-class dispatch: RFIS, RQuick, LDS merge
sort, sample-sort levels) against the oracle's per-segment sort."""
import numpy as np
import pytest

from gen import gen
from oracle import oracle as O
from paper_1606_08766_amd import rsort as R
from tests.gpu_util import gpu_segmented, same_bits

pytestmark = pytest.mark.gpu

ALGOS = {
    "default": dict(rfis_max=1024, rquick_max=4096),
    "merge_only": dict(rfis_max=1, rquick_max=1),
    "rquick_wide": dict(rfis_max=64, rquick_max=4096),
}


def check_against_oracle(keys, off, payload=None):
    ko, po, plo, _ = gpu_segmented(keys, off, payload)
    ek, ep, epl = O.segmented(keys, off, payload)
    assert same_bits(ko, ek)
    assert np.array_equal(po, ep)
    if payload is not None:
        assert np.array_equal(plo, epl)


@pytest.mark.parametrize("algo", list(ALGOS))
@pytest.mark.parametrize("n", [64, 256, 1024, 4096])
@pytest.mark.parametrize("dist", ["uniform", "dup8"])
def test_config3_small_arrays(algo, n, dist):
    """Many independent arrays of equal size n, u32 keys (uniform or 8 distinct values)."""
    count = 512
    if dist == "uniform":
        keys = gen.keys("u32", "uniform", count * n, seed=1)
    else:
        keys = gen.keys("u32", "topbits", count * n, seed=1, param=3)
    off = np.arange(0, count * n + 1, n, dtype=np.uint64)
    with R.tuned(**ALGOS[algo]):
        check_against_oracle(keys, off)


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


def test_single_big_segment_with_payload():
    keys, pay, off = gen.segmented("u64", np.array([3_000_000], np.uint64), ["gaussian"], seed=4)
    check_against_oracle(keys, off, pay)


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
