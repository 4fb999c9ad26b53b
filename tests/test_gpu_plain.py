"""Parity of rsort_plain (multilevel sample sort) against the CPU oracle.

Element-by-element bit equality with the oracle at sizes spanning several
tiles, every level count and the ragged tails; at the full 2^28-key
workload the closed forms (Zero, Reverse, DeterDupl), the characterising
invariants and ranks recomputed one by one from the definition."""
import numpy as np
import pytest
import torch

from gen import gen
from oracle import oracle as O
from paper_1606_08766_amd import rsort as R
from tests.checks import check_sorted, closed_form
from tests.gpu_util import banner, dev, gpu_sort, host, same_bits

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 63, 64, 65, 255, 256, 257, 1000, 1023, 1024, 1025, 2047, 2049, 4095, 4096, 4097, 8191, 8193,
         12287, 12288, 12289, 12290, 40000, 65539, 300007, (1 << 20) + 7]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kt,dist", [("u64", "uniform"), ("u32", "uniform"), ("f32", "uniform"),
                                     ("u64", "deterdupl"), ("u64", "zero"), ("u32", "topbits"),
                                     ("f32", "gaussian"), ("u64", "reverse")])
def test_plain_parity(n, kt, dist):
    x = gen.keys(kt, dist, n, seed=n + 3, param=3 if dist == "topbits" else 0)
    ko, po = gpu_sort(x)
    ek, ep, _ = O.sort(x)
    assert same_bits(ko, ek)
    assert np.array_equal(po, ep)


@pytest.mark.parametrize("n", [5000, 12289, 300007, (1 << 20) + 7, 1 << 22])
@pytest.mark.parametrize("kt", ["u64", "u32"])
def test_plain_wide_range_duplicates(n, kt):
    """Few distinct keys spread over the whole key range: final buckets hold
    runs of equal keys whose key range is too wide for exact single-word
    compares, so the order among equal keys must come from their positions."""
    x = gen.keys(kt, "widedup", n, seed=n + 11, param=300 if n > 5000 else 40)
    ko, po = gpu_sort(x)
    ek, ep, _ = O.sort(x)
    assert same_bits(ko, ek)
    assert np.array_equal(po, ep)


@pytest.mark.parametrize("kt", ["u64", "u32"])
@pytest.mark.parametrize("block_log2", [12, 15])
def test_plain_tied_and_untied_blocks(kt, block_log2):
    """Blocks of 2^block_log2 equal keys alternate with blocks of random keys,
    so the waves of the count and scatter passes move in and out of the
    classification mode that skips the key-only descent after a tile in which
    every key tied a splitter key.  Both modes compute the same bucket; the
    output equals the oracle's."""
    n = (1 << 24) + 11
    x = gen.keys(kt, "uniform", n, seed=21 + block_log2)
    blocks = (np.arange(n) >> block_log2) & 1
    x[blocks == 1] = x.dtype.type(12345)
    ko, po = gpu_sort(x)
    ek, ep, _ = O.sort(x, threads=8)
    assert same_bits(ko, ek) and np.array_equal(po, ep)


def test_plain_keys_only_and_empty():
    x = gen.keys("u64", "uniform", 100000, seed=5)
    ko, po = gpu_sort(x, with_perm=False)
    assert po is None
    assert same_bits(ko, O.sort(x)[0])
    banner("empty plain sort")
    k0, p0 = R.sort(torch.empty(0, dtype=torch.uint64, device="cuda"))
    assert k0.numel() == 0 and p0.numel() == 0


def test_config1_uniform_2p20_seed1():
    """2^20 uniform u64 keys from seed 1 (a single sample-sort level)."""
    n = 1 << 20
    x = gen.keys("u64", "uniform", n, seed=1)
    ko, po = gpu_sort(x)
    ek, ep, _ = O.sort(x)
    assert same_bits(ko, ek) and np.array_equal(po, ep)


def test_f32_specials():
    specials = np.array([0xFFC00000, 0xFF800000, 0xBF800000, 0x80000000, 0x00000000, 0x3F800000, 0x7F800000,
                         0x7FC00000, 0x7FC00001, 0xFFC00001, 0x00000001, 0x80000001], dtype=np.uint32)
    rng = np.random.default_rng(0)
    for n in (12, 5000, 50000):
        x = specials[rng.integers(0, specials.size, n)].view(np.float32)
        ko, po = gpu_sort(x)
        ek, ep, _ = O.sort(x)
        assert same_bits(ko, ek) and np.array_equal(po, ep)


@pytest.mark.parametrize("dist", ["uniform", "gaussian", "zero", "deterdupl", "reverse"])
def test_config2_full_size(dist):
    """2^28 u64 keys, two sample-sort levels: closed forms or the
    characterising invariants, plus ranks of sampled outputs computed by the
    oracle one by one."""
    n = 1 << 28
    x = gen.keys("u64", dist, n, seed=1)
    ko, po = gpu_sort(x)
    if dist in ("zero", "deterdupl", "reverse"):
        ek, ep = closed_form(dist, n)
        assert np.array_equal(ko, ek) and np.array_equal(po, ep)
    else:
        check_sorted(x, ko, po)
    rng = np.random.default_rng(7)
    for r in rng.integers(0, n, 3):
        assert O.rank(x, int(po[r])) == int(r)


@pytest.mark.parametrize("kt,dist", [("u32", "uniform"), ("u32", "gaussian"), ("f32", "uniform"), ("f32", "gaussian")])
def test_full_size_32bit_keys(kt, dist):
    """2^28 u32 and f32 keys (f32 uniform: random bit patterns with NaNs,
    infinities and signed zeros), two sample-sort levels: the characterising
    invariants plus ranks of sampled outputs computed by the oracle."""
    n = 1 << 28
    x = gen.keys(kt, dist, n, seed=3)
    ko, po = gpu_sort(x)
    check_sorted(x, ko, po)
    rng = np.random.default_rng(11)
    for r in rng.integers(0, n, 3):
        assert O.rank(x, int(po[r])) == int(r)


@pytest.mark.parametrize("kt,dist", [("u32", "deterdupl"), ("u32", "zero"), ("f32", "deterdupl")])
def test_full_size_32bit_tied_keys(kt, dist):
    """2^28 32-bit keys of 16 distinct values or all equal: the first level's
    splitters repeat keys, so its count stores bucket ids for the scatter.
    The output equals the closed form."""
    n = 1 << 28
    x = gen.keys(kt, dist, n, seed=3)
    ko, po = gpu_sort(x)
    ek, ep = closed_form(dist, n, dtype=np.float32 if kt == "f32" else np.uint32)
    assert np.array_equal(ko, ek) and np.array_equal(po, ep)


def test_repeat_calls_identical():
    x = gen.keys("u64", "gaussian", 3_000_000, seed=9)
    a = gpu_sort(x)
    b = gpu_sort(x)
    assert same_bits(a[0], b[0]) and np.array_equal(a[1], b[1])
