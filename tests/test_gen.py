"""Generator checks: published SplitMix64 values, determinism, distribution facts."""
import numpy as np

from gen import gen


def test_splitmix64_published_sequence():
    # first outputs of SplitMix64 seeded with 0
    assert gen.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert gen.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert gen.splitmix64(0, 2) == 0x06C45D188009454F


def test_determinism_and_stream_offset():
    a = gen.keys("u64", "uniform", 1000, seed=1)
    b = gen.keys("u64", "uniform", 1000, seed=1)
    assert np.array_equal(a, b)
    c = gen.keys("u64", "uniform", 500, seed=1, stream_off=500)
    assert np.array_equal(a[500:], c)
    u = gen.keys("u32", "uniform", 1000, seed=1)
    assert np.array_equal(u, (a & np.uint64(0xFFFFFFFF)).astype(np.uint32))


def test_distribution_facts():
    n = 1 << 16
    assert (gen.keys("u64", "zero", n) == 0).all()
    assert np.array_equal(gen.keys("u64", "reverse", n), np.arange(n - 1, -1, -1, dtype=np.uint64))
    d = gen.keys("u64", "deterdupl", n)
    assert np.array_equal(np.bincount(d.astype(np.int64)), np.full(16, n // 16))
    t = gen.keys("u32", "topbits", n, param=3)
    assert t.max() == 7 and np.bincount(t).min() > n // 8 * 0.9
    g = gen.keys("u64", "gaussian", 1 << 18).astype(np.float64) - 2.0 ** 63
    z = g / 2.0 ** 40
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01
    wd = gen.keys("u64", "widedup", n, seed=4)
    assert np.unique(wd).size == 300 and wd.max() > 1 << 62 and wd.min() < 1 << 58


def test_log_uniform_sizes():
    s = gen.log_uniform_sizes(100000, 0, 18, seed=1)
    assert s.min() >= 1 and s.max() <= 1 << 18
    med = np.median(s.astype(np.float64))
    assert 400 < med < 650  # log-uniform on [1, 2^18]: median 2^9


def test_segmented_layout():
    sizes = np.array([3, 0, 5], dtype=np.uint64)
    k, p, off = gen.segmented("u32", sizes, ["uniform", "zero", "deterdupl"])
    assert list(off) == [0, 3, 3, 8]
    assert list(k[3:8]) == [0, 1, 2, 3, 4]
