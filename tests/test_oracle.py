"""Pins for the CPU oracle, independent of the oracle's own code.

  P1  closed forms (Zero, Reverse, DeterDupl, sorted inputs)
  P2  the three characterising invariants (tests/checks.py)
  P3  brute force: a separate O(n^2) rank formula over exhaustive tiny inputs
  P4  numpy's stable argsort on the special cases where it applies
  P5  the paper's RFIS compare-decision table (Appendix F) equals lexicographic
      (key, row, column, position) order
  plus: f32 totalOrder special values, segmented = per-segment, classification
  against brute force and numpy searchsorted, and the binary-tree median's
  closed forms (Section 3.2).
"""
import itertools
import os
import struct

import numpy as np
import pytest

from gen import gen
from oracle import oracle as O
from tests.checks import check_sorted, closed_form


def brute_rank_sort(vals):
    """rank(i) = #{j : v_j < v_i} + #{j < i : v_j == v_i}; out[rank(i)] = i."""
    n = len(vals)
    perm = [None] * n
    for i in range(n):
        r = sum(1 for j in range(n) if vals[j] < vals[i]) + sum(1 for j in range(i) if vals[j] == vals[i])
        perm[r] = i
    return perm


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("dist", ["zero", "reverse", "deterdupl", "sorted"])
@pytest.mark.parametrize("n", [1, 2, 17, 1000, 1 << 16, (1 << 20) + 5])
def test_p1_closed_forms(dist, n):
    x = gen.keys("u64", dist, n)
    ko, po, _ = O.sort(x)
    ek, ep = closed_form(dist, n)
    assert np.array_equal(ko, ek)
    assert np.array_equal(po, ep)


@pytest.mark.parametrize("dist", ["zero", "reverse", "deterdupl"])
def test_p1_closed_forms_u32_mt(dist):
    n = (1 << 18) + 3
    x = gen.keys("u32", dist, n)
    ko, po, _ = O.sort(x, threads=4)
    ek, ep = closed_form(dist, n, dtype=np.uint32)
    assert np.array_equal(ko, ek) and np.array_equal(po, ep)


# ---------------------------------------------------------------- P2
@pytest.mark.parametrize("kt,dist", [("u64", "uniform"), ("u64", "gaussian"), ("u32", "uniform"),
                                     ("u32", "topbits"), ("f32", "uniform"), ("f32", "gaussian")])
def test_p2_invariants(kt, dist):
    n = (1 << 17) + 11
    x = gen.keys(kt, dist, n, seed=5)
    pl = gen.payload(n, seed=9)
    ko, po, plo = O.sort(x, pl)
    check_sorted(x, ko, po, pl, plo)
    ko2, po2, plo2 = O.sort(x, pl, threads=3)
    assert np.array_equal(ko.view(np.uint8), ko2.view(np.uint8))
    assert np.array_equal(po, po2) and np.array_equal(plo, plo2)


def test_p2_catches_planted_errors():
    """The characterising checks reject outputs with typical mistakes."""
    x = gen.keys("u64", "deterdupl", 4096)
    ko, po, _ = O.sort(x)
    bad = po.copy()
    bad[[10, 11]] = bad[[11, 10]]            # equal keys, positions swapped
    with pytest.raises(AssertionError):
        check_sorted(x, ko, bad)
    bad = po.copy()
    bad[5] = bad[6]                            # not a bijection
    with pytest.raises(AssertionError):
        check_sorted(x, ko, bad)
    kbad = ko.copy()
    kbad[100] ^= np.uint64(1)                  # key bits changed
    with pytest.raises(AssertionError):
        check_sorted(x, kbad, po)


# ---------------------------------------------------------------- P3
@pytest.mark.parametrize("n", range(0, 8))
def test_p3_all_ternary_inputs(n):
    for t in itertools.product(range(3), repeat=n):
        x = np.array(t, dtype=np.uint32)
        ko, po, _ = O.sort(x)
        assert list(po) == brute_rank_sort(list(t))
        assert list(ko) == sorted(t)


@pytest.mark.parametrize("n", range(1, 8))
def test_p3_all_permutations(n):
    for t in itertools.permutations(range(n)):
        x = np.array(t, dtype=np.uint64)
        _, po, _ = O.sort(x)
        inv = [0] * n
        for i, v in enumerate(t):
            inv[v] = i
        assert list(po) == inv


F32_SPECIALS_IN_ORDER = [
    0xFFC00000,  # -NaN (quiet, sign set)
    0xFF800000,  # -inf
    0xBF800000,  # -1
    0x80000000,  # -0
    0x00000000,  # +0
    0x3F800000,  # +1
    0x7F800000,  # +inf
    0x7FC00000,  # +NaN
]


@pytest.mark.parametrize("n", range(1, 5))
def test_p3_f32_specials_exhaustive(n):
    # the class index of each special in totalOrder is its list position
    for t in itertools.product(range(8), repeat=n):
        x = np.array([F32_SPECIALS_IN_ORDER[c] for c in t], dtype=np.uint32).view(np.float32)
        ko, po, _ = O.sort(x)
        assert list(po) == brute_rank_sort(list(t))
        assert list(ko.view(np.uint32)) == [F32_SPECIALS_IN_ORDER[c] for c in sorted(t)]


def test_f32_total_order_matches_float_compare():
    """On non-NaN values totalOrder agrees with < except that -0 < +0."""
    rng = np.random.default_rng(3)
    bits = rng.integers(0, 2 ** 32, size=200000, dtype=np.uint64).astype(np.uint32)
    f = bits.view(np.float32)
    ok = ~np.isnan(f)
    bits, f = bits[ok], f[ok]
    ords = np.array([O.ord_f32(int(b)) for b in bits[:5000]], dtype=np.uint64)
    fs = f[:5000].astype(np.float64)
    a = np.argsort(ords, kind="stable")
    assert (np.diff(fs[a]) >= 0).all()
    assert O.ord_f32(0x80000000) < O.ord_f32(0)
    # NaN payload ordering: larger payload further from zero
    assert O.ord_f32(0x7FC00001) > O.ord_f32(0x7FC00000) > O.ord_f32(0x7F800000)
    assert O.ord_f32(0xFFC00001) < O.ord_f32(0xFFC00000) < O.ord_f32(0xFF800000)


def test_rank_matches_sort():
    x = gen.keys("u32", "topbits", 5000, param=4, seed=3)
    _, po, _ = O.sort(x)
    for r in (0, 1, 17, 2500, 4999):
        assert O.rank(x, int(po[r])) == r


# ---------------------------------------------------------------- P4
@pytest.mark.parametrize("kt,dist", [("u64", "uniform"), ("u64", "gaussian"), ("u32", "uniform"),
                                     ("u32", "topbits"), ("u64", "deterdupl")])
def test_p4_numpy_stable_argsort(kt, dist):
    n = 1 << 20
    x = gen.keys(kt, dist, n, seed=11)
    ko, po, _ = O.sort(x)
    ref = np.argsort(x, kind="stable")
    assert np.array_equal(po, ref.astype(np.uint32))
    assert np.array_equal(ko, x[ref])


def test_p4_numpy_f32_non_nan():
    n = 1 << 18
    x = gen.keys("f32", "gaussian", n, seed=4)
    _, po, _ = O.sort(x)
    assert np.array_equal(po, np.argsort(x, kind="stable").astype(np.uint32))


# ---------------------------------------------------------------- P5
LEFT, HERE, RIGHT = -1, 0, 1
UP, DOWN = -1, 1


def rfis_table_a_gt_b(x, colC, i, y, rowR, j):
    """Appendix F's compare table on PE (r, c): a = (x, r, C, i) from the row,
    b = (y, R, c, j) from the column; C in {left, here, right}, R in {up, here, down}."""
    if rowR == UP:
        return x >= y
    if rowR == DOWN:
        return x > y
    # b from this row (R = r)
    if colC == LEFT:
        return x > y
    if colC == RIGHT:
        return x >= y
    return i > j


def test_p5_rfis_table_is_lexicographic():
    r, c = 5, 5
    checked = 0
    for x, y in itertools.product(range(3), repeat=2):
        for colC in (LEFT, HERE, RIGHT):
            for rowR in (UP, HERE, DOWN):
                for i, j in itertools.product(range(3), repeat=2):
                    if colC == HERE and rowR == HERE:
                        # both local to PE (r, c): distinct slots of a sorted array
                        if i == j or (x < y and i > j) or (x > y and i < j):
                            continue
                    a = (x, r, c + colC, i)
                    b = (y, r + rowR, c, j)
                    assert rfis_table_a_gt_b(x, colC, i, y, rowR, j) == (a > b), (a, b)
                    checked += 1
    assert checked > 200


# ---------------------------------------------------------------- segmented
def test_segmented_equals_per_segment():
    sizes = np.array([0, 1, 5, 0, 64, 1000, 3, 4097, 0], dtype=np.uint64)
    dists = ["uniform", "zero", "deterdupl", "uniform", "reverse", "deterdupl", "zero", "gaussian", "zero"]
    k, p, off = gen.segmented("u64", sizes, dists, seed=3)
    ko, po, plo = O.segmented(k, off, p)
    for s in range(sizes.size):
        a, b = int(off[s]), int(off[s + 1])
        ref = np.argsort(k[a:b], kind="stable")
        assert np.array_equal(po[a:b], ref.astype(np.uint32))
        assert np.array_equal(ko[a:b], k[a:b][ref])
        assert np.array_equal(plo[a:b], p[a:b][ref])


# ---------------------------------------------------------------- classification
def test_classify_brute_force():
    rng = np.random.default_rng(1)
    keys = rng.integers(0, 4, size=300).astype(np.uint64)
    pos = rng.permutation(300).astype(np.uint32)
    sk = rng.integers(0, 4, size=7).astype(np.uint64)
    sp = rng.integers(0, 300, size=7).astype(np.uint32)
    b = O.classify(keys, pos, sk, sp)
    for i in range(300):
        e = (int(keys[i]), int(pos[i]))
        assert b[i] == sum(1 for s in zip(sk.tolist(), sp.tolist()) if s < e)


def test_classify_matches_searchsorted():
    n = 1 << 16
    keys = gen.keys("u32", "topbits", n, param=4, seed=2)
    comb = (keys.astype(np.uint64) << np.uint64(32)) | np.arange(n, dtype=np.uint64)
    spl = np.sort(np.random.default_rng(0).choice(comb, 255, replace=False))
    b = O.classify(keys, None, (spl >> np.uint64(32)).astype(np.uint32),
                   (spl & np.uint64(0xFFFFFFFF)).astype(np.uint32))
    assert np.array_equal(b, np.searchsorted(spl, comb, side="left").astype(np.uint32))


# ---------------------------------------------------------------- median tree (Section 3.2)
@pytest.mark.parametrize("log2_p", [0, 1, 3, 5])
def test_median_tree_exact_when_window_keeps_everything(log2_p):
    """If k covers the whole input and every leaf holds an even count, each window
    keeps all values padded symmetrically, so the root returns the exact lower or
    upper median."""
    p = 1 << log2_p
    rng = np.random.default_rng(log2_p)
    per = 4
    vals = rng.choice(1 << 40, size=p * per, replace=False).astype(np.uint64)
    off = np.arange(0, p * per + 1, per, dtype=np.uint64)
    k = p * per
    s = np.sort(vals)
    for root in (0, 1):
        coins = np.zeros(p + 1, dtype=np.uint8)
        coins[p] = root
        v, side = O.median_tree(vals, off, log2_p, k, coins)
        assert side == 0
        assert v == s[p * per // 2 - 1 + root]


def test_median_tree_single_leaf_small_window():
    vals = np.array([9, 1, 7, 3, 5, 11], dtype=np.uint64)
    off = np.array([0, 6], dtype=np.uint64)
    assert O.median_tree(vals, off, 0, 2, np.array([0, 0], np.uint8)) == (5, 0)
    assert O.median_tree(vals, off, 0, 2, np.array([0, 1], np.uint8)) == (7, 0)


def test_median_tree_sentinels_and_odd_leaves():
    # two leaves of one element each, k = 2: leaf coins pick (-inf, v) or (v, +inf)
    vals = np.array([10, 20], dtype=np.uint64)
    off = np.array([0, 1, 2], dtype=np.uint64)
    # both leaves forward (v, +inf): merged (10, 20, +inf, +inf), middle (20, +inf)
    assert O.median_tree(vals, off, 1, 2, np.array([1, 1, 0], np.uint8)) == (20, 0)
    assert O.median_tree(vals, off, 1, 2, np.array([1, 1, 1], np.uint8))[1] == 1
    # both forward (-inf, v): merged (-inf, -inf, 10, 20), middle (-inf, 10)
    assert O.median_tree(vals, off, 1, 2, np.array([0, 0, 0], np.uint8))[1] == -1
    assert O.median_tree(vals, off, 1, 2, np.array([0, 0, 1], np.uint8)) == (10, 0)


def _golden_rank_error():
    path = os.path.join(os.path.dirname(__file__), "golden", "median_tree_rank_error.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    return {int(r[0]): (float(r[1]), float(r[2])) for r in rows}


def _median_tree_rank_errors(n, runs, seed):
    """Rank errors |r/(n-1) - 1/2| of the oracle's binary-tree median over
    `runs` inputs of n distinct uniform 32-bit integers, two per leaf, k = 2."""
    rng = np.random.default_rng(seed)
    p = n // 2
    off = np.arange(0, n + 1, 2, dtype=np.uint64)
    errs = np.empty(runs)
    for r in range(runs):
        vals = rng.choice(1 << 32, size=n, replace=False).astype(np.uint64)
        coins = rng.integers(0, 2, size=p + 1).astype(np.uint8)
        v, side = O.median_tree(vals, off, p.bit_length() - 1, 2, coins)
        assert side == 0
        errs[r] = abs(int((vals < v).sum()) / (n - 1) - 0.5)
    return errs


def test_median_tree_reproduces_printed_rank_error_curve():
    """Figure 4 (Appendix H): 2000 runs per n on uniform 32-bit integers.  With
    two elements per leaf and k = 2 (the reading of the experiment's setup) the
    oracle reproduces the printed maxima exactly at n = 4, 8 and 16, where the
    worst case is hit with near-certainty in 2000 runs.  For n = 32 .. 2048 the
    maximum of 2000 runs is itself a random quantity, and the test only asks
    that it lies within -20 % / +25 % of the printed value.  The printed
    "variance" is matched as the mean squared rank error (the variance of
    r/(n-1) about its expectation 1/2), within 12 %."""
    gold = _golden_rank_error()
    for n in (4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048):
        errs = _median_tree_rank_errors(n, 2000, seed=1)
        gmax, gvar = gold[n]
        if n <= 16:
            assert errs.max() == pytest.approx(gmax, abs=1e-6)
        else:
            assert 0.8 * gmax <= errs.max() <= 1.25 * gmax, n
        assert errs.max() <= 1.44 * n ** -0.39 * 1.05 or n < 32  # the appendix's fitted bound
        assert np.mean(errs ** 2) == pytest.approx(gvar, rel=0.12), n
