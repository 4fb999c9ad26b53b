"""GPU parity of the hypercube quicksort over workgroups (rsort_rquick_mw)
against the oracle's sort, with and without the tie-break, and its load
balance (Section 6: random redistribution plus binary-tree median splitters
keep the PE parts near n / p; without tie-breaking, equal keys pile up)."""
import numpy as np
import pytest
import torch

from gen import gen
from oracle import oracle as O
from paper_1606_08766_amd import rsort as R
from tests.gpu_util import banner, dev, host, same_bits

pytestmark = pytest.mark.gpu


def run(x, log2_p, k=16, tie_break=True, seed=7):
    banner("rquick_mw n=%d log2_p=%d k=%d tie_break=%s" % (x.size, log2_p, k, tie_break))
    ko, po, load = R.rquick_mw(dev(x), log2_p, k=k, tie_break=tie_break, seed=seed)
    return host(ko), host(po), host(load).astype(np.int64)


@pytest.mark.parametrize("n,log2_p", [(1, 1), (5, 3), (1000, 2), (8193, 2), ((1 << 13) + 3, 4), ((1 << 16) + 5, 4),
                                      (1 << 18, 5), ((1 << 18) + 7, 8)])
@pytest.mark.parametrize("dist", ["uniform", "zero", "deterdupl", "reverse", "gaussian"])
def test_rquick_mw_matches_oracle(n, log2_p, dist):
    x = gen.keys("u32", dist, n, seed=n % 97 + log2_p)
    ek, ep, _ = O.sort(x, threads=4)
    ko, po, load = run(x, log2_p)
    assert same_bits(ko, ek) and np.array_equal(po, ep)
    p = 1 << log2_p
    assert load[0] <= -(-n // p)  # the shuffle keeps parts within one key of n / p


@pytest.mark.parametrize("dist", ["uniform", "zero", "deterdupl"])
def test_rquick_mw_without_tie_break_is_exact(dist):
    n, log2_p = (1 << 16) + 11, 4
    x = gen.keys("u32", dist, n, seed=3)
    ek, ep, _ = O.sort(x, threads=4)
    ko, po, load = run(x, log2_p, tie_break=False)
    assert same_bits(ko, ek) and np.array_equal(po, ep)
    if dist == "zero":
        assert load[-1] == n  # every split sends all equal keys to one side


@pytest.mark.parametrize("dist", ["uniform", "zero", "deterdupl", "dup8"])
def test_rquick_mw_local_tie_scheme_sorts_keys(dist):
    """The paper's local choice among copies of the splitter key: the keys
    come out sorted (unique), equal keys in some order, so the permutation is
    checked for being a valid sorting permutation."""
    n, log2_p = (1 << 17) + 3, 5
    x = gen.keys("u32", "topbits" if dist == "dup8" else dist, n, seed=4, param=3 if dist == "dup8" else 0)
    ek, _, _ = O.sort(x, threads=4)
    ko, po, load = run(x, log2_p, tie_break="local")
    assert same_bits(ko, ek)
    assert np.array_equal(np.sort(po.astype(np.int64)), np.arange(n)) and same_bits(x[po], ek)
    if dist == "zero":
        # every split halves a part of equal keys: a part grows by at most one per round
        assert load[-1] <= -(-n // (1 << log2_p)) + log2_p + 1


def test_rquick_mw_f32_specials_and_windows():
    n = (1 << 15) + 9
    x = gen.keys("f32", "uniform", n, seed=11)  # random bit patterns: NaNs, infinities, signed zeros
    ek, ep, _ = O.sort(x, threads=4)
    for k in (2, 8, 16):
        ko, po, _ = run(x, 3, k=k, seed=k)
        assert same_bits(ko, ek) and np.array_equal(po, ep)


def test_rquick_mw_load_balance():
    """With the tie-break every final part stays near n / p on uniform and
    all-equal keys; without it all-equal keys end on one PE."""
    n, log2_p = 1 << 18, 6
    p = 1 << log2_p
    for dist in ("uniform", "zero"):
        x = gen.keys("u32", dist, n, seed=5)
        _, _, load = run(x, log2_p)
        assert load[-1] <= 1.5 * n / p, (dist, load)


def test_rquick_mw_workspace_status_stays_ok():
    """The LDS-capacity guard of the local sort never fires for accepted
    shapes: the largest part is exactly ceil(n / p) after the shuffle."""
    n, log2_p = (1 << 18) + 5, 6
    x = gen.keys("u32", "uniform", n, seed=8)
    ws = torch.empty(R.rquick_mw_workspace_bytes(n, log2_p), dtype=torch.uint8, device="cuda")
    banner("rquick_mw workspace status")
    _, _, load = R.rquick_mw(dev(x), log2_p, workspace=ws)
    assert R.workspace_status(ws) == R.OK
    assert int(host(load)[0]) <= -(-n // (1 << log2_p))


def test_rquick_mw_seed_changes_nothing_in_the_output():
    n = (1 << 17) + 1
    x = gen.keys("u32", "deterdupl", n, seed=9)
    a = run(x, 5, seed=1)
    b = run(x, 5, seed=2)
    assert same_bits(a[0], b[0]) and np.array_equal(a[1], b[1])
