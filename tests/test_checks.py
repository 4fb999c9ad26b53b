"""The device-side output checker used at sizes the oracle cannot sort as a
whole, pinned on the CPU: the oracle's output passes it, and planted mistakes
(a swapped pair, a permutation entry of another segment, a payload error, a
duplicated position) each fail it."""
import numpy as np
import pytest
import torch

from gen import gen
from oracle import oracle as O
from tests.checks import check_sorted_segmented_device


def _case(kt):
    sizes = np.array([5, 0, 300, 1, 2000, 77], dtype=np.uint64)
    keys, pay, off = gen.segmented(kt, sizes, ["uniform", "zero", "deterdupl", "uniform", "reverse", "gaussian"],
                                   seed=4)
    ko, po, plo = O.segmented(keys, off, pay)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    return t(keys), off, t(ko), t(po), t(pay), t(plo)


@pytest.mark.parametrize("kt", ["u64", "u32"])
def test_device_checker_accepts_the_oracle(kt):
    keys, off, ko, po, pay, plo = _case(kt)
    check_sorted_segmented_device(keys, off, ko, po, pay, plo, chunk=97)


@pytest.mark.parametrize("kt", ["u64", "u32"])
@pytest.mark.parametrize("mistake", ["swap", "foreign_perm", "payload", "dup_perm"])
def test_device_checker_rejects_planted_mistakes(kt, mistake):
    keys, off, ko, po, pay, plo = _case(kt)
    ko, po, plo = ko.clone(), po.clone(), plo.clone()
    a = int(off[2]) + 10  # inside the 300-key segment
    if mistake == "swap":
        for t in (ko, po, plo):
            t[a], t[a + 1] = t[a + 1].clone(), t[a].clone()
    elif mistake == "foreign_perm":
        po[int(off[5])] = 1500  # a position beyond its 77-key segment
    elif mistake == "payload":
        plo[a] ^= 1
    else:
        po[a + 1] = po[a]
        ko[a + 1] = ko[a]
        plo[a + 1] = plo[a]
    with pytest.raises(AssertionError):
        check_sorted_segmented_device(keys, off, ko, po, pay, plo, chunk=97)


@pytest.mark.parametrize("kt", ["u64", "u32"])
def test_single_array_device_checker(kt):
    """check_sorted_device (64-bit permutations) accepts the oracle's output
    and rejects a swapped pair, a duplicated position and a wrong key."""
    from tests.checks import check_sorted_device

    x = gen.keys(kt, "deterdupl", 5000, seed=3)
    ek, ep, _ = O.sort(x)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    keys, ko, po = t(x), t(ek), t(ep.astype(np.uint64))
    check_sorted_device(keys, ko, po, chunk=333)
    for mistake in ("swap", "dup", "key"):
        k2, p2 = ko.clone(), po.clone()
        if mistake == "swap":
            k2[100], k2[4000] = ko[4000].clone(), ko[100].clone()
            p2[100], p2[4000] = po[4000].clone(), po[100].clone()
        elif mistake == "dup":
            p2[101] = p2[100]
            k2[101] = k2[100]
        else:
            kv = k2.view(torch.int64 if kt == "u64" else torch.int32)
            kv[7] += 1
        with pytest.raises(AssertionError):
            check_sorted_device(keys, k2, p2, chunk=333)
