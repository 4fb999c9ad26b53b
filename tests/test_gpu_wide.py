"""rsort_plain64 (64-bit positions, for 2^32 keys and more): bit-exact
against the oracle at sizes it sorts quickly, and at 2^32 + 17 keys checked
on the device for the characterising properties plus ranks of sampled
outputs computed from the definition by the oracle."""
import numpy as np
import pytest
import torch

from gen import gen
from oracle import oracle as O
from paper_1606_08766_amd import rsort as R
from tests.checks import check_sorted_device
from tests.gpu_util import banner, dev, host, same_bits

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 2, 63, 1000, 12289, 300007, (1 << 20) + 7, 3_000_001])
@pytest.mark.parametrize("kt,dist", [("u64", "uniform"), ("u32", "uniform"), ("f32", "uniform"),
                                     ("u64", "deterdupl"), ("u64", "zero"), ("u32", "topbits"),
                                     ("f32", "gaussian")])
def test_plain64_parity(n, kt, dist):
    x = gen.keys(kt, dist, n, seed=n + 21, param=3 if dist == "topbits" else 0)
    banner("plain64 %s %s n=%d" % (kt, dist, n))
    ko, po = R.sort64(dev(x))
    torch.cuda.synchronize()
    ek, ep, _ = O.sort(x)
    assert same_bits(host(ko), ek)
    assert np.array_equal(host(po), ep.astype(np.uint64))


def test_plain64_keys_only_and_status():
    x = gen.keys("u64", "gaussian", 500_000, seed=4)
    ws = torch.empty(R.plain64_workspace_bytes(R.U64, x.size), dtype=torch.uint8, device="cuda")
    banner("plain64 keys only")
    ko, po = R.sort64(dev(x), with_perm=False, workspace=ws)
    assert po is None
    assert R.workspace_status(ws) == R.OK
    assert same_bits(host(ko), O.sort(x)[0])


def test_plain64_beyond_2p32_keys():
    """2^32 + 17 u32 keys, uniform over all 2^32 values (so about a third of
    them repeat a key and the order of equal keys is decided by 64-bit
    positions)."""
    n = (1 << 32) + 17
    x = gen.keys("u32", "uniform", n, seed=9)
    banner("plain64 u32 n=2^32+17")
    xd = dev(x)
    ws = torch.empty(R.plain64_workspace_bytes(R.U32, n), dtype=torch.uint8, device="cuda")
    ko, po = R.sort64(xd, workspace=ws)
    assert R.workspace_status(ws) == R.OK
    del ws
    torch.cuda.synchronize()
    banner("plain64 u32 n=2^32+17: device checks")
    check_sorted_device(xd, ko, po)
    rng = np.random.default_rng(5)
    for r in [0, n - 1] + rng.integers(0, n, 1).tolist():
        assert O.rank(x, int(po[r].item())) == int(r)
