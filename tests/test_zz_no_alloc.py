"""rsort_plain_noalloc (the entry point for callers that cannot allocate)
called through the C ABI: its output equals rsort_plain's on the same input,
bit for bit, on two calls in a row (the second smaller, so it runs on the
scratch the first one left behind); sizes beyond its static scratch are
refused before any device work."""
import ctypes

import numpy as np
import pytest
import torch

from gen import gen
from paper_1606_08766_amd import rsort as R
from tests.gpu_util import banner, dev, host, same_bits

pytestmark = pytest.mark.gpu


def _noalloc(x: torch.Tensor, kt: int):
    ko = torch.empty_like(x)
    po = torch.empty(x.numel(), dtype=torch.uint32, device=x.device)
    st = torch.cuda.current_stream()
    rc = R.lib().rsort_plain_noalloc(kt, ctypes.c_void_p(x.data_ptr()), x.numel(), ctypes.c_void_p(ko.data_ptr()),
                                     ctypes.c_void_p(po.data_ptr()), ctypes.c_void_p(st.cuda_stream))
    assert rc == R.OK, R.strerror(rc)
    torch.cuda.synchronize()
    return host(ko), host(po)


def _plain(x: torch.Tensor, kt: int):
    ko = torch.empty_like(x)
    po = torch.empty(x.numel(), dtype=torch.uint32, device=x.device)
    ws = torch.empty(max(R.plain_workspace_bytes(kt, x.numel()), 256), dtype=torch.uint8, device=x.device)
    st = torch.cuda.current_stream()
    rc = R.lib().rsort_plain(kt, ctypes.c_void_p(x.data_ptr()), x.numel(), ctypes.c_void_p(ko.data_ptr()),
                             ctypes.c_void_p(po.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                             ctypes.c_void_p(st.cuda_stream))
    assert rc == R.OK, R.strerror(rc)
    torch.cuda.synchronize()
    return host(ko), host(po)


@pytest.mark.parametrize("kt_name,dist,n1,n2", [("u64", "uniform", 2_000_003, 300_007),
                                                ("u64", "deterdupl", 1 << 21, 9000),
                                                ("f32", "uniform", 3_000_000, 1 << 20),
                                                ("u32", "zero", 77_777, 5000)])
def test_noalloc_equals_plain_on_two_calls(kt_name, dist, n1, n2):
    kt = {"u64": R.U64, "u32": R.U32, "f32": R.F32}[kt_name]
    for n, seed in ((n1, 1), (n2, 2)):
        x = dev(gen.keys(kt_name, dist, n, seed=seed))
        banner("noalloc %s %s n=%d" % (kt_name, dist, n))
        a = _noalloc(x, kt)
        banner("plain %s %s n=%d" % (kt_name, dist, n))
        b = _plain(x, kt)
        assert same_bits(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_noalloc_refuses_sizes_beyond_its_scratch():
    n = 1 << 24  # needs far more than the 64 MiB scratch
    assert R.plain_workspace_bytes(R.U64, n) > (64 << 20)
    rc = R.lib().rsort_plain_noalloc(R.U64, ctypes.c_void_p(16), n, ctypes.c_void_p(1 << 40), None, None)
    assert rc == R.ENOMEM
