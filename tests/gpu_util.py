"""Helpers for the GPU tests: device copies and a case banner printed (and
flushed) before every GPU call so a failing run names its case."""
import sys

import numpy as np
import torch

from paper_1606_08766_amd import rsort as R


def banner(msg: str):
    sys.stdout.write("[gpu] %s\n" % msg)
    sys.stdout.flush()


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy()


def gpu_sort(x: np.ndarray, with_perm: bool = True):
    banner("plain sort n=%d dtype=%s" % (x.size, x.dtype))
    ko, po = R.sort(dev(x), with_perm=with_perm)
    torch.cuda.synchronize()
    return host(ko), (host(po) if po is not None else None)


def gpu_segmented(keys: np.ndarray, offsets: np.ndarray, payload=None, with_perm=True, check_status=True):
    banner("segmented sort n=%d segs=%d dtype=%s payload=%s" % (keys.size, offsets.size - 1, keys.dtype,
                                                                 payload is not None))
    kt = R.KT_OF_DTYPE[torch.from_numpy(keys[:0]).dtype]
    ws = torch.empty(max(R.segmented_workspace_bytes(kt, keys.size, offsets.size - 1, payload is not None), 256),
                     dtype=torch.uint8, device="cuda")
    ko, po, plo = R.segmented_sort(dev(keys), dev(offsets.astype(np.uint64)),
                                   dev(payload) if payload is not None else None, with_perm=with_perm, workspace=ws)
    st = R.workspace_status(ws)
    if check_status:
        assert st == R.OK, R.strerror(st)
    return host(ko), (host(po) if po is not None else None), (host(plo) if plo is not None else None), st


def same_bits(a: np.ndarray, b: np.ndarray) -> bool:
    return a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8))
