"""Output checks used by the tests.

``check_sorted`` verifies three properties that together characterise the
unique correct output of a sort under the (key, input position) order:
  1. perm is a bijection on 0..n-1;
  2. keys_out[r] equals keys_in[perm[r]] bit for bit (same for payload);
  3. (ord(keys_out[r]), perm[r]) is strictly increasing in r.
Any output passing all three equals the definition, so these checks pin
parity at sizes where running a reference sort is too slow.

``closed_form`` returns the exact output for input families whose sorted order
follows from their formula alone.
"""
from __future__ import annotations

import numpy as np


def ord_bits(keys: np.ndarray) -> np.ndarray:
    """Order-preserving unsigned view (f32: IEEE 754 totalOrder on bit patterns)."""
    if keys.dtype == np.float32:
        b = keys.view(np.uint32)
        neg = (b >> np.uint32(31)).astype(bool)
        return np.where(neg, ~b, b | np.uint32(0x80000000))
    return keys


def check_sorted(keys_in, keys_out, perm, payload_in=None, payload_out=None, chunk=1 << 26):
    n = keys_in.size
    assert keys_out.size == n and perm.size == n
    if n == 0:
        return
    assert perm.dtype == np.uint32
    assert int(perm.max()) < n, "perm entry out of range"
    seen = np.zeros(n, dtype=bool)
    seen[perm] = True
    assert seen.all(), "perm is not a bijection"
    del seen
    kin = keys_in.view(np.uint64 if keys_in.itemsize == 8 else np.uint32)
    kout = keys_out.view(kin.dtype)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        p = perm[a:b]
        assert np.array_equal(kout[a:b], kin[p]), "keys_out[r] != keys_in[perm[r]] near %d" % a
        if payload_in is not None:
            assert np.array_equal(payload_out[a:b], payload_in[p]), "payload mismatch near %d" % a
        lo = max(a - 1, 0)
        o = ord_bits(keys_out[lo:b])
        q = perm[lo:b]
        inc = (o[1:] > o[:-1]) | ((o[1:] == o[:-1]) & (q[1:] > q[:-1]))
        if not inc.all():
            r = lo + int(np.argmin(inc))
            raise AssertionError("order violated between ranks %d and %d" % (r, r + 1))


def closed_form(dist: str, n: int, dtype=np.uint64, distinct: int = 16):
    """Exact (keys_out, perm) for zero / reverse / deterdupl / sorted inputs."""
    r = np.arange(n, dtype=np.uint64)
    if dist == "zero":
        return np.zeros(n, dtype=dtype), r.astype(np.uint32)
    if dist == "sorted":
        return r.astype(dtype), r.astype(np.uint32)
    if dist == "reverse":
        return r.astype(dtype), (np.uint64(n - 1) - r).astype(np.uint32)
    if dist == "deterdupl":
        d = distinct
        # key v occurs at positions v, v+d, v+2d, ... ; count of key v is ceil((n-v)/d)
        cnt = np.array([(n - v + d - 1) // d if v < n else 0 for v in range(d)], dtype=np.uint64)
        start = np.concatenate([[0], np.cumsum(cnt)[:-1]]).astype(np.uint64)
        key = np.repeat(np.arange(d, dtype=np.int64), cnt.astype(np.int64)).astype(np.uint64)
        j = r - start[key.astype(np.int64)]
        return key.astype(dtype), (np.uint64(d) * j + key).astype(np.uint32)
    raise ValueError(dist)


def check_sorted_segmented_device(keys, offsets, keys_out, perm, payload=None, payload_out=None,
                                  chunk=1 << 27):
    """The three characterising properties of ``check_sorted``, per segment,
    evaluated with plain torch operations on device tensors (for inputs of
    billions of keys, where host checks would take minutes):

      1. perm maps every segment onto its own positions bijectively;
      2. keys_out[r] == keys[start(r) + perm[r]] bit for bit (and payload);
      3. (ord(keys_out[r]), perm[r]) strictly increases inside each segment.

    keys/keys_out: u64 or u32 tensors (unsigned order; f32 is not handled
    here); offsets: host numpy u64 array of num_segs + 1 entries; perm: u32."""
    import torch

    n = keys.numel()
    dev = keys.device
    assert keys_out.numel() == n and perm.numel() == n
    if n == 0:
        return
    wide = keys.element_size() == 8
    sdt = torch.int64 if wide else torch.int32
    flip = torch.tensor(-(1 << 63) if wide else -(1 << 31), dtype=sdt, device=dev)
    off = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).to(dev)
    lengths = off[1:] - off[:-1]
    nseg = lengths.numel()
    seg = torch.repeat_interleave(torch.arange(nseg, device=dev, dtype=torch.int32), lengths, output_size=n)
    seen = torch.zeros(n, dtype=torch.bool, device=dev)
    kin = keys.view(sdt)
    kout = keys_out.view(sdt)
    pin = perm.view(torch.int32)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        sg = seg[a:b].long()
        p = pin[a:b].long() & 0xFFFFFFFF
        assert bool((p < lengths[sg]).all()), "perm entry outside its segment near %d" % a
        g = off[sg] + p
        seen[g] = True
        assert torch.equal(kout[a:b], kin[g]), "keys_out[r] != keys[start + perm[r]] near %d" % a
        if payload is not None:
            assert torch.equal(payload_out.view(torch.int32)[a:b], payload.view(torch.int32)[g]), \
                "payload mismatch near %d" % a
        lo = max(a - 1, 0)
        o = kout[lo:b] ^ flip
        q = pin[lo:b].long() & 0xFFFFFFFF
        same = seg[lo + 1:b] == seg[lo:b - 1]
        inc = (o[1:] > o[:-1]) | ((o[1:] == o[:-1]) & (q[1:] > q[:-1]))
        bad = same & ~inc
        if bool(bad.any()):
            r = lo + int(torch.nonzero(bad)[0].item())
            raise AssertionError("order violated between ranks %d and %d" % (r, r + 1))
        del sg, p, g, o, q, same, inc, bad
    assert bool(seen.all()), "perm is not a bijection on some segment"


def check_sorted_device(keys, keys_out, perm, chunk=1 << 27):
    """``check_sorted``'s three characterising properties for one array with
    a 64-bit permutation, evaluated with plain torch operations on device
    tensors (arrays of 2^32 keys and more): perm is a bijection on 0..n-1,
    keys_out[r] == keys[perm[r]] bit for bit, and (ord(keys_out[r]), perm[r])
    strictly increases.  keys: u64 or u32 tensors (unsigned order); perm: u64."""
    import torch

    n = keys.numel()
    assert keys_out.numel() == n and perm.numel() == n
    if n == 0:
        return
    dev = keys.device
    wide = keys.element_size() == 8
    sdt = torch.int64 if wide else torch.int32
    flip = torch.tensor(-(1 << 63) if wide else -(1 << 31), dtype=sdt, device=dev)
    kin, kout, p64 = keys.view(sdt), keys_out.view(sdt), perm.view(torch.int64)
    seen = torch.zeros(n, dtype=torch.bool, device=dev)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        p = p64[a:b]
        assert bool(((p >= 0) & (p < n)).all()), "perm entry out of range near %d" % a
        seen[p] = True
        assert torch.equal(kout[a:b], kin[p]), "keys_out[r] != keys[perm[r]] near %d" % a
        lo = max(a - 1, 0)
        o = kout[lo:b] ^ flip
        q = p64[lo:b]
        inc = (o[1:] > o[:-1]) | ((o[1:] == o[:-1]) & (q[1:] > q[:-1]))
        if not bool(inc.all()):
            r = lo + int(torch.nonzero(~inc)[0].item())
            raise AssertionError("order violated between ranks %d and %d" % (r, r + 1))
        del p, o, q, inc
    assert bool(seen.all()), "perm is not a bijection"
