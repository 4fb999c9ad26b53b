"""Python binding of librsort (argument marshalling only).

Device memory and streams come from PyTorch; every sorting step runs in the
library's HIP kernels.  The functions mirror the C ABI in include/rsort.h.
Importing this module does not need a GPU; calling a sort does, and fails
with an exception if the library is not built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librsort.so")
# Tuning measured by the autotuner (paper_1606_08766_amd/autotune.py) on an
# MI355X, applied when the library is loaded.  RSORT_TUNING=<path> selects
# another file, RSORT_TUNING=none keeps the compiled defaults.  Every tuning
# yields the same output; only speed differs.
DEFAULT_TUNING = os.path.join(_PKG, "tuning_mi355x.json")

U32, U64, F32 = 0, 1, 2
# Key types by tensor dtype.  Signed integer tensors are not mapped: their
# keys would be ordered by the unsigned bit pattern (negative after
# positive), so they are rejected unless the caller passes kt explicitly.
KT_OF_DTYPE = {torch.uint32: U32, torch.uint64: U64, torch.float32: F32}
KEY_BYTES = {U32: 4, U64: 8, F32: 4}

OK, PENDING, EINVAL, ENOMEM, EDEVICE, EBUSY, ENOTFOUND = 0, 1, -1, -2, -3, -4, -5

EXPORTS = [
    "rsort_strerror", "rsort_version", "rsort_plain_workspace", "rsort_plain", "rsort_segmented_workspace",
    "rsort_segmented", "rsort_workspace_status", "rsort_stats", "rsort_get_tuning", "rsort_set_tuning",
    "rsort_server_create", "rsort_server_destroy", "rsort_submit", "rsort_poll", "rsort_wait", "rsort_release",
    "rsort_server_counters", "rsort_median_tree_workspace", "rsort_median_tree", "rsort_timing_begin",
    "rsort_timing_end", "rsort_class_stats", "rsort_server_request_bytes", "rsort_rquick_mw_workspace",
    "rsort_rquick_mw", "rsort_plain_noalloc", "rsort_bandwidth_probe",
    "rsort_plain64_workspace", "rsort_plain64",
]


class RsortError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__("%s: %s (%d)" % (what or "rsort", strerror(code), code))


class Tuning(ctypes.Structure):
    _fields_ = [
        ("oversample", ctypes.c_uint32), ("target", ctypes.c_uint32), ("cap", ctypes.c_uint32),
        ("max_levels", ctypes.c_uint32), ("rfis_max", ctypes.c_uint32), ("rquick_max", ctypes.c_uint32),
        ("seed", ctypes.c_uint64), ("tile_log2", ctypes.c_uint32), ("force_fallback", ctypes.c_uint32),
        ("extra_levels", ctypes.c_uint32), ("class_shape", ctypes.c_uint32),
    ]


class Request(ctypes.Structure):
    _fields_ = [("kt", ctypes.c_int), ("keys_in", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("keys_out", ctypes.c_void_p), ("perm_out", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("t_submit_ns", ctypes.c_uint64), ("t_start_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("batch_size", ctypes.c_uint32),
                ("dev_begin_ns", ctypes.c_uint64), ("dev_end_ns", ctypes.c_uint64)]


_lib = None


def lib():
    """The loaded librsort.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librsort.so is not built (run __graft_entry__.build()); "
                               "there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, u32, i32, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_size_t
        L.rsort_strerror.restype = ctypes.c_char_p
        L.rsort_strerror.argtypes = [i32]
        L.rsort_version.restype = i32
        L.rsort_plain_workspace.restype = sz
        L.rsort_plain_workspace.argtypes = [i32, u64]
        L.rsort_plain.restype = i32
        L.rsort_plain.argtypes = [i32, vp, u64, vp, vp, vp, sz, vp]
        L.rsort_segmented_workspace.restype = sz
        L.rsort_segmented_workspace.argtypes = [i32, u64, u32, i32]
        L.rsort_segmented.restype = i32
        L.rsort_segmented.argtypes = [i32, vp, vp, vp, u32, u64, vp, vp, vp, vp, sz, vp]
        L.rsort_workspace_status.restype = i32
        L.rsort_workspace_status.argtypes = [vp, vp]
        L.rsort_stats.restype = i32
        L.rsort_stats.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.rsort_get_tuning.restype = i32
        L.rsort_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
        L.rsort_set_tuning.restype = i32
        L.rsort_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
        L.rsort_server_create.restype = i32
        L.rsort_server_create.argtypes = [i32, u64, u32, ctypes.POINTER(vp)]
        L.rsort_server_destroy.restype = i32
        L.rsort_server_destroy.argtypes = [vp]
        L.rsort_submit.restype = i32
        L.rsort_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(u64)]
        L.rsort_poll.restype = i32
        L.rsort_poll.argtypes = [vp, u64, ctypes.POINTER(Result)]
        L.rsort_wait.restype = i32
        L.rsort_wait.argtypes = [vp, u64, u32, ctypes.POINTER(Result)]
        L.rsort_release.restype = i32
        L.rsort_release.argtypes = [vp, u64]
        L.rsort_server_counters.restype = i32
        L.rsort_server_counters.argtypes = [vp] + [ctypes.POINTER(u64)] * 4
        L.rsort_server_request_bytes.restype = sz
        L.rsort_server_request_bytes.argtypes = [i32, u64]
        L.rsort_class_stats.restype = i32
        L.rsort_class_stats.argtypes = [vp, vp, u32, vp, vp, vp]
        L.rsort_timing_begin.restype = i32
        L.rsort_timing_end.restype = i32
        L.rsort_timing_end.argtypes = [u32, vp, u32, vp, vp, ctypes.POINTER(u32)]
        L.rsort_median_tree_workspace.restype = sz
        L.rsort_median_tree_workspace.argtypes = [u32, u32, u32]
        L.rsort_median_tree.restype = i32
        L.rsort_median_tree.argtypes = [vp, u64, vp, u32, u32, vp, u32, vp, vp, sz, vp]
        L.rsort_rquick_mw_workspace.restype = sz
        L.rsort_rquick_mw_workspace.argtypes = [u64, u32]
        L.rsort_plain64_workspace.restype = sz
        L.rsort_plain64_workspace.argtypes = [i32, u64]
        L.rsort_plain64.restype = i32
        L.rsort_plain64.argtypes = [i32, vp, u64, vp, vp, vp, sz, vp]
        L.rsort_bandwidth_probe.restype = i32
        L.rsort_bandwidth_probe.argtypes = [i32, vp, vp, u64, vp]
        L.rsort_plain_noalloc.restype = i32
        L.rsort_plain_noalloc.argtypes = [i32, vp, u64, vp, vp, vp]
        L.rsort_rquick_mw.restype = i32
        L.rsort_rquick_mw.argtypes = [i32, vp, u64, u32, u32, i32, u64, vp, vp, vp, vp, sz, vp]
        _lib = L
        path = os.environ.get("RSORT_TUNING", DEFAULT_TUNING)
        if path != "none" and os.path.exists(path):
            from paper_1606_08766_amd import autotune

            autotune.load(path)
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().rsort_strerror(code).decode()
    except RuntimeError:
        return "status %d" % code


def _check(rc: int, what: str):
    if rc != OK:
        raise RsortError(rc, what)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _kt(keys: torch.Tensor, kt=None) -> int:
    if kt is not None:
        if kt not in KEY_BYTES:
            raise ValueError("unknown key type %r" % (kt,))
        if keys.element_size() != KEY_BYTES[kt]:
            raise TypeError("key type %d needs %d-byte elements, got %s" % (kt, KEY_BYTES[kt], keys.dtype))
        return kt
    if keys.dtype in (torch.int32, torch.int64):
        raise TypeError("signed %s keys would be sorted by their unsigned bit pattern; pass uint32 / uint64 "
                        "tensors, or kt=U32 / U64 to sort the bits as unsigned on purpose" % keys.dtype)
    if keys.dtype not in KT_OF_DTYPE:
        raise TypeError("unsupported key dtype %s" % keys.dtype)
    return KT_OF_DTYPE[keys.dtype]


def _require_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("tensors must be contiguous device tensors")


def _require_like(t, name: str, device, numel: int, elem_bytes: int, dtypes=None):
    """An output / side tensor the library reads or writes through a raw
    pointer: on the keys' device, contiguous, of the right element size (and
    dtype, if given) and length."""
    if t is None:
        return
    if not t.is_cuda or not t.is_contiguous() or t.device != device:
        raise ValueError("%s must be a contiguous tensor on %s" % (name, device))
    if t.element_size() != elem_bytes or (dtypes is not None and t.dtype not in dtypes):
        raise TypeError("%s has dtype %s" % (name, t.dtype))
    if t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))


_U32_LIKE = (torch.uint32, torch.int32)


def _keep_alive(stream, *ts):
    """Tensors used by work enqueued on an explicitly given stream other than
    the current one must not return to torch's caching allocator before that
    work has run: record them on that stream."""
    if stream is None or stream == torch.cuda.current_stream():
        return
    for t in ts:
        if t is not None:
            t.record_stream(stream)


# ----------------------------------------------------------------------------- plain
def plain_workspace_bytes(kt: int, n: int) -> int:
    return int(lib().rsort_plain_workspace(kt, n))


def sort(keys: torch.Tensor, with_perm: bool = True, kt=None, workspace: torch.Tensor | None = None,
         out: tuple | None = None, stream=None):
    """Sort a 1-D device tensor of u32 / u64 / f32 keys.

    Returns (keys_out, perm_out or None); perm_out[r] is the input position of
    the element of rank r (equal keys keep input order)."""
    kt = _kt(keys, kt)
    _require_cuda(keys)
    n = keys.numel()
    if out is not None:
        ko, po = out
    else:
        ko = torch.empty_like(keys)
        po = torch.empty(n, dtype=torch.uint32, device=keys.device) if with_perm else None
    _require_like(ko, "keys_out", keys.device, n, keys.element_size())
    _require_like(po, "perm_out", keys.device, n, 4, _U32_LIKE)
    wsb = plain_workspace_bytes(kt, n)
    if workspace is None:
        workspace = torch.empty(max(wsb, 256), dtype=torch.uint8, device=keys.device)
    _require_cuda(workspace)
    rc = lib().rsort_plain(kt, _ptr(keys), n, _ptr(ko), _ptr(po), _ptr(workspace), workspace.numel(), _stream(stream))
    _check(rc, "rsort_plain")
    _keep_alive(stream, keys, ko, po, workspace)
    return ko, po


def plain64_workspace_bytes(kt: int, n: int) -> int:
    return int(lib().rsort_plain64_workspace(kt, n))


def sort64(keys: torch.Tensor, with_perm: bool = True, kt=None, workspace: torch.Tensor | None = None,
           out: tuple | None = None, stream=None):
    """rsort_plain64: the same sort with 64-bit positions (any n up to 2^36).
    Returns (keys_out, perm_out as a u64 tensor, or None)."""
    kt = _kt(keys, kt)
    _require_cuda(keys)
    n = keys.numel()
    if out is not None:
        ko, po = out
    else:
        ko = torch.empty_like(keys)
        po = torch.empty(n, dtype=torch.uint64, device=keys.device) if with_perm else None
    _require_like(ko, "keys_out", keys.device, n, keys.element_size())
    _require_like(po, "perm_out", keys.device, n, 8, (torch.uint64, torch.int64))
    if workspace is None:
        workspace = torch.empty(max(plain64_workspace_bytes(kt, n), 256), dtype=torch.uint8, device=keys.device)
    _require_cuda(workspace)
    rc = lib().rsort_plain64(kt, _ptr(keys), n, _ptr(ko), _ptr(po), _ptr(workspace), workspace.numel(),
                             _stream(stream))
    _check(rc, "rsort_plain64")
    _keep_alive(stream, keys, ko, po, workspace)
    return ko, po


# ----------------------------------------------------------------------------- segmented
def segmented_workspace_bytes(kt: int, n_total: int, num_segs: int, has_payload: bool) -> int:
    return int(lib().rsort_segmented_workspace(kt, n_total, num_segs, 1 if has_payload else 0))


def segmented_sort(keys: torch.Tensor, offsets: torch.Tensor, payload: torch.Tensor | None = None,
                   with_perm: bool = True, kt=None, workspace: torch.Tensor | None = None, out: tuple | None = None,
                   stream=None):
    """Sort every segment [offsets[s], offsets[s+1]) independently.

    offsets: device u64 (or int64) tensor of num_segs + 1 entries.  Returns
    (keys_out, perm_out or None, payload_out or None); perm is segment-local."""
    kt = _kt(keys, kt)
    _require_cuda(keys, offsets, payload)
    n = keys.numel()
    ns = offsets.numel() - 1
    if ns < 0:
        raise ValueError("offsets needs num_segs + 1 >= 1 entries")
    _require_like(offsets, "offsets", keys.device, ns + 1, 8, (torch.uint64, torch.int64))
    _require_like(payload, "payload", keys.device, n, 4, _U32_LIKE)
    if out is not None:
        ko, po, plo = out
    else:
        ko = torch.empty_like(keys)
        po = torch.empty(n, dtype=torch.uint32, device=keys.device) if with_perm else None
        plo = torch.empty_like(payload) if payload is not None else None
    _require_like(ko, "keys_out", keys.device, n, keys.element_size())
    _require_like(po, "perm_out", keys.device, n, 4, _U32_LIKE)
    _require_like(plo, "payload_out", keys.device, n, 4, _U32_LIKE)
    if (payload is None) != (plo is None):
        raise ValueError("payload and payload_out go together")
    wsb = segmented_workspace_bytes(kt, n, ns, payload is not None)
    if workspace is None:
        workspace = torch.empty(max(wsb, 256), dtype=torch.uint8, device=keys.device)
    _require_cuda(workspace)
    rc = lib().rsort_segmented(kt, _ptr(keys), _ptr(payload), _ptr(offsets), ns, n, _ptr(ko), _ptr(plo), _ptr(po),
                               _ptr(workspace), workspace.numel(), _stream(stream))
    _check(rc, "rsort_segmented")
    _keep_alive(stream, keys, offsets, payload, ko, po, plo, workspace)
    return ko, po, plo


def workspace_status(workspace: torch.Tensor, stream=None) -> int:
    return int(lib().rsort_workspace_status(_ptr(workspace), _stream(stream)))


def stats(workspace: torch.Tensor, stream=None) -> dict:
    """Diagnostics of the last call that used this workspace (see rsort_stats)."""
    import numpy as np

    sk = np.zeros(511, np.uint64)
    sp = np.zeros(511, np.uint32)
    bs = np.zeros(512, np.uint32)
    lm = np.zeros(8, np.uint32)
    lb = np.zeros(8, np.uint32)
    nb, lv, ov = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    rc = lib().rsort_stats(_ptr(workspace), _stream(stream), sk.ctypes.data, sp.ctypes.data, bs.ctypes.data,
                           ctypes.byref(nb), ctypes.byref(lv), lm.ctypes.data, lb.ctypes.data, ctypes.byref(ov))
    k = nb.value
    return {"status": rc, "k": k, "levels": lv.value, "splitter_keys": sk[:max(k - 1, 0)],
            "splitter_pos": sp[:max(k - 1, 0)], "bucket_sizes": bs[:k], "level_max": lm[:lv.value],
            "level_buckets": lb[:lv.value], "oversize": ov.value}


def class_stats(workspace: torch.Tensor, stream=None) -> list:
    """Per final-bucket size class: (largest bucket, buckets, keys) of the last
    call that used this workspace."""
    import numpy as np

    m = 32
    cm = np.zeros(m, np.uint32)
    nb = np.zeros(m, np.uint32)
    nk = np.zeros(m, np.uint64)
    rc = lib().rsort_class_stats(_ptr(workspace), _stream(stream), m, cm.ctypes.data, nb.ctypes.data, nk.ctypes.data)
    if rc < 0:
        raise RsortError(rc, "rsort_class_stats")
    return [(int(cm[i]), int(nb[i]), int(nk[i])) for i in range(rc)]


# ----------------------------------------------------------------------------- tuning
def get_tuning() -> Tuning:
    t = Tuning()
    _check(lib().rsort_get_tuning(ctypes.byref(t)), "rsort_get_tuning")
    return t


def set_tuning(**kw):
    t = Tuning()
    for k, v in kw.items():
        setattr(t, k, v)
    _check(lib().rsort_set_tuning(ctypes.byref(t)), "rsort_set_tuning")


class tuned:
    """Context manager: temporarily change tuning fields."""

    def __init__(self, **kw):
        self.kw = kw

    def __enter__(self):
        self.saved = get_tuning()
        set_tuning(**self.kw)
        return self

    def __exit__(self, *a):
        s = self.saved
        set_tuning(oversample=s.oversample, target=s.target, cap=s.cap, max_levels=s.max_levels,
                   rfis_max=s.rfis_max, rquick_max=s.rquick_max, seed=s.seed, tile_log2=s.tile_log2,
                   force_fallback=1 if s.force_fallback else 2, extra_levels=s.extra_levels,
                   class_shape=s.class_shape)


# ----------------------------------------------------------------------------- timing
def timing_begin():
    _check(lib().rsort_timing_begin(), "rsort_timing_begin")


def timing_end(max_entries: int = 128) -> dict:
    """Stop kernel timing; returns {kernel name: (launches, total ms)}."""
    import numpy as np

    name_len = 160
    names = ctypes.create_string_buffer(max_entries * name_len)
    launches = np.zeros(max_entries, np.uint32)
    ms = np.zeros(max_entries, np.float64)
    n = ctypes.c_uint32()
    _check(lib().rsort_timing_end(max_entries, names, name_len, launches.ctypes.data, ms.ctypes.data,
                                  ctypes.byref(n)), "rsort_timing_end")
    out = {}
    raw = names.raw
    for i in range(n.value):
        nm = raw[i * name_len:(i + 1) * name_len].split(b"\0", 1)[0].decode()
        out[nm] = (int(launches[i]), float(ms[i]))
    return out


# ----------------------------------------------------------------------------- bandwidth probes
def bandwidth_probe(kind: str, src: torch.Tensor, dst: torch.Tensor, nbytes: int, stream=None):
    """Enqueue the library's read-only ("read") or copy ("copy") probe over
    nbytes of src (see rsort_bandwidth_probe)."""
    _require_cuda(src, dst)
    rc = lib().rsort_bandwidth_probe({"read": 0, "copy": 1}[kind], _ptr(src), _ptr(dst), nbytes, _stream(stream))
    _check(rc, "rsort_bandwidth_probe")


# ----------------------------------------------------------------------------- median tree
def median_tree(vals: torch.Tensor, per_problem: int, leaf_off: torch.Tensor, log2_p: int, k: int,
                coins: torch.Tensor, num_problems: int, stream=None) -> torch.Tensor:
    """Device binary-tree approximate median; returns a u64 tensor [num_problems, 2]
    of (value, side) with side 0 real, 1 below-all sentinel, 2 above-all sentinel."""
    _require_cuda(vals, leaf_off, coins)
    out = torch.empty(2 * num_problems, dtype=torch.uint64, device=vals.device)
    wsb = int(lib().rsort_median_tree_workspace(log2_p, k, num_problems))
    if wsb == 0:
        raise RsortError(EINVAL, "rsort_median_tree_workspace")
    ws = torch.empty(wsb, dtype=torch.uint8, device=vals.device)
    rc = lib().rsort_median_tree(_ptr(vals), per_problem, _ptr(leaf_off), log2_p, k, _ptr(coins), num_problems,
                                 _ptr(out), _ptr(ws), wsb, _stream(stream))
    _check(rc, "rsort_median_tree")
    return out.view(num_problems, 2)


# ----------------------------------------------------------------------------- hypercube quicksort
def rquick_mw_workspace_bytes(n: int, log2_p: int) -> int:
    return int(lib().rsort_rquick_mw_workspace(n, log2_p))


def rquick_mw(keys: torch.Tensor, log2_p: int, k: int = 16, tie_break=True, seed: int = 0x5EED,
              with_perm: bool = True, kt=None, workspace: torch.Tensor | None = None, stream=None):
    """Hypercube quicksort of one u32 / f32 array over 2^log2_p workgroups
    (rsort_rquick_mw).  Returns (keys_out, perm_out or None, load) where
    load[0] is the largest PE part after the redistribution and load[1 + r]
    the largest after exchange round r (a device u32 tensor).  tie_break:
    True / 1 = (key, position) split, False / 0 = key-only ablation,
    "local" / 2 = the paper's local choice among copies of the splitter key
    (sorted keys, equal keys in no fixed order)."""
    mode = 2 if tie_break == "local" else int(tie_break)
    _require_cuda(keys)
    kt = _kt(keys, kt)
    n = keys.numel()
    ko = torch.empty_like(keys)
    po = torch.empty(n, dtype=torch.uint32, device=keys.device) if with_perm else None
    load = torch.zeros(log2_p + 1, dtype=torch.uint32, device=keys.device)
    wsb = rquick_mw_workspace_bytes(n, log2_p)
    if workspace is None:
        workspace = torch.empty(max(wsb, 256), dtype=torch.uint8, device=keys.device)
    rc = lib().rsort_rquick_mw(kt, _ptr(keys), n, log2_p, k, mode, seed & (2**64 - 1), _ptr(ko),
                               _ptr(po), _ptr(load), _ptr(workspace), workspace.numel(), _stream(stream))
    _check(rc, "rsort_rquick_mw")
    return ko, po, load


# ----------------------------------------------------------------------------- server
class Server:
    """Continuous-batching sort server (rsort_server_*).  device < 0 uses the
    host-only fake executor (admission logic only, buffers untouched).
    hbm_budget_bytes is reserved at creation as the server's scratch arena."""

    @staticmethod
    def request_bytes(kt: int, n: int) -> int:
        """Arena bytes a request of n keys takes when it runs alone."""
        return int(lib().rsort_server_request_bytes(kt, n))

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 64 << 30, max_inflight: int = 8):
        h = ctypes.c_void_p()
        _check(lib().rsort_server_create(device, hbm_budget_bytes, max_inflight, ctypes.byref(h)),
               "rsort_server_create")
        self.h = h

    def submit(self, kt: int, keys_in_ptr: int, n: int, keys_out_ptr: int, perm_out_ptr: int | None) -> int:
        r = Request(kt, keys_in_ptr, n, keys_out_ptr, perm_out_ptr)
        t = ctypes.c_uint64()
        rc = lib().rsort_submit(self.h, ctypes.byref(r), ctypes.byref(t))
        _check(rc, "rsort_submit")
        return t.value

    def submit_tensors(self, keys: torch.Tensor, keys_out: torch.Tensor, perm_out: torch.Tensor | None, kt=None):
        """Submit device tensors.  The server's streams do not wait on the
        caller's stream, so the work that produced `keys` on the current
        stream is waited for here (host synchronisation) before submitting."""
        kt = _kt(keys, kt)
        _require_cuda(keys)
        _require_like(keys_out, "keys_out", keys.device, keys.numel(), keys.element_size())
        _require_like(perm_out, "perm_out", keys.device, keys.numel(), 4, _U32_LIKE)
        torch.cuda.current_stream(keys.device).synchronize()
        return self.submit(_kt(keys, kt), keys.data_ptr(), keys.numel(), keys_out.data_ptr(),
                           perm_out.data_ptr() if perm_out is not None else None)

    def poll(self, ticket: int):
        r = Result()
        rc = lib().rsort_poll(self.h, ticket, ctypes.byref(r))
        return rc, r

    def wait(self, ticket: int, timeout_ms: int = 60000):
        r = Result()
        rc = lib().rsort_wait(self.h, ticket, timeout_ms, ctypes.byref(r))
        return rc, r

    def release(self, ticket: int) -> int:
        return lib().rsort_release(self.h, ticket)

    def counters(self):
        v = [ctypes.c_uint64() for _ in range(4)]
        _check(lib().rsort_server_counters(self.h, *[ctypes.byref(x) for x in v]), "rsort_server_counters")
        return {"queued": v[0].value, "running": v[1].value, "finished": v[2].value, "bytes_in_use": v[3].value}

    def close(self):
        if self.h:
            lib().rsort_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
