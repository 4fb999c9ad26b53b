"""CPU ORACLE (test infrastructure only) -- Python view of ``oracle.cpp``.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The GPU library never calls it, and it shares no code
with the GPU library.

Definition followed (paper Section 2 and Appendices F/G): sorting n keys
returns the unique permutation pi with (ord(x[pi(r)]), pi(r)) strictly
increasing, i.e. ascending keys with equal keys in ascending input position.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

KT_U32, KT_U64, KT_F32 = 0, 1, 2
_KT = {np.dtype(np.uint32): KT_U32, np.dtype(np.uint64): KT_U64, np.dtype(np.float32): KT_F32}

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (no HIP headers)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp, u64, i32, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32
        L.oracle_ord_f32.restype = u32
        L.oracle_ord_f32.argtypes = [u32]
        L.oracle_sort.restype = i32
        L.oracle_sort.argtypes = [i32, vp, u64, vp, vp, vp, vp]
        L.oracle_sort_mt.restype = i32
        L.oracle_sort_mt.argtypes = [i32, vp, u64, vp, vp, vp, vp, i32]
        L.oracle_segmented.restype = i32
        L.oracle_segmented.argtypes = [i32, vp, vp, vp, u64, vp, vp, vp]
        L.oracle_classify.restype = i32
        L.oracle_classify.argtypes = [i32, vp, vp, u64, vp, vp, u64, vp]
        L.oracle_rank.restype = u64
        L.oracle_rank.argtypes = [i32, vp, u64, u64]
        L.oracle_median_tree.restype = i32
        L.oracle_median_tree.argtypes = [vp, vp, u32, u32, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def kt_of(keys: np.ndarray) -> int:
    return _KT[keys.dtype]


def ord_f32(bits: int) -> int:
    return int(lib().oracle_ord_f32(bits))


def sort(keys: np.ndarray, payload: np.ndarray | None = None, threads: int = 1):
    """Returns (keys_out, perm_out, payload_out or None)."""
    keys = np.ascontiguousarray(keys)
    n = keys.size
    ko = np.empty_like(keys)
    po = np.empty(n, dtype=np.uint32)
    pl = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32)
    plo = None if pl is None else np.empty(n, dtype=np.uint32)
    if threads <= 1:
        rc = lib().oracle_sort(kt_of(keys), _ptr(keys), n, _ptr(pl), _ptr(ko), _ptr(po), _ptr(plo))
    else:
        rc = lib().oracle_sort_mt(kt_of(keys), _ptr(keys), n, _ptr(pl), _ptr(ko), _ptr(po),
                                  _ptr(plo), threads)
    if rc != 0:
        raise ValueError("oracle_sort rejected its arguments")
    return ko, po, plo


def rank(keys: np.ndarray, i: int) -> int:
    """Rank of element i (its output position) straight from the definition, O(n)."""
    keys = np.ascontiguousarray(keys)
    return int(lib().oracle_rank(kt_of(keys), _ptr(keys), keys.size, i))


def segmented(keys: np.ndarray, offsets: np.ndarray, payload: np.ndarray | None = None):
    """Per-segment sort with segment-local perm; returns (keys_out, perm_out, payload_out)."""
    keys = np.ascontiguousarray(keys)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = keys.size
    ko = np.empty_like(keys)
    po = np.empty(n, dtype=np.uint32)
    pl = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32)
    plo = None if pl is None else np.empty(n, dtype=np.uint32)
    rc = lib().oracle_segmented(kt_of(keys), _ptr(keys), _ptr(pl), _ptr(offsets), offsets.size - 1,
                                _ptr(ko), _ptr(po), _ptr(plo))
    if rc != 0:
        raise ValueError("oracle_segmented rejected its arguments")
    return ko, po, plo


def classify(keys: np.ndarray, pos: np.ndarray | None, skeys: np.ndarray, spos: np.ndarray):
    """bucket[i] = #{splitters strictly below (key_i, pos_i)} (positional tie-break)."""
    keys = np.ascontiguousarray(keys)
    skeys = np.ascontiguousarray(skeys, dtype=keys.dtype)
    spos = np.ascontiguousarray(spos, dtype=np.uint32)
    p = None if pos is None else np.ascontiguousarray(pos, dtype=np.uint32)
    out = np.empty(keys.size, dtype=np.uint32)
    rc = lib().oracle_classify(kt_of(keys), _ptr(keys), _ptr(p), keys.size, _ptr(skeys), _ptr(spos),
                               skeys.size, _ptr(out))
    if rc != 0:
        raise ValueError("oracle_classify rejected its arguments")
    return out


def median_tree(vals: np.ndarray, leaf_off: np.ndarray, log2_p: int, k: int, coins: np.ndarray):
    """Binary-tree approximate median; returns (value, side) with side -1/0/+1 for
    -inf / real / +inf."""
    vals = np.ascontiguousarray(vals, dtype=np.uint64)
    leaf_off = np.ascontiguousarray(leaf_off, dtype=np.uint64)
    coins = np.ascontiguousarray(coins, dtype=np.uint8)
    assert leaf_off.size == (1 << log2_p) + 1 and coins.size >= (1 << log2_p) + 1
    res = ctypes.c_uint64()
    side = ctypes.c_int32()
    rc = lib().oracle_median_tree(_ptr(vals), _ptr(leaf_off), log2_p, k, _ptr(coins),
                                  ctypes.byref(res), ctypes.byref(side))
    if rc != 0:
        raise ValueError("oracle_median_tree rejected its arguments")
    return int(res.value), int(side.value)
