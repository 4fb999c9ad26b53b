"""Seeded synthetic inputs (numpy arrays) from the C generators in ``gen.c``.

Both the CPU oracle and the GPU library are fed from these arrays; this module
contains no sorting arithmetic.  Distribution names follow the instances of
the paper's experimental section (Uniform, Gaussian, DeterDupl, Zero, Reverse).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgen.so")

KT_U32, KT_U64, KT_F32 = 0, 1, 2
KEY_DTYPES = {KT_U32: np.uint32, KT_U64: np.uint64, KT_F32: np.float32}
KT_BY_NAME = {"u32": KT_U32, "u64": KT_U64, "f32": KT_F32}

DISTS = {
    "uniform": 0,
    "gaussian": 1,
    "zero": 2,
    "deterdupl": 3,
    "reverse": 4,
    "sorted": 5,
    "topbits": 6,
    "widedup": 7,
}

_lib = None


def build(force: bool = True) -> str:
    """Compile libgen.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u64, i32, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        L.gen_splitmix64.restype = u64
        L.gen_splitmix64.argtypes = [u64, u64]
        L.gen_keys.restype = i32
        L.gen_keys.argtypes = [i32, i32, u64, u64, u64, u64, vp]
        L.gen_payload.restype = i32
        L.gen_payload.argtypes = [u64, u64, u64, vp]
        L.gen_log_uniform_sizes.restype = i32
        L.gen_log_uniform_sizes.argtypes = [u64, u64, ctypes.c_double, ctypes.c_double, vp]
        L.gen_segmented.restype = i32
        L.gen_segmented.argtypes = [i32, u64, u64, vp, vp, u64, vp, vp]
        _lib = L
    return _lib


def _kt(kt):
    return KT_BY_NAME[kt] if isinstance(kt, str) else int(kt)


def splitmix64(seed: int, i: int) -> int:
    return int(lib().gen_splitmix64(seed, i))


def keys(kt, dist: str, n: int, seed: int = 1, stream_off: int = 0, param: int = 0,
         out: np.ndarray | None = None) -> np.ndarray:
    """n keys of type kt ('u32' | 'u64' | 'f32') from distribution ``dist``."""
    kt = _kt(kt)
    if out is None:
        out = np.empty(n, dtype=KEY_DTYPES[kt])
    assert out.dtype == KEY_DTYPES[kt] and out.size == n and out.flags.c_contiguous
    rc = lib().gen_keys(kt, DISTS[dist], param, seed, n, stream_off, out.ctypes.data)
    if rc != 0:
        raise ValueError("gen_keys failed")
    return out


def payload(n: int, seed: int = 2, stream_off: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    lib().gen_payload(seed, n, stream_off, out.ctypes.data)
    return out


def log_uniform_sizes(count: int, lo_log2: float, hi_log2: float, seed: int = 1) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    lib().gen_log_uniform_sizes(seed, count, lo_log2, hi_log2, out.ctypes.data)
    return out


def segmented(kt, sizes: np.ndarray, dists, seed: int = 1, with_payload: bool = True):
    """Concatenated segments; returns (keys, payload or None, offsets[count+1])."""
    kt = _kt(kt)
    sizes = np.asarray(sizes, dtype=np.uint64)
    count = sizes.size
    offsets = np.zeros(count + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offsets[1:])
    total = int(offsets[-1])
    dist_codes = np.array([DISTS[d] if isinstance(d, str) else int(d) for d in dists], dtype=np.int32)
    assert dist_codes.size == count
    k = np.empty(total, dtype=KEY_DTYPES[kt])
    p = np.empty(total, dtype=np.uint32) if with_payload else None
    rc = lib().gen_segmented(kt, seed, count, offsets.ctypes.data, dist_codes.ctypes.data, 0,
                             k.ctypes.data, p.ctypes.data if p is not None else None)
    if rc != 0:
        raise ValueError("gen_segmented failed")
    return k, p, offsets


def pick_dists(count: int, choices, seed: int = 7):
    """Distribution name per item, uniform over ``choices`` from the stream."""
    return [choices[splitmix64(seed, s) % len(choices)] for s in range(count)]
