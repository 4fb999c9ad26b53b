"""rsort: robust multilevel sample sort for AMD MI355X (gfx950).

The sorting work runs in the HIP kernels of librsort.so (C ABI in
include/rsort.h); ``rsort`` is its Python binding.
"""
from . import rsort  # noqa: F401
