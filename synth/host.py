"""Host-side fast path of the seeded generator (``synth/csrc/philox_host.c``).

Bit-identical to ``synth.philox.values_at`` (a CPU test checks it on both
value maps), but computed in C over all host threads, so that whole blocks of
a large operand, or thousands of sampled rows of it, are generated in seconds
rather than minutes.  It holds no arithmetic of the contraction method.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphilox_host.so")
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with `python paper_2007_08056_amd/build.py`")
        lib = ctypes.CDLL(LIB_PATH)
        lib.synth_host_values.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_int, ctypes.c_double, ctypes.c_void_p]
        lib.synth_host_values.restype = ctypes.c_int
        lib.synth_host_fill.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.c_int, ctypes.c_double]
        lib.synth_host_fill.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def available() -> bool:
    return os.path.exists(LIB_PATH)


def values_at(e, seed: int, tensor_id: int, dist: int, scale: float = 1.0) -> np.ndarray:
    """Binary64 values of elements ``e`` (any int array shape), as synth.philox.values_at."""
    e = np.ascontiguousarray(e, dtype=np.int64)
    out = np.empty(e.shape, dtype=np.float64)
    rc = _lib().synth_host_values(e.ctypes.data, e.size, int(seed) & 0xFFFFFFFF, int(tensor_id) & 0xFFFFFFFF,
                                  int(dist), float(scale), out.ctypes.data)
    if rc:
        raise ValueError(f"unknown distribution {dist}")
    return out


def fill(shape, seed: int, tensor_id: int, dist: int, scale: float = 1.0, first: int = 0,
         out: np.ndarray | None = None) -> np.ndarray:
    """A C-ordered binary64 array whose element i is the value of element first + i."""
    shape = tuple(int(s) for s in shape)
    if out is None:
        out = np.empty(shape, dtype=np.float64)
    if out.dtype != np.float64 or not out.flags.c_contiguous or out.shape != shape:
        raise ValueError("fill: out must be a C-contiguous float64 array of the given shape")
    rc = _lib().synth_host_fill(out.ctypes.data, out.size, int(first), int(seed) & 0xFFFFFFFF,
                                int(tensor_id) & 0xFFFFFFFF, int(dist), float(scale))
    if rc:
        raise ValueError(f"unknown distribution {dist}")
    return out
