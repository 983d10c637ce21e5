"""Device-side fill of the seeded synthetic inputs (bit-identical to synth.philox)."""
from __future__ import annotations

import ctypes
import os

import torch

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynthgen.so")
if not os.path.exists(_PATH):
    raise ImportError(f"{_PATH} is missing; build it with `python paper_2007_08056_amd/build.py`")
_LIB = ctypes.CDLL(_PATH)
_LIB.synth_fill.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32,
                            ctypes.c_uint32, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                            ctypes.c_void_p]
_LIB.synth_fill.restype = ctypes.c_int


def fill_(out: torch.Tensor, seed: int, tensor_id: int, dist: int, scale: float = 1.0, first: int = 0):
    """Overwrite a contiguous float64/float32 device tensor with elements first.. of (seed, tensor_id)."""
    if not (out.is_cuda and out.is_contiguous()) or out.dtype not in (torch.float64, torch.float32):
        raise ValueError("fill_ needs a contiguous float64/float32 device tensor")
    stream = torch.cuda.current_stream(out.device).cuda_stream
    rc = _LIB.synth_fill(ctypes.c_void_p(out.data_ptr()), out.numel(), int(first), int(seed) & 0xFFFFFFFF,
                         int(tensor_id) & 0xFFFFFFFF, int(dist), float(scale),
                         0 if out.dtype == torch.float64 else 1, ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError(f"synth_fill failed with HIP error {rc}")
    return out


def device_input(wl, name: str, dtype=torch.float64, device="cuda:0") -> torch.Tensor:
    """The standard reduced form of input ``name`` of workload ``wl`` on the device."""
    op = wl.operands[name]
    t = torch.empty(wl.reduced_shape(name), dtype=dtype, device=device)
    return fill_(t, wl.seed, op.tensor_id, op.dist, op.scale)
