"""ctypes binding of libsymtensor.so (the C ABI of include/symtensor.h).

Argument marshalling only: every step of the contraction runs in the HIP
library.  Importing this module on a machine without the built library raises
immediately -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsymtensor.so")

SYMT_MAX_FACTORS = 4
SYMT_MAX_ORDER = 12

SYMT_OK = 0
SYMT_EINVAL = -1
SYMT_EEINSUM = -2
SYMT_ESYM = -3
SYMT_EDTYPE = -4
SYMT_EWORKSPACE = -5
SYMT_EALIAS = -6
SYMT_EUNSUPPORTED = -7
SYMT_EHIP = -8

SYMT_F64 = 0
SYMT_F32 = 1
SYMT_C128 = 2
SYMT_C64 = 3
COMPUTE = {"f64": 0, "f32": 1, "bf16x3": 2}
SYMT_FLAG_STEPS = 0x100

EXPORTED = (
    "symtensor_create", "symtensor_destroy", "symtensor_plan", "symtensor_workspace_size",
    "symtensor_contract", "symtensor_align", "symtensor_unalign", "symtensor_sector_gemm",
    "symtensor_sector_gemm_workspace_size", "symtensor_set_timing", "symtensor_read_timing",
    "symtensor_status_string", "symtensor_last_error", "symtensor_contract_static",
)
SYMT_STATIC_WORKSPACE_BYTES = 128 << 20


class SymtGroup(ctypes.Structure):
    _fields_ = [("nfactors", c_int32), ("order", c_int32 * SYMT_MAX_FACTORS)]


class SymtTensor(ctypes.Structure):
    _fields_ = [("nmodes", c_int32), ("signs", c_char_p), ("charge", c_int32),
                ("dims", POINTER(c_int64)), ("dtype", c_int32), ("data", c_void_p),
                ("mode_charges", POINTER(c_int32)), ("sectors", POINTER(c_int32))]


class SymtPlanInfo(ctypes.Structure):
    _fields_ = [("s", c_int32), ("t", c_int32), ("v", c_int32), ("sigma", c_int32),
                ("group_size", c_int32), ("m", c_int64), ("k", c_int64), ("n", c_int64),
                ("elems_u", c_int64), ("elems_v", c_int64), ("elems_w", c_int64),
                ("flops", c_double), ("bytes_u_al", c_size_t), ("bytes_v_al", c_size_t),
                ("bytes_w_al", c_size_t), ("workspace_bytes", c_size_t),
                ("w_signs", c_char * (SYMT_MAX_ORDER + 1)), ("w_charge", c_int32), ("fused", c_int32),
                ("fused_v", c_int32), ("fused_w", c_int32)]


class SymtError(RuntimeError):
    def __init__(self, code, detail):
        self.code = code
        super().__init__(f"{status_string(code)} ({code}): {detail}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with `python paper_2007_08056_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    p_tensor = POINTER(SymtTensor)
    p_group = POINTER(SymtGroup)
    lib.symtensor_create.argtypes = [POINTER(c_void_p), c_int]
    lib.symtensor_destroy.argtypes = [c_void_p]
    lib.symtensor_plan.argtypes = [c_char_p, p_group, p_tensor, p_tensor, p_tensor, c_int32,
                                   POINTER(SymtPlanInfo)]
    lib.symtensor_workspace_size.argtypes = [c_char_p, p_group, p_tensor, p_tensor, p_tensor,
                                             c_int32, POINTER(c_size_t)]
    lib.symtensor_contract.argtypes = [c_void_p, c_char_p, p_group, p_tensor, p_tensor, p_tensor,
                                       c_int32, c_void_p, c_size_t, c_void_p]
    lib.symtensor_contract_static.argtypes = [c_void_p, c_char_p, p_group, p_tensor, p_tensor, p_tensor,
                                              c_int32, c_void_p]
    lib.symtensor_align.argtypes = [c_void_p, c_char_p, p_group, p_tensor, p_tensor, p_tensor,
                                    c_int32, c_int32, c_void_p, c_size_t, c_void_p]
    lib.symtensor_unalign.argtypes = [c_void_p, c_char_p, p_group, p_tensor, p_tensor, p_tensor,
                                      c_int32, c_void_p, c_void_p]
    lib.symtensor_sector_gemm.argtypes = [c_void_p, c_int32, c_int64, c_int64, c_int64, c_int64,
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    lib.symtensor_sector_gemm_workspace_size.argtypes = [c_int32, c_int64, c_int64, c_int64, c_int64,
                                                         POINTER(c_size_t)]
    lib.symtensor_set_timing.argtypes = [c_void_p, c_int32]
    lib.symtensor_read_timing.argtypes = [c_void_p, POINTER(c_double), POINTER(c_int64)]
    lib.symtensor_status_string.argtypes = [c_int]
    lib.symtensor_status_string.restype = c_char_p
    lib.symtensor_last_error.argtypes = [c_void_p]
    lib.symtensor_last_error.restype = c_char_p
    for name in EXPORTED:
        if name not in ("symtensor_status_string", "symtensor_last_error"):
            getattr(lib, name).restype = c_int
    return lib


LIB = _load()


def status_string(code: int) -> str:
    return LIB.symtensor_status_string(code).decode()


def last_error(ctx=None) -> str:
    return LIB.symtensor_last_error(ctx).decode()


def check(code: int, ctx=None):
    if code != SYMT_OK:
        raise SymtError(code, last_error(ctx))


def make_group(orders) -> SymtGroup:
    orders = tuple(int(o) for o in (orders if isinstance(orders, (tuple, list)) else (orders,)))
    g = SymtGroup()
    g.nfactors = len(orders)
    for i, o in enumerate(orders):
        g.order[i] = o
    return g


class TensorDesc:
    """Keeps a SymtTensor and the buffers it points to alive together."""

    def __init__(self, signs: str, charge: int, dims, dtype: int, data_ptr: int | None, mode_charges=None,
                 sectors=None):
        self._signs = signs.encode()
        self._dims = (c_int64 * max(1, len(dims)))(*[int(d) for d in dims])
        self._charges = None
        if mode_charges is not None:
            flat = [int(x) for row in mode_charges for x in row]
            self._charges = (c_int32 * len(flat))(*flat)
        self._sectors = None
        if sectors is not None:
            self._sectors = (c_int32 * len(sectors))(*[int(h) for h in sectors])
        self.c = SymtTensor(len(signs), self._signs, int(charge), self._dims, int(dtype),
                            c_void_p(data_ptr) if data_ptr else None, self._charges, self._sectors)

    def set_data(self, data_ptr: int | None):
        self.c.data = c_void_p(data_ptr) if data_ptr else None

    @property
    def ref(self):
        return ctypes.byref(self.c)


_CTX = {}


def context(device: int):
    ctx = _CTX.get(device)
    if ctx is None:
        h = c_void_p()
        check(LIB.symtensor_create(ctypes.byref(h), int(device)))
        ctx = h
        _CTX[device] = ctx
    return ctx


def plan(einsum: str, group: SymtGroup, u: TensorDesc, v: TensorDesc, w: TensorDesc | None,
         compute: int) -> SymtPlanInfo:
    info = SymtPlanInfo()
    check(LIB.symtensor_plan(einsum.encode(), ctypes.byref(group), u.ref, v.ref,
                             w.ref if w is not None else None, int(compute), ctypes.byref(info)))
    return info
