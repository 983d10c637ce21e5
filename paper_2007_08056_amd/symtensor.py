"""Python front end: symmetric tensors on torch device memory and the contraction.

``SymTensor`` pairs a standard reduced form (a torch tensor of shape
[|G|]*(N-1) + [n_0, ..., n_{N-1}], the layout of the paper's API example,
Sec. 3) with its symmetry label (sign string, total charge, group).
``einsum(subscripts, u, v)`` contracts two of them through the HIP library:
align both operands, one sector-batched product, unalign the result
(Alg. 2).  It is differentiable: the backward pass is two more contractions
of the same kind (dU = dW . V over the J modes, dV = U . dW over the I
modes), whose aligned operands are recomputed from the saved standard forms
rather than stored.

PyTorch supplies device memory and the current HIP stream; no arithmetic of
the method happens in Python.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

from . import _lib as L

_DTYPE_CODE = {torch.float64: L.SYMT_F64, torch.float32: L.SYMT_F32,
               torch.complex128: L.SYMT_C128, torch.complex64: L.SYMT_C64}


def _group_tuple(group):
    return tuple(int(o) for o in (group if isinstance(group, (tuple, list)) else (group,)))


def group_size(group) -> int:
    g = 1
    for o in _group_tuple(group):
        g *= o
    return g


def _norm_charges(tables, n, G):
    """Charge tables as a tuple of n rows of G ints, or None for all-identity."""
    if tables is None:
        return None
    rows = tuple(tuple(int(x) for x in row) for row in tables)
    if len(rows) != n or any(len(r) != G for r in rows):
        raise ValueError(f"charge tables must be {n} rows of {G} entries")
    return None if all(r == tuple(range(G)) for r in rows) else rows


@dataclass
class SymTensor:
    """A tensor with cyclic (or product-of-cyclic) group symmetry, stored reduced.

    ``mode_charges`` optionally gives, per mode, the charge carried by each
    sector label (a permutation of the group elements); None: every label is
    its own charge (include/symtensor.h, symt_tensor).  ``sectors``
    optionally gives each mode's number of sectors H_m, a divisor of |G|
    (coefficient sign |G|/H_m); None: |G| each.
    """
    data: torch.Tensor
    signs: str
    charge: int
    group: tuple
    mode_charges: tuple | None = None
    sectors: tuple | None = None

    def __post_init__(self):
        self.group = _group_tuple(self.group)
        n = len(self.signs)
        G = group_size(self.group)
        if self.sectors is not None:
            self.sectors = tuple(int(h) for h in self.sectors)
            if len(self.sectors) != n:
                raise ValueError(f"sectors must hold {n} counts")
            if all(h == G for h in self.sectors):
                self.sectors = None
        hs = self.sectors or (G,) * n
        if self.data.dim() != 2 * n - 1 or tuple(int(s) for s in self.data.shape[: n - 1]) != hs[: n - 1]:
            raise ValueError(f"reduced form must have shape {list(hs[: n - 1])} + dims, got {tuple(self.data.shape)}")
        if self.data.dtype not in _DTYPE_CODE:
            raise TypeError("reduced form must be float64, float32, complex128 or complex64")
        self.charge = int(self.charge) % G
        self.mode_charges = _norm_charges(self.mode_charges, n, G)

    @property
    def dims(self):
        n = len(self.signs)
        return tuple(int(d) for d in self.data.shape[n - 1:])

    @property
    def order(self):
        return len(self.signs)

    def desc(self, data=None) -> L.TensorDesc:
        d = self.data if data is None else data
        return L.TensorDesc(self.signs, self.charge, self.dims, _DTYPE_CODE[d.dtype],
                            d.data_ptr() if d.numel() else None, self.mode_charges, self.sectors)

    def key(self):
        """Every descriptor field but the data pointer (a planning cache key)."""
        return (self.signs, self.charge, self.dims, self.data.dtype, self.mode_charges, self.sectors)

    def table(self, m):
        G = group_size(self.group)
        return tuple(range(G)) if self.mode_charges is None else self.mode_charges[m]


def _check_dense(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("operand data must live on a HIP device")
    if not t.is_contiguous():
        raise ValueError("operand data must be contiguous")


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _code(compute: str, steps: bool) -> int:
    return L.COMPUTE[compute] | (L.SYMT_FLAG_STEPS if steps else 0)


# Planned contractions: key -> (group, descriptors of u, v, w, plan info).  The
# descriptors are reused with their data pointers replaced on every call, so a
# contraction is planned once per key here (and once per key in the library's
# context, which caches its own plans).
_PLANS: dict = {}
_MAX_PLANS = 1024


# Tuning variables the library's planner reads (include/symtensor.h): part of every key.
_TUNING_VARS = ("SYMT_FUSED_V", "SYMT_GEMM_TILE", "SYMT_GEMM_SK")


def _planned(subscripts, u, v, w, code):
    key = (subscripts, u.group, u.key(), v.key(), w.key() if w is not None else None, code,
           tuple(os.environ.get(k) for k in _TUNING_VARS))
    ent = _PLANS.get(key)
    if ent is None:
        if u.group != v.group:
            raise ValueError("operands use different groups")
        g = L.make_group(u.group)
        du, dv = u.desc(), v.desc()
        dw = w.desc() if w is not None else None
        info = L.plan(subscripts, g, du, dv, dw, code)
        if len(_PLANS) >= _MAX_PLANS:
            _PLANS.clear()
        ent = _PLANS[key] = (g, du, dv, dw, info)
    return ent


def plan(subscripts: str, u: SymTensor, v: SymTensor, compute: str = "f64", w: SymTensor | None = None,
         steps: bool = False):
    """Shapes, flops, workspace and derived output rule of a contraction (host only)."""
    return _planned(subscripts, u, v, w, _code(compute, steps))[4]


def derived_charges(subscripts: str, u: SymTensor, v: SymTensor):
    """Charge tables of the output: u's rows on its kept modes, v's on its kept modes."""
    if u.mode_charges is None and v.mode_charges is None:
        return None
    tu, rest = subscripts.split(",")
    tv, tw = rest.split("->")
    return tuple(u.table(tu.index(m)) if m in tu else v.table(tv.index(m)) for m in tw)


def derived_sectors(subscripts: str, u: SymTensor, v: SymTensor):
    """Sector counts of the output: u's on its kept modes, v's on its kept modes."""
    if u.sectors is None and v.sectors is None:
        return None
    G = group_size(u.group)
    tu, rest = subscripts.split(",")
    tv, tw = rest.split("->")
    hu, hv = u.sectors or (G,) * len(tu), v.sectors or (G,) * len(tv)
    return tuple(hu[tu.index(m)] if m in tu else hv[tv.index(m)] for m in tw)


def output_like(subscripts: str, u: SymTensor, v: SymTensor, dtype=None) -> SymTensor:
    """A zero-filled output with the derived sign string, charge, charge tables and sector counts."""
    info = plan(subscripts, u, v)
    tu, rest = subscripts.split(",")
    tv, tw = rest.split("->")
    dims = []
    for m in tw:
        dims.append(u.dims[tu.index(m)] if m in tu else v.dims[tv.index(m)])
    G = group_size(u.group)
    hs = derived_sectors(subscripts, u, v) or (G,) * len(tw)
    shape = list(hs[: len(tw) - 1]) + dims
    dtype = dtype or u.data.dtype
    data = torch.zeros(shape, dtype=dtype, device=u.data.device)
    return SymTensor(data, info.w_signs.decode(), info.w_charge, u.group, derived_charges(subscripts, u, v),
                     derived_sectors(subscripts, u, v))


def contract_into(subscripts: str, u: SymTensor, v: SymTensor, w: SymTensor, compute: str = "f64",
                  workspace: torch.Tensor | None = None, steps: bool = False):
    """w.data <- contraction of u and v (no autograd); returns w.

    ``steps=True`` runs the three separate steps even where the fused product
    applies (include/symtensor.h, FUSED PRODUCT).
    """
    for t in (u.data, v.data, w.data):
        _check_dense(t)
    dev = u.data.device
    code = _code(compute, steps)
    g, du, dv, dw, info = _planned(subscripts, u, v, w, code)
    for d, t in ((du, u.data), (dv, v.data), (dw, w.data)):
        d.set_data(t.data_ptr() if t.numel() else None)
    if workspace is None or workspace.numel() < info.workspace_bytes:
        workspace = torch.empty(max(1, info.workspace_bytes), dtype=torch.uint8, device=dev)
    ctx = L.context(dev.index or 0)
    L.check(L.LIB.symtensor_contract(ctx, subscripts.encode(), ctypes.byref(g), du.ref, dv.ref,
                                     dw.ref, code, ctypes.c_void_p(workspace.data_ptr()),
                                     workspace.numel(), ctypes.c_void_p(_stream(dev))), ctx)
    return w


def _swap(subscripts):
    tu, rest = subscripts.split(",")
    tv, tw = rest.split("->")
    return tu, tv, tw


class _Contract(torch.autograd.Function):
    @staticmethod
    def forward(ctx, subscripts, meta_u, meta_v, meta_w, compute, ud, vd):
        u = SymTensor(ud, *meta_u)
        v = SymTensor(vd, *meta_v)
        w = SymTensor(torch.empty(meta_w[5], dtype=ud.dtype, device=ud.device), *meta_w[:5])
        contract_into(subscripts, u, v, w, compute)
        ctx.save_for_backward(ud, vd)
        ctx.meta = (subscripts, meta_u, meta_v, meta_w, compute)
        return w.data

    @staticmethod
    def backward(ctx, gw):
        subscripts, meta_u, meta_v, meta_w, compute = ctx.meta
        ud, vd = ctx.saved_tensors
        tu, tv, tw = _swap(subscripts)
        dW = SymTensor(gw.contiguous().to(ud.dtype), *meta_w[:5])
        # complex operands: gradients with respect to the conjugate (Wirtinger),
        # so the other factor enters conjugated
        conj = (lambda t: t.conj().resolve_conj()) if ud.is_complex() else (lambda t: t)
        gu = gv = None
        if ctx.needs_input_grad[5]:
            # dU[I,K] = sum_J dW[I,J] V[K,J]; the derived rule of (dW, V) is U's.
            out = SymTensor(torch.empty_like(ud), *meta_u)
            contract_into(f"{tw},{tv}->{tu}", dW, SymTensor(conj(vd), *meta_v), out, compute)
            gu = out.data
        if ctx.needs_input_grad[6]:
            # dV[K,J] = sum_I U[I,K] dW[I,J]; the derived rule of (U, dW) is V's up to a global sign.
            out = SymTensor(torch.empty_like(vd), *meta_v)
            contract_into(f"{tu},{tw}->{tv}", SymTensor(conj(ud), *meta_u), dW, out, compute)
            gv = out.data
        return None, None, None, None, None, gu, gv


def einsum(subscripts: str, u: SymTensor, v: SymTensor, compute: str = "f64") -> SymTensor:
    """W = contraction of u and v (Eq. ctr), differentiable with respect to u.data and v.data."""
    if u.group != v.group:
        raise ValueError("operands use different groups")
    if compute not in L.COMPUTE:
        raise ValueError(f"compute must be one of {list(L.COMPUTE)}")
    info = plan(subscripts, u, v, compute)
    tu, tv, tw = _swap(subscripts)
    dims = [u.dims[tu.index(m)] if m in tu else v.dims[tv.index(m)] for m in tw]
    G = group_size(u.group)
    ws = derived_sectors(subscripts, u, v)
    shape = tuple(list((ws or (G,) * len(tw))[: len(tw) - 1]) + dims)
    meta_u = (u.signs, u.charge, u.group, u.mode_charges, u.sectors)
    meta_v = (v.signs, v.charge, v.group, v.mode_charges, v.sectors)
    wc = derived_charges(subscripts, u, v)
    meta_w = (info.w_signs.decode(), info.w_charge, u.group, wc, ws, shape)
    wd = _Contract.apply(subscripts, meta_u, meta_v, meta_w, compute, u.data, v.data)
    return SymTensor(wd, meta_w[0], meta_w[1], u.group, wc, ws)


# ---------------------------------------------------------------------------
# The three steps on their own (tests, profiling)
# ---------------------------------------------------------------------------
def align(subscripts: str, u: SymTensor, v: SymTensor, operand: int, compute: str = "f64",
          out: torch.Tensor | None = None) -> torch.Tensor:
    """Aligned form of u (operand 0) or v (operand 1) in the compute mode's layout.

    f64 / f32: a (|G|, M, K) or (|G|, K, N) tensor.  bf16x3: an int16 tensor of
    raw bf16 bits, (2, |G|, M, K) for u and (2, |G|, N, K) for v (hi plane first).
    Complex operands: the real representation of C (include/symtensor.h,
    COMPLEX OPERANDS), a real tensor with K and N doubled.
    `out`, if given, is a contiguous tensor of that shape and dtype, overwritten.
    """
    dev = u.data.device
    g = L.make_group(u.group)
    du, dv = u.desc(), v.desc()
    info = L.plan(subscripts, g, du, dv, None, L.COMPUTE[compute])
    G, M, K, N = info.group_size, info.m, info.k, info.n
    if compute == "f64":
        shape, dtype = ((G, M, K) if operand == 0 else (G, K, N)), torch.float64
    elif compute == "f32":
        shape, dtype = ((G, M, K) if operand == 0 else (G, K, N)), torch.float32
    else:
        shape, dtype = ((2, G, M, K) if operand == 0 else (2, G, N, K)), torch.int16
    if out is None:
        out = torch.empty(shape, dtype=dtype, device=dev)
    elif tuple(out.shape) != shape or out.dtype != dtype or not out.is_contiguous() or out.device != dev:
        raise ValueError(f"align: out must be a contiguous {dtype} tensor of shape {shape} on {dev}")
    ctx = L.context(dev.index or 0)
    nbytes = out.numel() * out.element_size()
    L.check(L.LIB.symtensor_align(ctx, subscripts.encode(), ctypes.byref(g), du.ref, dv.ref, None,
                                  L.COMPUTE[compute], int(operand),
                                  ctypes.c_void_p(out.data_ptr()) if nbytes else None, nbytes,
                                  ctypes.c_void_p(_stream(dev))), ctx)
    return out


def unalign(subscripts: str, u: SymTensor, v: SymTensor, w: SymTensor, aligned_w: torch.Tensor,
            compute: str = "f64") -> SymTensor:
    dev = u.data.device
    g = L.make_group(u.group)
    ctx = L.context(dev.index or 0)
    du, dv, dw = u.desc(), v.desc(), w.desc()
    L.check(L.LIB.symtensor_unalign(ctx, subscripts.encode(), ctypes.byref(g), du.ref, dv.ref, dw.ref,
                                    L.COMPUTE[compute], ctypes.c_void_p(aligned_w.data_ptr()),
                                    ctypes.c_void_p(_stream(dev))), ctx)
    return w


def sector_gemm_workspace_size(compute: str, batch: int, m: int, k: int, n: int) -> int:
    """Bytes with which sector_gemm may run stream-K on this shape (0: never)."""
    out = ctypes.c_size_t()
    L.check(L.LIB.symtensor_sector_gemm_workspace_size(L.COMPUTE[compute], batch, m, k, n,
                                                       ctypes.byref(out)))
    return out.value


def sector_gemm(a: torch.Tensor, b: torch.Tensor, compute: str = "f64", c: torch.Tensor | None = None,
                workspace: torch.Tensor | None | bool = True):
    """c[q] = a[q] b[q] on the aligned layouts (see include/symtensor.h).

    ``workspace``: a uint8 device tensor, True (allocate what the launch model
    asks for) or None (one workgroup per tile).
    """
    dev = a.device
    if compute == "bf16x3":
        _, batch, m, k = a.shape
        n = b.shape[2]
        cdt = torch.float64
    else:
        batch, m, k = a.shape
        n = b.shape[2]
        cdt = a.dtype
    if c is None:
        c = torch.empty((batch, m, n), dtype=cdt, device=dev)
    if workspace is True:
        need = sector_gemm_workspace_size(compute, batch, m, k, n)
        workspace = torch.empty(need, dtype=torch.uint8, device=dev) if need else None
    ws_ptr = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
    ws_bytes = workspace.numel() if workspace is not None else 0
    ctx = L.context(dev.index or 0)
    L.check(L.LIB.symtensor_sector_gemm(ctx, L.COMPUTE[compute], batch, m, k, n,
                                        ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                        ctypes.c_void_p(c.data_ptr()), ws_ptr, ws_bytes,
                                        ctypes.c_void_p(_stream(dev))), ctx)
    return c


def set_timing(device, enable: bool):
    L.check(L.LIB.symtensor_set_timing(L.context(device), int(bool(enable))))


def read_timing(device):
    """Summed milliseconds and launches per step: align U, align V, product, unalign W."""
    ms = (ctypes.c_double * 4)()
    n = (ctypes.c_int64 * 4)()
    ctx = L.context(device)
    L.check(L.LIB.symtensor_read_timing(ctx, ms, n), ctx)
    return list(ms), list(n)
