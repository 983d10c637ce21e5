"""The allocation-free entry point against symtensor_contract, through the C ABI.

symtensor_contract_static runs the same contraction on the library's own
device array.  Two calls in a row, the second on a smaller input (the array
keeps the first call's contents), are each compared with the workspace entry
point's result on the same inputs and with the oracle; a third call that
needs more workspace than the array holds must fail before any launch.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_08056_amd as P
    return P


def _static(P, sub, u, v, w, compute):
    L = P._lib
    ctx = L.context(0)
    code = L.COMPUTE[compute]
    rc = L.LIB.symtensor_contract_static(ctx, sub.encode(), ctypes.byref(L.make_group(u.group)), u.desc().ref,
                                         v.desc().ref, w.desc().ref, code,
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, L.last_error(ctx)


def _workload_case(P, wl, compute):
    import synth.gpu as SG
    st = wl.steps[0]
    dt = torch.float64 if compute == "f64" else torch.float32
    t = {}
    for name in wl.inputs:
        op = wl.operands[name]
        t[name] = P.SymTensor(SG.device_input(wl, name, dtype=dt, device=DEV), op.signs, op.charge, wl.group)
    return st, t[st.u], t[st.v]


@pytest.mark.parametrize("compute", ["f64", "f32", "bf16x3"])
def test_static_entry_point_matches_contract(P, compute):
    from paper_2007_08056_amd import _lib as L
    for wl in (synth.configs.ccd_ladder_z8(), synth.configs.plain_z4()):      # larger first, then smaller
        st, u, v = _workload_case(P, wl, compute)
        say(f"no-alloc {wl.name} {compute}: symtensor_contract_static, then symtensor_contract")
        # W in the compute type (split-bf16: binary64): the fused path, whose workspace is small
        wdt = torch.float32 if compute == "f32" else torch.float64
        w_static = P.output_like(st.einsum, u, v, dtype=wdt)
        w_static.data.fill_(float("nan"))
        rc, msg = _static(P, st.einsum, u, v, w_static, compute)
        assert rc == 0, msg
        w_ref = P.output_like(st.einsum, u, v, dtype=wdt)
        P.contract_into(st.einsum, u, v, w_ref, compute)
        torch.cuda.synchronize()
        info = P.plan(st.einsum, u, v, compute, w_ref)
        got, ref = H.to_np(w_static.data).astype(np.float64), H.to_np(w_ref.data).astype(np.float64)
        assert not np.isnan(got).any()
        if info.workspace_bytes <= L.SYMT_STATIC_WORKSPACE_BYTES:
            # the same plan on the same inputs: the same sums in the same order
            assert np.array_equal(got, ref), wl.name
        # and against the oracle on the same (rounded) inputs, within the product's bound
        syms = {k: H.sym_of(op, wl.group) for k, op in wl.operands.items()}
        Ru, Rv = synth.host_input(wl, st.u), synth.host_input(wl, st.v)
        if compute != "f64":
            Ru, Rv = Ru.astype(np.float32).astype(np.float64), Rv.astype(np.float32).astype(np.float64)
        oref, _ = O.contract_blocks(st.einsum, Ru, syms[st.u], Rv, syms[st.v])
        absref, _ = O.contract_blocks(st.einsum, np.abs(Ru), syms[st.u], np.abs(Rv), syms[st.v])
        k = H.contracted_extent(st.einsum, syms[st.u])
        assert np.all(np.abs(got - oref) <= H.bound_factor(compute, k) * absref), wl.name
        if compute == "f64":
            assert H.rel_err(got, oref) <= 1e-12
        del u, v, w_static, w_ref
        torch.cuda.empty_cache()


def test_static_entry_point_without_stream_k_pieces(P, monkeypatch):
    """Z_8 ladder with stream-K forced on a tile whose pieces exceed the array: the product runs
    one workgroup per tile and matches the workspace entry point within the f64 bound."""
    from paper_2007_08056_amd import _lib as L
    monkeypatch.setenv("SYMT_GEMM_TILE", "d128x128s2")
    monkeypatch.setenv("SYMT_GEMM_SK", "1")
    wl = synth.configs.ccd_ladder_z8()
    st, u, v = _workload_case(P, wl, "f64")
    info = P.plan(st.einsum, u, v, "f64")
    say(f"no-alloc {wl.name}: workspace {info.workspace_bytes} bytes with stream-K pieces")
    w_static = P.output_like(st.einsum, u, v)
    rc, msg = _static(P, st.einsum, u, v, w_static, "f64")
    assert rc == 0, msg
    w_ref = P.output_like(st.einsum, u, v)
    P.contract_into(st.einsum, u, v, w_ref, "f64")
    torch.cuda.synchronize()
    assert H.rel_err(H.to_np(w_static.data), H.to_np(w_ref.data)) <= 1e-13
    if info.workspace_bytes > L.SYMT_STATIC_WORKSPACE_BYTES:
        say("  pieces did not fit: one workgroup per tile")


def test_static_entry_point_rejects_oversized_workspace(P):
    """Three-step path (forced) on the Z_8 ladder: the aligned forms need ~1.5 GB; SYMT_EWORKSPACE
    and the output untouched."""
    from paper_2007_08056_amd import _lib as L
    wl = synth.configs.ccd_ladder_z8()
    st, u, v = _workload_case(P, wl, "f64")
    w = P.output_like(st.einsum, u, v)
    w.data.fill_(5.0)
    ctx = L.context(0)
    rc = L.LIB.symtensor_contract_static(ctx, st.einsum.encode(), ctypes.byref(L.make_group(u.group)),
                                         u.desc().ref, v.desc().ref, w.desc().ref,
                                         L.COMPUTE["f64"] | L.SYMT_FLAG_STEPS, None)
    assert rc == L.SYMT_EWORKSPACE, L.last_error(ctx)
    torch.cuda.synchronize()
    assert bool((w.data == 5.0).all())
