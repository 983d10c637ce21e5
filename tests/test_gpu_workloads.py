"""The five workloads at their full sizes on the GPU, against the CPU oracle.

Inputs come from the seeded generator on both sides (bit-identical).  Small
workloads are compared element by element with the loop-over-blocks oracle;
the Z_16 ladder, too large for any full oracle, is compared on sampled output
elements computed one by one by the oracle's brute-force sum.
"""
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


@pytest.fixture(scope="module")
def SG():
    import synth.gpu as SG
    return SG


def _inputs(P, SG, wl, dtype=torch.float64):
    out = {}
    for name in wl.inputs:
        op = wl.operands[name]
        out[name] = P.SymTensor(SG.device_input(wl, name, dtype=dtype, device=DEV), op.signs, op.charge,
                                wl.group)
    return out


def _syms(wl):
    return {k: H.sym_of(op, wl.group) for k, op in wl.operands.items()}


def test_plain_z4_full(P, SG):
    wl = synth.configs.plain_z4()
    st = wl.steps[0]
    say(f"workload {wl.name} {st.einsum}")
    t = _inputs(P, SG, wl)
    syms = _syms(wl)
    Ru, Rv = synth.host_input(wl, st.u), synth.host_input(wl, st.v)
    ref, sw, zero_ok = O.contract_dense(st.einsum, Ru, syms[st.u], Rv, syms[st.v])
    refb, _ = O.contract_blocks(st.einsum, Ru, syms[st.u], Rv, syms[st.v])
    assert zero_ok
    for compute in ("f64", "f32", "bf16x3"):
        w = P.output_like(st.einsum, t[st.u], t[st.v])
        P.contract_into(st.einsum, t[st.u], t[st.v], w, compute)
        got = H.to_np(w.data)
        absref, _ = O.contract_blocks(st.einsum, np.abs(Ru), syms[st.u], np.abs(Rv), syms[st.v])
        k = H.contracted_extent(st.einsum, syms[st.u])
        assert np.all(np.abs(got - refb) <= H.bound_factor(compute, k) * absref), compute
        if compute == "f64":
            assert H.rel_err(got, ref) <= 1e-12 and H.rel_err(got, refb) <= 1e-12
            assert np.array_equal(O.expand(got, sw) == 0, O.expand(ref, sw) == 0)


@pytest.mark.timeout(600)
def test_ccd_ladder_z8_full(P, SG):
    wl = synth.configs.ccd_ladder_z8()
    st = wl.steps[0]
    say(f"workload {wl.name} {st.einsum} full, loop-over-blocks oracle")
    t = _inputs(P, SG, wl)
    syms = _syms(wl)
    w = P.output_like(st.einsum, t[st.u], t[st.v])
    P.contract_into(st.einsum, t[st.u], t[st.v], w, "f64")
    got = H.to_np(w.data)
    Ru, Rv = synth.host_input(wl, st.u), synth.host_input(wl, st.v)
    ref, sw = O.contract_blocks(st.einsum, Ru, syms[st.u], Rv, syms[st.v])
    absref, _ = O.contract_blocks(st.einsum, np.abs(Ru), syms[st.u], np.abs(Rv), syms[st.v])
    err = H.rel_err(got, ref)
    say(f"  f64 normwise relative error {err:.3e}")
    assert err <= 1e-12
    k = H.contracted_extent(st.einsum, syms[st.u])
    assert np.all(np.abs(got - ref) <= H.bound_factor("f64", k) * absref)
    assert w.signs == sw.sign_string() and w.charge == sw.charge


@pytest.mark.timeout(600)
def test_mps_env_z2z3_chain_full(P, SG):
    wl = synth.configs.mps_env_z2z3()
    say(f"workload {wl.name} three-step chain")
    syms = _syms(wl)
    host = {k: synth.host_input(wl, k) for k in wl.inputs}
    absh = {k: np.abs(v) for k, v in host.items()}
    for st in wl.steps:                      # the binary64 oracle chain, and |.| bounds
        host[st.w], sw = O.contract_blocks(st.einsum, host[st.u], syms[st.u], host[st.v], syms[st.v])
        absh[st.w], _ = O.contract_blocks(st.einsum, absh[st.u], syms[st.u], absh[st.v], syms[st.v])
        assert O.same_symmetry(sw, syms[st.w])
    tol = {"f64": 1e-12, "f32": 2e-5, "bf16x3": 5e-4}
    for compute in ("f64", "f32", "bf16x3"):
        dev = _inputs(P, SG, wl)
        for st in wl.steps:
            out = P.output_like(st.einsum, dev[st.u], dev[st.v])
            P.contract_into(st.einsum, dev[st.u], dev[st.v], out, compute)
            dev[st.w] = out
            err = H.rel_err(H.to_np(out.data), host[st.w])
            say(f"  {compute} {st.einsum}: normwise relative error {err:.3e}")
            assert err <= tol[compute]
            if compute == "f64":
                assert np.array_equal(O.expand(H.to_np(out.data), syms[st.w]) == 0,
                                      O.expand(host[st.w], syms[st.w]) == 0)


@pytest.mark.parametrize("compute", ["f64", "f32", "bf16x3"])
@pytest.mark.timeout(600)
def test_ccd_ladder_z16_full_sampled(P, SG, compute):
    """Z_16, virtual 32, occupied 8: 8.8 TFLOP of allowed-block products, sampled outputs."""
    wl = synth.configs.ccd_ladder_z16()
    st = wl.steps[0]
    say(f"workload {wl.name} {compute}: generating inputs")
    syms = _syms(wl)
    dt = torch.float64 if compute == "f64" else torch.float32
    t = _inputs(P, SG, wl, dtype=dt)
    w = P.output_like(st.einsum, t[st.u], t[st.v], dtype=torch.float64)
    say(f"workload {wl.name} {compute}: contracting")
    P.contract_into(st.einsum, t[st.u], t[st.v], w, compute)
    torch.cuda.synchronize()
    del t
    torch.cuda.empty_cache()
    rng = np.random.default_rng(16)
    sw = syms[st.w]
    red, full = H.random_w_positions(sw, 96, rng)
    got = np.array([w.data[r].item() for r in red])
    fu, fv = H.value_fn(wl, st.u), H.value_fn(wl, st.v)
    if compute != "f64":
        fu, fv = H.f32_value_fn(fu), H.f32_value_fn(fv)
    say(f"workload {wl.name} {compute}: oracle on {len(red)} sampled outputs")
    ref = O.sample_contract(st.einsum, syms[st.u], syms[st.v], fu, fv, full)
    absref = O.sample_contract(st.einsum, syms[st.u], syms[st.v], H.value_fn(wl, st.u, True),
                               H.value_fn(wl, st.v, True), full)
    k = H.contracted_extent(st.einsum, syms[st.u])
    err = H.rel_err(got, ref)
    say(f"  {compute}: normwise relative error on samples {err:.3e} (vs the oracle on the same "
        f"{'binary32-rounded ' if compute != 'f64' else ''}inputs)")
    assert np.all(np.abs(got - ref) <= H.bound_factor(compute, k) * absref)
    if compute == "f64":
        assert err <= 1e-12
    else:
        # against the binary64 inputs as well: adds the input rounding
        ref64 = O.sample_contract(st.einsum, syms[st.u], syms[st.v], H.value_fn(wl, st.u),
                                  H.value_fn(wl, st.v), full)
        err64 = H.rel_err(got, ref64)
        say(f"  {compute}: normwise relative error vs FP64 oracle {err64:.3e}")
        assert np.all(np.abs(got - ref64) <= (H.bound_factor(compute, k) + 2.1 * H.U32) * absref)
