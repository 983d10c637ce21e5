"""Hand-written backward of the contraction, on the differentiated MPS environment chain.

L = <E', R> with E' = ((E A) W) A contracted left to right; gradients with
respect to A (used twice), W and E come from the library's backward (two more
symmetric contractions per step, aligned forms recomputed).  Checked against
* dense torch autograd on the CPU in binary64 (zero blocks materialised), every
  entry, on a chain with the bond block shrunk to 4; the dense gradient must be
  exactly zero off the conservation rule;
* central finite differences of the binary64 oracle forward (h = 1e-6) along
  seeded random directions, at the full bond block of 128.  L is linear in E
  and W and quadratic in A, so the central difference has no truncation error.
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
PARAMS = ("E", "A", "W")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_08056_amd as P
    return P


def _gpu_loss_and_grads(P, wl, host, compute, dtype):
    ts = {}
    for k in PARAMS:
        op = wl.operands[k]
        d = torch.from_numpy(host[k]).to(DEV, dtype).requires_grad_(True)
        ts[k] = P.SymTensor(d, op.signs, op.charge, wl.group)
    cur = dict(ts)
    for st in wl.steps:
        cur[st.w] = P.einsum(st.einsum, cur[st.u], cur[st.v], compute)
    R = torch.from_numpy(host["R"]).to(DEV, dtype)
    loss = (cur[wl.output].data * R).sum()
    loss.backward()
    return float(loss.item()), {k: H.to_np(ts[k].data.grad).astype(np.float64) for k in PARAMS}


def _oracle_loss(wl, syms, vals):
    cur = dict(vals)
    for st in wl.steps:
        cur[st.w], _ = O.contract_blocks(st.einsum, cur[st.u], syms[st.u], cur[st.v], syms[st.v])
    return float(np.sum(cur[wl.output] * vals["R"]))


def _dense_grads(wl, syms, host):
    """Dense binary64 autograd on the CPU: every tensor expanded with its zero blocks."""
    dense = {k: torch.from_numpy(O.expand(host[k], syms[k])).requires_grad_(k in PARAMS) for k in host}
    cur = dict(dense)
    for st in wl.steps:
        a = cur[st.u]
        b = cur[st.v].contiguous()
        cur[st.w] = torch.einsum(st.einsum, a, b)
    loss = (cur[wl.output] * dense["R"]).sum()
    loss.backward()
    return float(loss.item()), {k: dense[k].grad.numpy() for k in PARAMS}


def _host_inputs(wl):
    return {k: synth.host_input(wl, k) for k in wl.inputs}


@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_grad_shrunk_chain_vs_dense_autograd(P, compute):
    wl = synth.configs.scaled(synth.configs.mps_env_grad(), {m: 4 for m in "acACAC"})
    say(f"grad {wl.name} {compute} vs dense autograd")
    syms = {k: H.sym_of(op, wl.group) for k, op in wl.operands.items()}
    host = _host_inputs(wl)
    dtype = torch.float64 if compute == "f64" else torch.float32
    if compute == "f32":
        host = {k: v.astype(np.float32).astype(np.float64) for k, v in host.items()}
    loss, grads = _gpu_loss_and_grads(P, wl, host, compute, dtype)
    dloss, dgrads = _dense_grads(wl, syms, host)
    assert abs(loss - dloss) <= (1e-12 if compute == "f64" else 1e-5) * abs(dloss)
    for k in PARAMS:
        red, zero_ok = O.reduce_full(dgrads[k], syms[k])
        assert zero_ok, f"dense gradient of {k} is nonzero off the rule"
        err = H.rel_err(grads[k], red)
        say(f"  dL/d{k}: relative error vs dense autograd {err:.3e}")
        assert err <= (1e-12 if compute == "f64" else 2e-5)


@pytest.mark.timeout(600)
def test_grad_full_bond_vs_finite_differences(P):
    wl = synth.configs.mps_env_grad()
    say(f"grad {wl.name} f64 vs central differences (h = 1e-6)")
    syms = {k: H.sym_of(op, wl.group) for k, op in wl.operands.items()}
    host = _host_inputs(wl)
    loss, grads = _gpu_loss_and_grads(P, wl, host, "f64", torch.float64)
    l0 = _oracle_loss(wl, syms, host)
    assert abs(loss - l0) <= 1e-12 * abs(l0)
    rng = np.random.default_rng(44)
    h = 1e-6
    for k in ("A", "W"):
        for rep in range(3):
            d = rng.standard_normal(host[k].shape)
            plus = dict(host)
            minus = dict(host)
            plus[k] = host[k] + h * d
            minus[k] = host[k] - h * d
            fd = (_oracle_loss(wl, syms, plus) - _oracle_loss(wl, syms, minus)) / (2 * h)
            an = float(np.sum(grads[k] * d))
            rel = abs(fd - an) / max(abs(fd), 1e-300)
            say(f"  dL/d{k} along direction {rep}: analytic {an:.10e} fd {fd:.10e} rel {rel:.2e}")
            assert rel <= 1e-7


@pytest.mark.timeout(600)
def test_grad_full_bond_f32_vs_f64(P):
    wl = synth.configs.mps_env_grad()
    say(f"grad {wl.name} f32 vs f64")
    host = _host_inputs(wl)
    _, g64 = _gpu_loss_and_grads(P, wl, host, "f64", torch.float64)
    _, g32 = _gpu_loss_and_grads(P, wl, host, "f32", torch.float32)
    for k in PARAMS:
        err = H.rel_err(g32[k], g64[k])
        say(f"  dL/d{k}: f32 relative error vs f64 {err:.3e}")
        assert err <= 1e-4
