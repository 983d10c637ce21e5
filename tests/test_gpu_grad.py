"""Hand-written backward of the contraction, on the differentiated MPS environment chain.

L = <E', R> with E' = ((E A) W) A contracted left to right; gradients with
respect to A (used twice), W and E come from the library's backward (two more
symmetric contractions per step, aligned forms recomputed).  Checked against
* dense torch autograd on the CPU in binary64 (zero blocks materialised), every
  entry, on a chain with the bond block shrunk to 4; the dense gradient must be
  exactly zero off the conservation rule;
* dense torch autograd on the CPU in binary64 at the full bond block of 128,
  every entry of dL/dE, dL/dA and dL/dW, for the f64 and the f32 library
  paths (the f32 one on binary32-rounded inputs, within a componentwise
  bound);
* central finite differences of the binary64 oracle forward at the full bond
  block, along 8 seeded directions per parameter and at 64 sampled entries.
  L is linear in E and W and quadratic in A, so the central difference has no
  truncation error.
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


def _dense_grads_abs(wl, syms, host):
    """The same dense autograd on |inputs|: bounds |dL/dx| term by term (componentwise bounds)."""
    return _dense_grads(wl, syms, {k: np.abs(v) for k, v in host.items()})


def _chain_bound_factor(P, wl, compute_u):
    """First-order componentwise bound of the chain's gradients, in units of the |.|-chain's gradient.

    Every contraction of the forward (T1, T2, E') and of the backward (two per
    step: dU sums over the step's N extent, dV over its M extent) adds at most
    gamma_k(u) + u (binary32 accumulation over k terms, then the stored
    result rounded) relative to the |.|-products it forms, and the two uses of
    A add one more rounding; summed over every contraction this bounds each
    gradient entry (Higham, Sec. 3.5, to first order).
    """
    from paper_2007_08056_amd import _lib as L
    total = 2 * compute_u
    g = L.make_group(wl.group)
    for st in wl.steps:
        ou, ov = wl.operands[st.u], wl.operands[st.v]
        info = L.plan(st.einsum, g, L.TensorDesc(ou.signs, ou.charge, ou.dims, L.SYMT_F32, None),
                      L.TensorDesc(ov.signs, ov.charge, ov.dims, L.SYMT_F32, None), None, L.COMPUTE["f32"])
        for k in (info.k, info.n, info.m):
            total += H.gamma(k, compute_u) + compute_u
    return total


@pytest.fixture(scope="module")
def full_bond(P):
    """Inputs of the differentiated chain at bond 128, and the library's f64 loss and gradients."""
    wl = synth.configs.mps_env_grad()
    syms = {k: H.sym_of(op, wl.group) for k, op in wl.operands.items()}
    host = _host_inputs(wl)
    say(f"grad {wl.name}: library f64 forward and backward")
    loss, grads = _gpu_loss_and_grads(P, wl, host, "f64", torch.float64)
    return wl, syms, host, loss, grads


@pytest.mark.timeout(600)
@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_grad_full_bond_vs_dense_autograd(P, full_bond, compute):
    """Every entry of dL/dE, dL/dA and dL/dW at bond 128 against dense binary64 autograd on the CPU."""
    wl, syms, host, loss, grads = full_bond
    if compute == "f32":
        host = {k: v.astype(np.float32).astype(np.float64) for k, v in host.items()}
        say(f"grad {wl.name}: library f32 forward and backward (binary32-rounded inputs)")
        loss, grads = _gpu_loss_and_grads(P, wl, host, "f32", torch.float32)
    say(f"grad {wl.name} {compute}: dense binary64 autograd on the CPU ({torch.get_num_threads()} threads)")
    dloss, dgrads = _dense_grads(wl, syms, host)
    assert abs(loss - dloss) <= (1e-12 if compute == "f64" else 1e-5) * abs(dloss)
    if compute == "f32":
        _, agrads = _dense_grads_abs(wl, syms, host)
        factor = 1.01 * _chain_bound_factor(P, wl, H.U32)
        say(f"  componentwise bound factor {factor:.3e}")
    for k in PARAMS:
        red, zero_ok = O.reduce_full(dgrads[k], syms[k])
        assert zero_ok, f"dense gradient of {k} is nonzero off the rule"
        err = H.rel_err(grads[k], red)
        say(f"  dL/d{k}: normwise relative error vs dense autograd {err:.3e}")
        if compute == "f64":
            assert err <= 1e-12
        else:
            assert err <= 1e-4
            bound, _ = O.reduce_full(agrads[k], syms[k])
            worst = float(np.max(np.abs(grads[k] - red) / np.maximum(factor * bound, 1e-300)))
            say(f"  dL/d{k}: largest error / componentwise bound {worst:.3e}")
            assert worst <= 1.0


@pytest.mark.timeout(900)
def test_grad_full_bond_vs_finite_differences(P, full_bond):
    """Central differences of the binary64 oracle at bond 128: 8 seeded directions for each of
    E, A and W (h = 1e-6) and 64 sampled entries (h = 1: L is at most quadratic in each
    parameter, so the central difference is exact for any h and a large h only cuts rounding)."""
    import multiprocessing as mp
    from tests import fd_chain
    wl, syms, host, loss, grads = full_bond
    l0 = _oracle_loss(wl, syms, host)
    assert abs(loss - l0) <= 1e-12 * abs(l0)
    rng = np.random.default_rng(44)
    jobs = [(k, "dir", 1000 * i + j, 1e-6) for i, k in enumerate(PARAMS) for j in range(8)]
    for i, k in enumerate(PARAMS):
        n = (22, 21, 21)[i]
        jobs += [(k, "entry", int(e), 1.0) for e in rng.choice(host[k].size, n, replace=False)]
    workers = 8
    say(f"grad {wl.name}: {len(jobs)} central differences of the oracle forward on {workers} CPU workers")
    with mp.get_context("spawn").Pool(workers, initializer=fd_chain.init, initargs=(2,)) as pool:
        fds = pool.map(fd_chain.central_difference, jobs, chunksize=1)
    for (k, kind, arg, h), fd in zip(jobs, fds):
        d = fd_chain.direction(host[k].shape, kind, arg)
        an = float(np.sum(grads[k] * d))
        if kind == "dir":
            rel = abs(fd - an) / max(abs(fd), 1e-300)
        else:
            rel = abs(fd - an) / max(float(np.max(np.abs(grads[k]))), 1e-300)
        if kind == "dir" or rel > 1e-9:
            say(f"  dL/d{k} {kind} {arg}: analytic {an:.12e} fd {fd:.12e} rel {rel:.2e}")
        assert rel <= 1e-8, (k, kind, arg)


# s, t or v = 0 (one delta pins Q): the backward of an outer product is a full
# contraction and vice versa, and the outer-product gradients take the sign
# ratio that gives the operand's own rule.
DEGENERATE = ["a,b->ab", "ab,c->abc", "ab,cd->acbd",        # v = 0: outer products
              "k,kb->b", "kl,klij->ij", "lk,klb->b",         # s = 0
              "ak,k->a", "abk,k->ab", "akl,lk->a"]           # t = 0


@pytest.mark.parametrize("sub", DEGENERATE)
@pytest.mark.parametrize("orders", [(4,), (2, 3)])
def test_grad_degenerate_contractions_vs_dense_autograd(P, sub, orders):
    from tests.seeding import seed
    rng = np.random.default_rng(seed(("grad-degenerate", sub, orders)))
    g = O.Group(orders)
    tu, rest = sub.split(",")
    tv, tw = rest.split("->")
    for sigma in (-1, 1):
        dims = {m: int(rng.integers(1, 5)) for m in set(tu + tv)}
        cu = {m: int(rng.choice([-1, 1])) for m in tu}
        cv = {m: (sigma * cu[m] if m in tu else int(rng.choice([-1, 1]))) for m in tv}
        su = O.Sym.make([cu[m] for m in tu], int(rng.integers(g.size)), [dims[m] for m in tu], g)
        sv = O.Sym.make([cv[m] for m in tv], int(rng.integers(g.size)), [dims[m] for m in tv], g)
        sw = O.output_symmetry(sub, su, sv)
        say(f"grad degenerate {sub} G={orders} sigma={sigma}")
        Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
        Rr = rng.standard_normal(sw.reduced_shape())
        ud = torch.from_numpy(Ru).to(DEV).requires_grad_(True)
        vd = torch.from_numpy(Rv).to(DEV).requires_grad_(True)
        u = P.SymTensor(ud, su.sign_string(), su.charge, orders)
        v = P.SymTensor(vd, sv.sign_string(), sv.charge, orders)
        w = P.einsum(sub, u, v, "f64")
        (w.data * torch.from_numpy(Rr).to(DEV)).sum().backward()
        # dense binary64 autograd on the CPU, zero blocks materialised
        Ud = torch.from_numpy(O.expand(Ru, su)).requires_grad_(True)
        Vd = torch.from_numpy(O.expand(Rv, sv)).requires_grad_(True)
        (torch.einsum(sub, Ud, Vd) * torch.from_numpy(O.expand(Rr, sw))).sum().backward()
        for name, got, dense, sym in (("u", ud.grad, Ud.grad, su), ("v", vd.grad, Vd.grad, sv)):
            red, zero_ok = O.reduce_full(dense.numpy(), sym)
            assert zero_ok, f"dense gradient of {name} is nonzero off its rule"
            err = H.rel_err(H.to_np(got), red)
            assert err <= 1e-12 or np.max(np.abs(red)) == 0, (name, err)
