"""Central finite differences of the differentiated MPS environment chain, on the CPU.

Worker-process side of the gradient tests: each job evaluates the binary64
oracle's loss L = <E', R>, E' = ((E A) W) A contracted left to right with the
loop-over-blocks form, at x + h d and x - h d for one parameter x (E, A or W)
and one direction d (a seeded normal direction, or one entry), and returns
(L(x + h d) - L(x - h d)) / (2 h).  L is linear in E and W and quadratic in
A, so the central difference has no truncation error for any h; only rounding
remains.  Imports NumPy, the oracle and the seeded generator only (no torch,
no GPU), so a pool of these workers can run beside a process that uses the GPU.
"""
from __future__ import annotations

import numpy as np

import oracle as O
import synth

_STATE: dict = {}


def init(threads: int, bond: int | None = None):
    from threadpoolctl import threadpool_limits
    _STATE["limit"] = threadpool_limits(limits=threads)
    wl = synth.configs.mps_env_grad()
    if bond is not None:
        wl = synth.configs.scaled(wl, {m: bond for m in "acAC"})
    g = O.Group(wl.group)
    _STATE["wl"] = wl
    _STATE["syms"] = {k: O.Sym.make(op.signs, op.charge, op.dims, g) for k, op in wl.operands.items()}
    _STATE["host"] = {k: synth.host_input(wl, k) for k in wl.inputs}


def chain_loss(vals) -> float:
    wl, syms = _STATE["wl"], _STATE["syms"]
    cur = dict(vals)
    for st in wl.steps:
        cur[st.w], _ = O.contract_blocks(st.einsum, cur[st.u], syms[st.u], cur[st.v], syms[st.v])
    return float(np.sum(cur[wl.output] * vals["R"]))


def direction(shape, kind: str, arg: int) -> np.ndarray:
    """A seeded normal direction (kind "dir", arg = seed) or one entry (kind "entry", arg = flat index)."""
    if kind == "dir":
        return np.random.default_rng(arg).standard_normal(shape)
    d = np.zeros(int(np.prod(shape)))
    d[arg] = 1.0
    return d.reshape(shape)


def central_difference(job) -> float:
    param, kind, arg, h = job
    host = dict(_STATE["host"])
    x = host[param]
    d = direction(x.shape, kind, arg)
    host[param] = x + h * d
    plus = chain_loss(host)
    host[param] = x - h * d
    minus = chain_loss(host)
    return (plus - minus) / (2.0 * h)
