"""Helpers shared by the GPU parity tests: workload operands on both sides, sampling."""
from __future__ import annotations

import math

import numpy as np
import torch

import oracle as O
import synth
from synth import host as synth_host
from synth import philox


def sym_of(op, group) -> O.Sym:
    return O.Sym.make(op.signs, op.charge, op.dims, O.Group(group))


def value_fn(wl, name, absolute=False):
    """Oracle-side values of an input at reduced-form coordinates, from the generator."""
    op = wl.operands[name]
    shape = wl.reduced_shape(name)

    gen = synth_host.values_at if synth_host.available() else philox.values_at

    def fn(secs, inner):
        e = np.ravel_multi_index(tuple(secs) + tuple(inner), shape)
        x = gen(e, wl.seed, op.tensor_id, op.dist, op.scale)
        return np.abs(x) if absolute else x
    return fn


def f32_value_fn(fn):
    """Values rounded to binary32 and widened back (inputs of the f32 / bf16x3 forms)."""
    def g(secs, inner):
        return fn(secs, inner).astype(np.float32).astype(np.float64)
    return g


def random_w_positions(sw: O.Sym, count: int, rng) -> tuple:
    """`count` random elements of W: (reduced-form index tuples, full-index array)."""
    G = sw.group.size
    n = sw.order
    red, full = [], []
    for _ in range(count):
        stored = tuple(int(x) for x in rng.integers(0, G, n - 1))
        secs = O.full_sectors(sw, stored)
        inner = tuple(int(rng.integers(0, d)) for d in sw.dims)
        red.append(stored + inner)
        full.append([S * d + i for S, d, i in zip(secs, sw.dims, inner)])
    return red, np.asarray(full, dtype=np.int64)


def gamma(k: int, u: float) -> float:
    return k * u / (1.0 - k * u)


U64 = 2.0 ** -53
U32 = 2.0 ** -24
U_BF16_PAIR = 2.0 ** -16


def bound_factor(compute: str, k: int) -> float:
    """Componentwise bound on |W_gpu - W_exact| in units of (|U| |V|) (Higham, Sec. 3.5).

    f64: two summation orders (kernel and oracle), gamma_k(u64) each.
    f32: inputs rounded to binary32 (u32 each) plus binary32 accumulation.
    bf16x3: hi + lo keeps 16 bits of each binary32 input, the dropped lo*lo term
    is below 2^-16 of the product, plus binary32 accumulation of the 3k products
    (hi*hi, hi*lo, lo*hi: one accumulator on the wide tiles; their |terms| sum to
    at most 1.01 |a||b|).
    """
    if compute == "f64":
        return 2.0 * gamma(k, U64)
    if compute == "f32":
        return 2.1 * U32 + 1.05 * gamma(k, U32) + gamma(k, U64)
    return 3.1 * U_BF16_PAIR + 2.1 * U32 + 1.02 * gamma(3 * k, U32) + gamma(k, U64)


def to_np(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def rel_err(got, ref) -> float:
    dt = np.result_type(np.asarray(got).dtype, np.asarray(ref).dtype, np.float64)   # complex stays complex
    got = np.asarray(got, dtype=dt)
    ref = np.asarray(ref, dtype=dt)
    den = np.max(np.abs(ref)) if ref.size else 0.0
    return float(np.max(np.abs(got - ref)) / den) if den > 0 else float(np.max(np.abs(got - ref), initial=0.0))


def contracted_extent(sub, su: O.Sym) -> int:
    tu, tv, tw, I, K, J = O.parse_einsum(sub)
    return math.prod(su.group.size * su.dims[tu.index(k)] for k in K)


def random_case(rng, orders, s, t, v, nmax=3, nmin=1, sigma=None, dim_choices=None):
    """A random contraction (subscripts and both operand symmetries) with s, t, v modes.

    Block dims are uniform in [nmin, nmax], or drawn from ``dim_choices``.
    """
    g = O.Group(orders)
    letters = iter("abcdefghijklmnop")
    I = [next(letters) for _ in range(s)]
    K = [next(letters) for _ in range(v)]
    J = [next(letters) for _ in range(t)]
    tu = list(I + K); rng.shuffle(tu)
    tv = list(K + J); rng.shuffle(tv)
    tw = list(I + J); rng.shuffle(tw)
    if dim_choices is None:
        dims = {m: int(rng.integers(nmin, nmax + 1)) for m in I + K + J}
    else:
        dims = {m: int(rng.choice(dim_choices)) for m in I + K + J}
    cu = {m: int(rng.choice([-1, 1])) for m in tu}
    sigma = int(rng.choice([-1, 1])) if sigma is None else sigma
    cv = {m: (sigma * cu[m] if m in K else int(rng.choice([-1, 1]))) for m in tv}
    su = O.Sym(tuple(cu[m] for m in tu), int(rng.integers(g.size)), tuple(dims[m] for m in tu), g)
    sv = O.Sym(tuple(cv[m] for m in tv), int(rng.integers(g.size)), tuple(dims[m] for m in tv), g)
    return f"{''.join(tu)},{''.join(tv)}->{''.join(tw)}", su, sv


def subgroup_case(rng, G, s, t, v, nmax=3):
    """A random contraction over Z_G whose modes have random sector counts H | G
    (coefficient sign G/H, Sec. 2.2), contracted modes sharing theirs, with total
    charges that some sector combination reaches."""
    g = O.Group(G)
    letters = iter("abcdefghijklmnop")
    I = [next(letters) for _ in range(s)]
    K = [next(letters) for _ in range(v)]
    J = [next(letters) for _ in range(t)]
    tu = list(I + K); rng.shuffle(tu)
    tv = list(K + J); rng.shuffle(tv)
    tw = list(I + J); rng.shuffle(tw)
    divs = [h for h in range(1, G + 1) if G % h == 0]
    hs = {m: int(rng.choice(divs)) for m in I + K + J}
    dims = {m: int(rng.integers(1, nmax + 1)) for m in I + K + J}
    cu = {m: int(rng.choice([-1, 1])) for m in tu}
    sigma = int(rng.choice([-1, 1]))
    cv = {m: (sigma * cu[m] if m in K else int(rng.choice([-1, 1]))) for m in tv}

    def reach(term, c):
        return sum(c[m] * (G // hs[m]) * int(rng.integers(hs[m])) for m in term) % G
    su = O.Sym.make([cu[m] for m in tu], reach(tu, cu), [dims[m] for m in tu], g, sectors=[hs[m] for m in tu])
    sv = O.Sym.make([cv[m] for m in tv], reach(tv, cv), [dims[m] for m in tv], g, sectors=[hs[m] for m in tv])
    return f"{''.join(tu)},{''.join(tv)}->{''.join(tw)}", su, sv


def dead_stored_tuples(sym):
    """Stored-sector tuples of the standard reduced form that hold no block."""
    return [st for st in O.stored_tuples(sym) if O.full_sectors(sym, st) is None]
