"""U(1)-symmetric test operands and their embedding in a cyclic group.

A U(1) tensor has integer charges: each mode m carries the charges
q_min[m] .. q_min[m] + P[m] - 1 (one block of n[m] indices per charge) and an
element is nonzero only where sum_m c_m q_m equals the total charge Z exactly.
The paper (Sec. 3) notes that such a symmetry can be emulated by a cyclic group
that is large enough; here a mode's charge q sits at sector label q - q_min[m]
of Z_G, i.e. label L of mode m carries charge (L + q_min[m]) mod G, which is a
per-mode charge table.  G >= P[m] keeps that map one-to-one; labels L >= P[m]
hold zero blocks.  Everything here is plain integer bookkeeping: the dense
tensors are built and contracted without any group arithmetic.
"""
import itertools

import numpy as np

import oracle as O


def dense_u1(rng, signs, Z, qmin, P, n):
    """Dense U(1) tensor, charge-major along each mode (charge q_min + p at rows p*n .. p*n + n - 1)."""
    T = np.zeros(tuple(p * d for p, d in zip(P, n)))
    for secs in itertools.product(*(range(p) for p in P)):
        if sum(c * (q0 + s) for c, q0, s in zip(signs, qmin, secs)) != Z:
            continue
        sl = tuple(slice(s * d, (s + 1) * d) for s, d in zip(secs, n))
        T[sl] = rng.standard_normal(tuple(n))
    return T


def tables(qmin, G):
    """Per-mode charge tables: label L of mode m carries charge (L + q_min[m]) mod G."""
    return [[(L + q0) % G for L in range(G)] for q0 in qmin]


def embed(T, signs, Z, qmin, P, n, G):
    """(Sym, reduced form) of the U(1) tensor T inside Z_G."""
    sym = O.Sym.make(signs, Z % G, n, O.Group(G), charges=tables(qmin, G))
    full = np.zeros(sym.full_shape())
    full[tuple(slice(0, p * d) for p, d in zip(P, n))] = T
    R, zero_ok = O.reduce_full(full, sym)
    if not zero_ok:
        raise AssertionError("a U(1)-allowed block is not allowed in Z_G")
    return sym, R


def physical_part(full_w, P, n):
    """The part of a full Z_G tensor at labels that carry U(1) charges, and the rest's max |value|."""
    sl = tuple(slice(0, p * d) for p, d in zip(P, n))
    rest = full_w.copy()
    rest[sl] = 0.0
    return full_w[sl], float(np.max(np.abs(rest))) if rest.size else 0.0


def random_case(rng, sub, G_extra=0, nmax=3):
    """A contraction of two random U(1) tensors: per-letter charge ranges and block sizes,
    signs with a uniform ratio over contracted letters, and the smallest G that emulates
    it (plus G_extra).  Returns a dict with everything the tests need."""
    tu, rest = sub.split(",")
    tv, tw = rest.split("->")
    letters = sorted(set(tu + tv))
    qmin = {m: int(rng.integers(-2, 1)) for m in letters}
    P = {m: int(rng.integers(2, 5)) for m in letters}
    n = {m: int(rng.integers(1, nmax + 1)) for m in letters}
    cu = {m: int(rng.choice([-1, 1])) for m in tu}
    sigma = int(rng.choice([-1, 1]))
    cv = {m: (sigma * cu[m] if m in tu else int(rng.choice([-1, 1]))) for m in tv}

    def total(term, c):
        # a total charge that some sector combination reaches
        return sum(c[m] * (qmin[m] + int(rng.integers(P[m]))) for m in term)

    Zu, Zv = total(tu, cu), total(tv, cv)
    G = max(P.values()) + G_extra
    Tu = dense_u1(rng, [cu[m] for m in tu], Zu, [qmin[m] for m in tu], [P[m] for m in tu], [n[m] for m in tu])
    Tv = dense_u1(rng, [cv[m] for m in tv], Zv, [qmin[m] for m in tv], [P[m] for m in tv], [n[m] for m in tv])
    su, Ru = embed(Tu, [cu[m] for m in tu], Zu, [qmin[m] for m in tu], [P[m] for m in tu],
                   [n[m] for m in tu], G)
    sv, Rv = embed(Tv, [cv[m] for m in tv], Zv, [qmin[m] for m in tv], [P[m] for m in tv],
                   [n[m] for m in tv], G)
    return dict(sub=sub, G=G, Tu=Tu, Tv=Tv, su=su, sv=sv, Ru=Ru, Rv=Rv,
                Pw=[P[m] for m in tw], nw=[n[m] for m in tw], ref=np.einsum(sub, Tu, Tv))
