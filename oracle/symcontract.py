"""Plain, slow CPU reference for contractions of tensors with cyclic-group symmetry.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this module; only
the test suite, the smoke check and the benchmark's CPU-baseline leg may call
it.  It shares no code with the GPU path.  Arithmetic is binary64 throughout,
complex binary64 when an operand is complex (tensors over R or C, Sec. 2.2).

Notation (paper Sec. 2.2, Eq. symtsr and Eq. redform).  A tensor of order N has
modes m = 0..N-1; mode m has |G| sectors and block dimension n_m, so its full
index is x_m = I_m * n_m + i_m (sector I_m, in-block position i_m).  With
coefficients c_m = +1 or -1 and total charge Z, an element can be nonzero only
if sum_m c_m I_m == Z in the group.  The standard reduced form stores the
sectors of modes 0..N-2 and every in-block index; the sector of the last mode
is implied by the conservation rule (paper Sec. 2.1 footnote, the assumption
Alg. 2 makes when it forms the aligned operands, API example of Sec. 3).

Groups are Z_{g_1} x ... x Z_{g_k} (Sec. 3 mentions products of cyclic
groups).  An element is flattened mixed-radix, first factor most significant,
and added component-wise.

Charge tables (optional, per mode): sector label L of mode m carries the
charge chi_m(L), a permutation of the group elements (identity when absent),
and the rule reads sum_m c_m chi_m(I_m) == Z.  Stored axes of every reduced
form, standard or aligned, are indexed by label; Q and the deltas of Alg. 2
are in charges.

Forms of the reference result (all must agree):

1. ``contract_dense``   expand both operands to full tensors with their zero
   blocks, one dense einsum, reduce (the symmetry-oblivious route of Sec. 2.1).
2. ``contract_blocks``  loop over allowed sector tuples, one block product each
   (Alg. 1, generalised to any number of free and contracted modes).
3. ``sample_contract``  selected output elements, each summed over every
   contracted full index with a conservation-aware element lookup;
   ``sample_contract_allowed`` the same sums over the allowed contracted
   sectors only (fast enough for thousands of elements of a large contraction).
4. ``contract_bruteforce`` pure-Python loops over full indices (tiny inputs).
5. ``contract_irrep_aligned`` Alg. 2 itself, with the generalized Kronecker
   deltas built as dense 0/1 tensors and every step an einsum, as the paper's
   library does (Sec. 3).  It also returns the three aligned reduced forms.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np


# ----------------------------------------------------------------------------
# Groups
# ----------------------------------------------------------------------------
def _ftype(*arrays):
    """binary64, or complex binary64 when any input is complex (tensors over R or C, Sec. 2.2)."""
    return np.result_type(*[np.asarray(a).dtype for a in arrays], np.float64)


class Group:
    """Z_{orders[0]} x Z_{orders[1]} x ...; elements are ints in [0, size)."""

    def __init__(self, orders):
        orders = tuple(int(o) for o in (orders if isinstance(orders, (tuple, list)) else (orders,)))
        if not orders or any(o < 1 for o in orders):
            raise ValueError("group orders must be positive")
        self.orders = orders
        self.size = int(np.prod(orders))

    def digits(self, e):
        out = []
        for o in reversed(self.orders):
            out.append(e % o)
            e = e // o
        return tuple(reversed(out))

    def element(self, digits):
        e = 0
        for d, o in zip(digits, self.orders):
            e = e * o + (d % o)
        return e

    def add(self, a, b):
        return self.element(tuple(x + y for x, y in zip(self.digits(a), self.digits(b))))

    def neg(self, a):
        return self.element(tuple(-x for x in self.digits(a)))

    def sub(self, a, b):
        return self.add(a, self.neg(b))

    def times(self, c, a):
        """c * a for an integer coefficient c (repeated addition / negation)."""
        return self.element(tuple(c * x for x in self.digits(a)))

    def total(self, coefs, elems):
        acc = 0
        for c, e in zip(coefs, elems):
            acc = self.add(acc, self.times(c, e))
        return acc


@dataclass(frozen=True)
class Sym:
    """Symmetry of one operand: signs (+1/-1), total charge, block dims, group,
    optional per-mode charge tables (None: every label is its own charge) and
    optional per-mode sector counts H_m (None: |G| each).

    A mode with H_m < |G| sectors carries the coefficient sign * |G| / H_m
    (Sec. 2.2, Eq. symtsr: c_i = +-G/H_i); its sectors are 0..H_m-1.
    Sector counts other than |G| need a cyclic group and no charge tables.
    """
    signs: tuple
    charge: int
    dims: tuple
    group: Group
    charges: tuple | None = None
    sectors: tuple | None = None

    @staticmethod
    def make(signs, charge, dims, group, charges=None, sectors=None):
        if isinstance(signs, str):
            signs = tuple(+1 if ch == "+" else -1 for ch in signs)
        if not isinstance(group, Group):
            group = Group(group)
        G = group.size
        if charges is not None:
            charges = tuple(tuple(int(x) for x in row) for row in charges)
            if len(charges) != len(signs) or any(sorted(r) != list(range(G)) for r in charges):
                raise ValueError("charge tables must be one permutation of the group per mode")
            if all(r == tuple(range(G)) for r in charges):
                charges = None
        if sectors is not None:
            sectors = tuple(int(h) for h in sectors)
            if len(sectors) != len(signs) or any(h < 1 or G % h for h in sectors):
                raise ValueError("sector counts must divide |G|, one per mode")
            if all(h == G for h in sectors):
                sectors = None
            elif len(group.orders) != 1 or charges is not None:
                raise ValueError("sector counts below |G| need a cyclic group and no charge tables")
        return Sym(tuple(int(s) for s in signs), int(charge) % G, tuple(int(d) for d in dims), group,
                   charges, sectors)

    def H(self, m):
        """Number of sectors of mode m."""
        return self.group.size if self.sectors is None else self.sectors[m]

    def coef(self, m):
        """Integer coefficient c_m of Eq. symtsr: sign * |G| / H_m."""
        return self.signs[m] * (self.group.size // self.H(m))

    @property
    def coefs(self):
        return tuple(self.coef(m) for m in range(self.order))

    def chi(self, m, label):
        """Charge of sector label `label` of mode m."""
        return label if self.charges is None else self.charges[m][label]

    def label(self, m, charge):
        """Sector label of mode m that carries `charge`."""
        return charge if self.charges is None else self.charges[m].index(charge)

    def table(self, m):
        return tuple(range(self.group.size)) if self.charges is None else self.charges[m]

    @property
    def order(self):
        return len(self.signs)

    def reduced_shape(self):
        return tuple(self.H(m) for m in range(self.order - 1)) + self.dims

    def full_shape(self):
        return tuple(self.H(m) * n for m, n in enumerate(self.dims))

    def sign_string(self):
        return "".join("+" if c > 0 else "-" for c in self.signs)


def allowed(sym: Sym, sectors) -> bool:
    """Conservation rule of Eq. symtsr: sum_m c_m chi_m(I_m) == Z."""
    return sym.group.total(sym.coefs, [sym.chi(m, s) for m, s in enumerate(sectors)]) == sym.charge


def implicit_sector(sym: Sym, known, position=None):
    """The one sector that the conservation rule leaves free.

    ``known`` lists the sectors of every mode except ``position`` (default: the
    last mode, the implicit one of the standard reduced form).  Solves
    c_p I_p == Z - sum_{m != p} c_m I_m; with c_p = +1 or -1 the inverse of c_p
    is c_p itself.  With c_p = s |G| / H_p (a subgroup mode) the equation has
    the one solution I_p = s (rest / (|G| / H_p)) mod H_p when |G| / H_p
    divides rest, and none otherwise: then None (no such block).
    """
    g = sym.group
    p = sym.order - 1 if position is None else position
    modes = [m for m in range(sym.order) if m != p]
    others = [sym.coef(m) for m in modes]
    rest = g.sub(sym.charge, g.total(others, [sym.chi(m, s) for m, s in zip(modes, known)]))
    d = g.size // sym.H(p)
    if d == 1:
        return sym.label(p, g.times(sym.signs[p], rest))
    if rest % d:
        return None
    return (sym.signs[p] * (rest // d)) % sym.H(p)


def full_sectors(sym: Sym, stored):
    """All sectors of a block from its stored ones, or None if the rule has no solution."""
    last = implicit_sector(sym, stored)
    return None if last is None else tuple(stored) + (last,)


def stored_tuples(sym: Sym):
    """Every stored-sector tuple of the standard reduced form (modes 0..N-2)."""
    return itertools.product(*[range(sym.H(m)) for m in range(sym.order - 1)])


# ----------------------------------------------------------------------------
# Reduced form <-> full tensor
# ----------------------------------------------------------------------------
def expand(R, sym: Sym) -> np.ndarray:
    """Full tensor with every zero block materialised (Eq. symtsr)."""
    R = np.asarray(R)
    R = R.astype(_ftype(R), copy=False)
    if R.shape != sym.reduced_shape():
        raise ValueError(f"reduced form has shape {R.shape}, expected {sym.reduced_shape()}")
    full = np.zeros(sym.full_shape(), dtype=R.dtype)
    for stored in stored_tuples(sym):
        secs = full_sectors(sym, stored)
        if secs is None:
            continue
        sl = tuple(slice(s * n, (s + 1) * n) for s, n in zip(secs, sym.dims))
        full[sl] = R[stored]
    return full


def reduce_full(T, sym: Sym):
    """Standard reduced form of a full tensor, and whether every disallowed block is exactly 0."""
    T = np.asarray(T)
    R = np.zeros(sym.reduced_shape(), dtype=T.dtype)
    zero_ok = True
    for secs in itertools.product(*[range(sym.H(m)) for m in range(sym.order)]):
        sl = tuple(slice(s * n, (s + 1) * n) for s, n in zip(secs, sym.dims))
        if allowed(sym, secs):
            R[secs[:-1]] = T[sl]
        elif np.any(T[sl] != 0):
            zero_ok = False
    return R, zero_ok


def lookup(R, sym: Sym, full_index):
    """One element of the full tensor, read from its reduced form (0 off the rule)."""
    secs = tuple(x // n for x, n in zip(full_index, sym.dims))
    inner = tuple(x % n for x, n in zip(full_index, sym.dims))
    if not allowed(sym, secs):
        return 0.0
    return R[secs[:-1] + inner].item()


# ----------------------------------------------------------------------------
# Contraction bookkeeping
# ----------------------------------------------------------------------------
def parse_einsum(sub: str):
    """Split "tu,tv->tw"; returns (tu, tv, tw, I, K, J).

    I: modes of U kept in W (order of U); K: modes shared by U and V, summed
    (order of U); J: modes of V kept in W (order of V) -- the s, v and t modes
    of Eq. ctr.
    """
    sub = sub.replace(" ", "")
    lhs, tw = sub.split("->")
    tu, tv = lhs.split(",")
    for t in (tu, tv, tw):
        if len(set(t)) != len(t):
            raise ValueError(f"repeated index in term {t!r}")
    I = [m for m in tu if m in tw and m not in tv]
    K = [m for m in tu if m in tv and m not in tw]
    J = [m for m in tv if m in tw and m not in tu]
    if any(m in tu and m in tv and m in tw for m in tw):
        raise ValueError("an index in all three terms is not a contraction of Eq. ctr")
    if set(tw) != set(I) | set(J) or set(tu) != set(I) | set(K) or set(tv) != set(K) | set(J):
        raise ValueError("every index must appear in exactly two terms")
    return tu, tv, tw, I, K, J


def contracted_sign_ratio(sub, su: Sym, sv: Sym) -> int:
    """sigma = c^V_k / c^U_k, required to be the same for every contracted mode.

    Alg. 2 assumes equal coefficients on the contracted modes (sigma = +1); the
    text right after Eq. ctr allows them to differ by a sign, as in the worked
    example of Sec. 2.1 (sigma = -1).  A mixed ratio is rejected: no single
    auxiliary sector Q then describes both operands.
    """
    tu, tv, tw, I, K, J = parse_einsum(sub)
    if not K:
        # v = 0 (outer product): Q is pinned to 0 and no ratio is defined; -1
        # makes W's coefficients U's followed by V's, Z^W = Z^U + Z^V
        return -1
    ratios = {su.signs[tu.index(k)] * sv.signs[tv.index(k)] for k in K}
    if len(ratios) != 1:
        raise ValueError("contracted modes carry mixed sign ratios")
    return ratios.pop()


def output_symmetry(sub, su: Sym, sv: Sym) -> Sym:
    """Symmetry of W implied by those of U and V (proof of Sec. 2.3).

    The two delta factors that survive the proof, delta(1) on (I, Q) and
    delta(3) on (J, Q), combine into sum c^U_I I - sigma sum c^V_J J ==
    Z^U - sigma Z^V.  Coefficients are listed in W's mode order.
    """
    tu, tv, tw, I, K, J = parse_einsum(sub)
    sigma = contracted_sign_ratio(sub, su, sv)
    g = su.group
    signs, dims, tables, hs = [], [], [], []
    for m in tw:
        if m in I:
            signs.append(su.signs[tu.index(m)])
            dims.append(su.dims[tu.index(m)])
            tables.append(su.table(tu.index(m)))
            hs.append(su.H(tu.index(m)))
        else:
            signs.append(-sigma * sv.signs[tv.index(m)])
            dims.append(sv.dims[tv.index(m)])
            tables.append(sv.table(tv.index(m)))
            hs.append(sv.H(tv.index(m)))
    charge = g.sub(su.charge, g.times(sigma, sv.charge))
    return Sym.make(tuple(signs), charge, tuple(dims), g, tables, hs)


def same_symmetry(a: Sym, b: Sym) -> bool:
    """(c, Z) and (-c, -Z) state the same rule and give the same reduced layout."""
    if a.dims != b.dims or a.group.orders != b.group.orders or a.sectors != b.sectors:
        return False
    if any(a.table(m) != b.table(m) for m in range(a.order)):
        return False
    if a.signs == b.signs and a.charge == b.charge:
        return True
    return tuple(-c for c in a.signs) == b.signs and a.group.neg(a.charge) == b.charge


def check_operands(sub, su: Sym, sv: Sym):
    tu, tv, tw, I, K, J = parse_einsum(sub)
    if len(tu) != su.order or len(tv) != sv.order:
        raise ValueError("term length does not match operand order")
    if not tw:
        raise ValueError("the output needs at least one mode")
    if su.group.orders != sv.group.orders:
        raise ValueError("operands use different groups")
    for k in K:
        if su.dims[tu.index(k)] != sv.dims[tv.index(k)]:
            raise ValueError(f"contracted mode {k} has different block sizes")
        if su.table(tu.index(k)) != sv.table(tv.index(k)):
            raise ValueError(f"contracted mode {k} has different charge tables")
        if su.H(tu.index(k)) != sv.H(tv.index(k)):
            raise ValueError(f"contracted mode {k} has different sector counts")
    return tu, tv, tw, I, K, J


def flop_count(sub, su: Sym, sv: Sym) -> int:
    """Multiply-adds x 2 over allowed block products only: 2 n^(s+t+v) G^(s+t+v-2) (Alg. 2, product step)."""
    tu, tv, tw, I, K, J = check_operands(sub, su, sv)
    n = 1
    for m in I + K:
        n *= su.dims[tu.index(m)]
    for m in J:
        n *= sv.dims[tv.index(m)]
    s, v, t = len(I), len(K), len(J)
    if su.sectors is None and sv.sectors is None:
        return 2 * n * su.group.size ** (s + t + v - 2)
    # subgroup modes: count the pairs of allowed U and V blocks that meet
    hs = {m: su.H(tu.index(m)) for m in I + K}
    hs.update({m: sv.H(tv.index(m)) for m in J})
    pairs = 0
    for secs in itertools.product(*[range(hs[m]) for m in I + K + J]):
        sec = dict(zip(I + K + J, secs))
        if allowed(su, [sec[m] for m in tu]) and allowed(sv, [sec[m] for m in tv]):
            pairs += 1
    return 2 * n * pairs


# ----------------------------------------------------------------------------
# Form 1: dense
# ----------------------------------------------------------------------------
def contract_dense(sub, Ru, su: Sym, Rv, sv: Sym):
    """Returns (R_W, sym_W, zero_ok): dense einsum of the expanded operands, reduced."""
    check_operands(sub, su, sv)
    sw = output_symmetry(sub, su, sv)
    Wf = np.einsum(sub, expand(Ru, su), expand(Rv, sv), optimize=True)
    Rw, zero_ok = reduce_full(Wf, sw)
    return Rw, sw, zero_ok


# ----------------------------------------------------------------------------
# Form 2: loop over symmetry blocks (Alg. 1, any s, t, v)
# ----------------------------------------------------------------------------
def contract_blocks(sub, Ru, su: Sym, Rv, sv: Sym, u_blocks=None):
    """Loop over every stored block of U and every free J-sector choice.

    For each stored block of U the sectors of all U modes follow from U's rule;
    the sectors of J except its last one are looped over, and the last one
    follows from V's rule (the role of J = A+B-I and L = A+B-K in Alg. 1).
    ``u_blocks`` optionally restricts the outer loop to the listed stored
    sector tuples of U (a sample of the full loop).
    """
    tu, tv, tw, I, K, J = check_operands(sub, su, sv)
    sw = output_symmetry(sub, su, sv)
    g = su.group
    G = g.size
    dt = _ftype(Ru, Rv)
    Ru = np.asarray(Ru, dtype=dt)
    Rv = np.asarray(Rv, dtype=dt)
    Rw = np.zeros(sw.reduced_shape(), dtype=dt)
    inner_sub = sub.replace(" ", "")
    outer = stored_tuples(su) if u_blocks is None else u_blocks
    for ustored in outer:
        ustored = tuple(ustored)
        usec = full_sectors(su, ustored)
        if usec is None:
            continue
        sec = {m: usec[p] for p, m in enumerate(tu)}
        for jfree in itertools.product(*[range(sv.H(tv.index(m))) for m in J[:-1]]):
            for m, e in zip(J[:-1], jfree):
                sec[m] = e
            if J:
                # last J sector from V's conservation rule, solved at its position in V
                known = [sec[m] for m in tv if m != J[-1]]
                sec[J[-1]] = implicit_sector(sv, known, position=tv.index(J[-1]))
                if sec[J[-1]] is None:
                    continue
            vsec = tuple(sec[m] for m in tv)
            wsec = tuple(sec[m] for m in tw)
            if not allowed(sv, vsec):
                # only with t = 0: V's rule then constrains U's contracted sectors
                assert not J
                continue
            assert allowed(sw, wsec)
            blk = np.einsum(inner_sub, Ru[ustored], Rv[vsec[:-1]], optimize=True)
            Rw[wsec[:-1]] += blk
    return Rw, sw


# ----------------------------------------------------------------------------
# Form 3: sampled brute force
# ----------------------------------------------------------------------------
def _vector_allowed(sym: Sym, secs):
    """Vectorised conservation test; secs is a list of int arrays (one per mode)."""
    g = sym.group
    shape = np.broadcast(*secs).shape
    ok = np.ones(shape, dtype=bool)
    chg = [np.asarray(sym.table(m), dtype=np.int64)[np.asarray(s)] for m, s in enumerate(secs)]
    stride = 1
    for o in reversed(g.orders):
        tot = np.zeros(shape, dtype=np.int64)
        for c, s in zip(sym.coefs, chg):
            tot += c * ((s // stride) % o)
        ok &= (tot - (sym.charge // stride) % o) % o == 0
        stride *= o
    return ok


def sample_contract(sub, su: Sym, sv: Sym, u_values, v_values, w_full_positions, dtype=np.float64):
    """W at the given full positions, each summed over every contracted full index.

    ``u_values(stored_sectors, inner)`` / ``v_values`` return operand values at
    reduced-form coordinates (lists of int arrays, sectors of modes 0..N-2 then
    the N in-block indices).  Each term's factors are looked up through the
    conservation rule, so disallowed entries contribute exactly zero; nothing
    else about the symmetry is used.  ``w_full_positions`` is an int array of
    shape (S, order_W); ``dtype`` is float64 or complex128.
    """
    tu, tv, tw, I, K, J = check_operands(sub, su, sv)
    kdims = [su.H(tu.index(k)) * su.dims[tu.index(k)] for k in K]
    grids = np.meshgrid(*[np.arange(d, dtype=np.int64) for d in kdims], indexing="ij")
    kfull = {k: gr.ravel() for k, gr in zip(K, grids)}
    out = np.zeros(len(w_full_positions), dtype=dtype)
    for s, pos in enumerate(np.asarray(w_full_positions, dtype=np.int64)):
        wfull = {m: int(x) for m, x in zip(tw, pos)}

        def gather(t, sym, fn):
            full = [np.full_like(kfull[K[0]], wfull[m]) if m in wfull else kfull[m] for m in t]
            secs = [x // n for x, n in zip(full, sym.dims)]
            inner = [x % n for x, n in zip(full, sym.dims)]
            ok = _vector_allowed(sym, secs)
            vals = np.zeros(ok.shape, dtype=dtype)
            idx = np.nonzero(ok)[0]
            if idx.size:
                vals[idx] = fn([x[idx] for x in secs[:-1]], [x[idx] for x in inner])
            return vals

        uv = gather(tu, su, u_values)
        vv = gather(tv, sv, v_values)
        out[s] = np.dot(uv, vv)
    return out


def sample_contract_allowed(sub, su: Sym, sv: Sym, u_values, v_values, w_full_positions,
                            dtype=np.float64, chunk: int = 1 << 20):
    """W at the given full positions, summed over the allowed contracted sectors only.

    The same sum as ``sample_contract`` (Eq. ctr at one output element) with its
    zero terms left out: an output element fixes the sectors of I and J; every
    contracted sector but the last is free, the last one follows from U's rule
    (no solution: no term), and V's rule must then hold as well (Eq. symtsr for
    both factors).  Each surviving sector tuple adds the dot product of the two
    factors over the contracted in-block indices.  The cost per element is the
    number of nonzero terms rather than every contracted full index, so
    thousands of elements of a large contraction can be checked.
    ``u_values`` / ``v_values`` are value functions as for ``sample_contract``.
    """
    tu, tv, tw, I, K, J = check_operands(sub, su, sv)
    pos = np.asarray(w_full_positions, dtype=np.int64).reshape(-1, len(tw))
    S = len(pos)
    out = np.zeros(S, dtype=dtype)
    if S == 0:
        return out
    sec, inn = {}, {}
    for c, m in enumerate(tw):
        n = su.dims[tu.index(m)] if m in tu else sv.dims[tv.index(m)]
        sec[m] = pos[:, c] // n
        inn[m] = pos[:, c] % n
    kdims = [su.dims[tu.index(k)] for k in K]
    nk = math.prod(kdims)
    kin = dict(zip(K, np.unravel_index(np.arange(nk, dtype=np.int64), kdims))) if K else {}
    # (sample, contracted sectors) of every nonzero term
    terms_s, terms_k = [], []
    free = [range(su.H(tu.index(k))) for k in K[:-1]]
    for s in range(S):
        for ks in itertools.product(*free):
            ksec = dict(zip(K[:-1], ks))
            if K:
                p = tu.index(K[-1])
                known = [int(sec[m][s]) if m in sec else ksec[m] for m in tu if m != K[-1]]
                last = implicit_sector(su, known, position=p)
                if last is None:
                    continue
                ksec[K[-1]] = last
            usec = [int(sec[m][s]) if m in sec else ksec[m] for m in tu]
            vsec = [int(sec[m][s]) if m in sec else ksec[m] for m in tv]
            if not (allowed(su, usec) and allowed(sv, vsec)):
                continue
            terms_s.append(s)
            terms_k.append(tuple(ksec[k] for k in K))
    if not terms_s:
        return out
    terms_s = np.asarray(terms_s, dtype=np.int64)
    terms_k = np.asarray(terms_k, dtype=np.int64).reshape(len(terms_s), len(K))
    per = max(1, chunk // max(nk, 1))
    for lo in range(0, len(terms_s), per):
        ts = terms_s[lo:lo + per]
        tk = terms_k[lo:lo + per]
        T = len(ts)

        def coords(term, sym, fn):
            secs, inner = [], []
            for m in term:
                if m in sec:
                    secs.append(np.repeat(sec[m][ts], nk))
                    inner.append(np.repeat(inn[m][ts], nk))
                else:
                    secs.append(np.repeat(tk[:, K.index(m)], nk))
                    inner.append(np.tile(kin[m], T))
            return fn(secs[:-1], inner).reshape(T, nk)

        uv = coords(tu, su, u_values)
        vv = coords(tv, sv, v_values)
        np.add.at(out, ts, np.sum(uv * vv, axis=1))
    return out


def reduced_value_fn(R, sym: Sym):
    """A value function (for sample_contract) backed by a stored reduced-form array."""
    R = np.asarray(R)

    def fn(secs, inner):
        return R[tuple(secs) + tuple(inner)]
    return fn


# ----------------------------------------------------------------------------
# Form 4: pure-Python brute force
# ----------------------------------------------------------------------------
def contract_bruteforce(sub, Ru, su: Sym, Rv, sv: Sym):
    """Eq. ctr summed over every full index, one scalar at a time (tiny inputs only)."""
    tu, tv, tw, I, K, J = check_operands(sub, su, sv)
    sw = output_symmetry(sub, su, sv)
    size = {}
    for t, sym in ((tu, su), (tv, sv)):
        for p, m in enumerate(t):
            size[m] = sym.H(p) * sym.dims[p]
    Wf = np.zeros(tuple(size[m] for m in tw), dtype=_ftype(Ru, Rv))
    for wi in itertools.product(*[range(size[m]) for m in tw]):
        idx = dict(zip(tw, wi))
        acc = 0.0
        for ki in itertools.product(*[range(size[m]) for m in K]):
            idx.update(zip(K, ki))
            a = lookup(Ru, su, tuple(idx[m] for m in tu))
            b = lookup(Rv, sv, tuple(idx[m] for m in tv))
            acc += a * b
        Wf[wi] = acc
    Rw, zero_ok = reduce_full(Wf, sw)
    return Rw, sw, zero_ok


# ----------------------------------------------------------------------------
# Form 5: Alg. 2 with dense generalized Kronecker deltas
# ----------------------------------------------------------------------------
def kron_delta(group: Group, coefs, q_coef, remainder, tables=None, radices=None):
    """Dense 0/1 tensor over (sector labels..., Q): 1 iff sum coefs*chi(S) + q_coef*Q == remainder.

    ``tables`` gives each sector axis's charge table (identity when absent);
    ``radices`` each sector axis's number of sectors (|G| when absent); the Q
    axis is a charge, |G| values.
    """
    G = group.size
    p = len(coefs)
    tables = tables or [tuple(range(G))] * p
    radices = list(radices) if radices is not None else [G] * p
    D = np.zeros(tuple(radices) + (G,), dtype=np.float64)
    for secs in itertools.product(*[range(r) for r in radices], range(G)):
        chg = [tables[a][x] for a, x in enumerate(secs[:-1])] + [secs[-1]]
        if group.total(list(coefs) + [q_coef], chg) == remainder:
            D[secs] = 1.0
    return D


def _full_sector_form(R, sym: Sym):
    """Order-2N array [S_0..S_{N-1}, i_0..i_{N-1}]: the reduced form times its delta (Eq. redform)."""
    N = sym.order
    # the operand's own delta over all N sector labels: 1 where the rule holds
    Dt = np.zeros(tuple(sym.H(m) for m in range(N)), dtype=np.float64)
    for secs in itertools.product(*[range(sym.H(m)) for m in range(N)]):
        if allowed(sym, secs):
            Dt[secs] = 1.0
    letters = _letters(2 * N)
    S, inner = letters[:N], letters[N:]
    return np.einsum(f"{''.join(S[:-1])}{''.join(inner)},{''.join(S)}->{''.join(S)}{''.join(inner)}",
                     np.asarray(R, dtype=_ftype(R)), Dt)


def _letters(n, skip=""):
    pool = [c for c in "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ" if c not in skip]
    if n > len(pool):
        raise ValueError("too many modes for the dense-delta reference")
    return pool[:n]


def alignment_deltas(sub, su: Sym, sv: Sym):
    """delta(1) on (I, Q), delta(2) on (K, Q), delta(3) on (J, Q) (Alg. 2, coefficient and delta steps).

    Q is the sum of the contracted sectors weighted by U's coefficients
    (delta(2): sum c^U_K K - Q == 0).  delta(1): sum c^U_I I + Q == Z^U.
    delta(3): sum c^V_J J + sigma Q == Z^V, which is Alg. 2's coefficient
    vector c^(C) when sigma = +1 and its sign-flipped form otherwise.
    """
    tu, tv, tw, I, K, J = check_operands(sub, su, sv)
    sigma = contracted_sign_ratio(sub, su, sv)
    g = su.group
    d1 = kron_delta(g, [su.coef(tu.index(m)) for m in I], +1, su.charge, [su.table(tu.index(m)) for m in I],
                    [su.H(tu.index(m)) for m in I])
    d2 = kron_delta(g, [su.coef(tu.index(m)) for m in K], -1, 0, [su.table(tu.index(m)) for m in K],
                    [su.H(tu.index(m)) for m in K])
    d3 = kron_delta(g, [sv.coef(tv.index(m)) for m in J], sigma, sv.charge, [sv.table(tv.index(m)) for m in J],
                    [sv.H(tv.index(m)) for m in J])
    return d1, d2, d3


def _align_operand(Rfs, t, sym: Sym, row_modes, col_modes, d_row, d_col):
    """Sum a full-sector operand against the row- and column-group deltas (Alg. 2, aligned-operand step).

    Output layout: [Q][row sectors but the last][row inner dims][col sectors
    but the last][col inner dims], reshaped to (|G|, M, Kc).
    """
    G = sym.group.size
    N = len(t)
    L = _letters(2 * N + 1)
    S = {m: L[p] for p, m in enumerate(t)}
    inner = {m: L[N + p] for p, m in enumerate(t)}
    q = L[2 * N]
    src = "".join(S[m] for m in t) + "".join(inner[m] for m in t)
    drow = "".join(S[m] for m in row_modes) + q
    dcol = "".join(S[m] for m in col_modes) + q
    out = (q + "".join(S[m] for m in row_modes[:-1]) + "".join(inner[m] for m in row_modes)
           + "".join(S[m] for m in col_modes[:-1]) + "".join(inner[m] for m in col_modes))
    A = np.einsum(f"{src},{drow},{dcol}->{out}", Rfs, d_row, d_col, optimize=True)
    # an empty group (s, t or v = 0) has one row or column; its delta pins Q
    nrow = int(np.prod([sym.H(t.index(m)) for m in row_modes[:-1]] + [sym.dims[t.index(m)] for m in row_modes]))
    ncol = int(np.prod([sym.H(t.index(m)) for m in col_modes[:-1]] + [sym.dims[t.index(m)] for m in col_modes]))
    return A.reshape(G, nrow, ncol)


def align_u(sub, Ru, su: Sym, sv: Sym):
    tu, tv, tw, I, K, J = check_operands(sub, su, sv)
    d1, d2, d3 = alignment_deltas(sub, su, sv)
    return _align_operand(_full_sector_form(Ru, su), tu, su, I, K, d1, d2)


def align_v(sub, Rv, su: Sym, sv: Sym):
    tu, tv, tw, I, K, J = check_operands(sub, su, sv)
    d1, d2, d3 = alignment_deltas(sub, su, sv)
    return _align_operand(_full_sector_form(Rv, sv), tv, sv, K, J, d2, d3)


def unalign_w(sub, Wal, su: Sym, sv: Sym):
    """Aligned output (|G|, M, N) -> standard reduced form of W (Alg. 2 final step)."""
    tu, tv, tw, I, K, J = check_operands(sub, su, sv)
    sw = output_symmetry(sub, su, sv)
    d1, d2, d3 = alignment_deltas(sub, su, sv)
    G = su.group.size
    NW = len(tw)
    dims = {m: sw.dims[p] for p, m in enumerate(tw)}
    hs = {m: sw.H(p) for p, m in enumerate(tw)}
    A = np.asarray(Wal).reshape((G,) + tuple(hs[m] for m in I[:-1]) + tuple(dims[m] for m in I)
                                + tuple(hs[m] for m in J[:-1]) + tuple(dims[m] for m in J))
    L = _letters(2 * NW + 1)
    S = {m: L[p] for p, m in enumerate(tw)}
    inner = {m: L[NW + p] for p, m in enumerate(tw)}
    q = L[2 * NW]
    src = (q + "".join(S[m] for m in I[:-1]) + "".join(inner[m] for m in I)
           + "".join(S[m] for m in J[:-1]) + "".join(inner[m] for m in J))
    d1s = "".join(S[m] for m in I) + q
    d3s = "".join(S[m] for m in J) + q
    full = "".join(S[m] for m in tw) + "".join(inner[m] for m in tw)
    Wfs = np.einsum(f"{src},{d1s},{d3s}->{full}", A, d1, d3, optimize=True)
    # drop the last sector axis: exactly one of its values is allowed per stored tuple
    return Wfs.sum(axis=NW - 1), sw


def contract_irrep_aligned(sub, Ru, su: Sym, Rv, sv: Sym):
    """Alg. 2 end to end; returns (R_W, sym_W, U_al, V_al, W_al)."""
    Ual = align_u(sub, Ru, su, sv)
    Val = align_v(sub, Rv, su, sv)
    Wal = np.matmul(Ual, Val)           # Alg. 2's product step, one product per Q
    Rw, sw = unalign_w(sub, Wal, su, sv)
    return Rw, sw, Ual, Val, Wal


def aligned_shape(sub, su: Sym, sv: Sym):
    """(|G|, M, K, N) of the aligned product: M = G^(s-1) n_I, K = G^(v-1) n_K, N = G^(t-1) n_J."""
    tu, tv, tw, I, K, J = check_operands(sub, su, sv)
    G = su.group.size
    nI = math.prod(su.dims[tu.index(m)] for m in I)
    nK = math.prod(su.dims[tu.index(m)] for m in K)
    nJ = math.prod(sv.dims[tv.index(m)] for m in J)
    hI = math.prod(su.H(tu.index(m)) for m in I[:-1])
    hK = math.prod(su.H(tu.index(m)) for m in K[:-1])
    hJ = math.prod(sv.H(tv.index(m)) for m in J[:-1])
    return (G, hI * nI, hK * nK, hJ * nJ)


# ----------------------------------------------------------------------------
# bfloat16 hi/lo split (the split-precision product form)
# ----------------------------------------------------------------------------
def bf16_round(x32):
    """Round binary32 values to the nearest bfloat16 (ties to even), returned as binary32."""
    b = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)


def bf16_split(x32):
    """hi = bf16(x), lo = bf16(x - hi); x - hi is exact in binary32."""
    x32 = np.asarray(x32, dtype=np.float32)
    hi = bf16_round(x32)
    lo = bf16_round(x32 - hi)
    return hi, lo
