"""The five synthetic workloads: group, einsum strings, signs, block sizes, value laws.

Pure data.  A tensor with cyclic (or product-of-cyclic) group symmetry is
described by its sign string (coefficient +1 or -1 per mode), its total charge
Z, and its block (inner) dimension per mode; every mode has |G| sectors.  The
stored array is the standard reduced form: sector axes of modes 0..N-2, then
the inner axes of all N modes, row-major (the layout of the paper's API
example, Sec. 3).  Values come from ``synth.philox`` keyed by
(seed, tensor id).

Workloads (shapes taken from the paper's coupled-cluster and tensor-network
contractions, Sec. 4 and Table 2); ``paper_suite_case`` gives the twelve
Table 2 cases of the Table 1 contractions (MM, CC1-3, MPS, PEPS):

* ``plain_z4``      w_abij = sum_kl u_abkl v_klij, Z_4, every block dim 4.
* ``ccd_ladder_z8`` w_abij = sum_cd V_abcd T_cdij, Z_8, virtual 24, occupied 6.
* ``mps_env_z2z3``  E'_{a'b'c'} = E_abc A_{a s a'} W_{b s s' b'} A_{c s' c'},
                    Z_2 x Z_3, bond 64, MPO bond 4, physical 2, contracted
                    pairwise left to right.
* ``ccd_ladder_z16`` the ladder at Z_16, virtual 32, occupied 8.
* ``mps_env_grad``  the environment chain at bond 128 with L = <E', R>.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from .philox import DIST_NORMAL, DIST_UNIFORM

DEFAULT_SEED = 20070805


@dataclass(frozen=True)
class Operand:
    name: str
    modes: str            # one letter per mode, einsum order
    signs: str            # '+' / '-' per mode
    charge: int           # total charge Z as a flattened group element
    dims: tuple           # block dimension per mode
    dist: int = DIST_UNIFORM
    scale: float = 1.0
    tensor_id: int = 0
    sectors: tuple | None = None   # sectors per mode (a divisor of |G|); None: |G| each

    @property
    def order(self) -> int:
        return len(self.modes)


@dataclass(frozen=True)
class Contraction:
    einsum: str           # "u,v->w" over mode letters
    u: str                # operand names
    v: str
    w: str


@dataclass(frozen=True)
class Workload:
    name: str
    group: tuple          # cyclic factor orders, e.g. (8,) or (2, 3)
    operands: dict        # name -> Operand (inputs and derived outputs)
    steps: tuple          # Contraction steps, executed in order
    inputs: tuple         # names of generated inputs
    output: str
    seed: int = DEFAULT_SEED
    extra: dict = field(default_factory=dict)

    @property
    def group_size(self) -> int:
        g = 1
        for o in self.group:
            g *= o
        return g

    def reduced_shape(self, name: str) -> tuple:
        op = self.operands[name]
        hs = op.sectors or (self.group_size,) * op.order
        return tuple(hs[: op.order - 1]) + tuple(op.dims)


def _ladder(name, G, nv, no, cid, h_ab=None):
    # h_ab: sectors of the external virtual modes a, b (a subgroup of Z_G), or all |G|
    sv = (h_ab, h_ab, G, G) if h_ab else None
    sw = (h_ab, h_ab, G, G) if h_ab else None
    ops = {
        "V": Operand("V", "abcd", "++--", 0, (nv, nv, nv, nv), DIST_NORMAL, 1.0, cid * 16 + 0, sv),
        "T": Operand("T", "cdij", "++--", 0, (nv, nv, no, no), DIST_NORMAL, 1e-2, cid * 16 + 1),
        "W": Operand("W", "abij", "++--", 0, (nv, nv, no, no), sectors=sw),
    }
    return Workload(name, (G,), ops, (Contraction("abcd,cdij->abij", "V", "T", "W"),),
                    ("V", "T"), "W")


def plain_z4() -> Workload:
    n = 4
    ops = {
        "u": Operand("u", "abkl", "++--", 0, (n, n, n, n), DIST_UNIFORM, 1.0, 0),
        "v": Operand("v", "klij", "++--", 0, (n, n, n, n), DIST_UNIFORM, 1.0, 1),
        "w": Operand("w", "abij", "++--", 0, (n, n, n, n)),
    }
    return Workload("plain_z4", (4,), ops, (Contraction("abkl,klij->abij", "u", "v", "w"),),
                    ("u", "v"), "w")


def ccd_ladder_z8() -> Workload:
    return _ladder("ccd_ladder_z8", 8, 24, 6, 1)


def ccd_ladder_z8_sub() -> Workload:
    """The Z_8 ladder with a and b in the Z_4 subgroup (4 sectors, coefficient 2)."""
    return _ladder("ccd_ladder_z8_sub", 8, 24, 6, 5, h_ab=4)


def ccd_ladder_z16() -> Workload:
    return _ladder("ccd_ladder_z16", 16, 32, 8, 3)


def _mps_env(name, bond, cid, with_r):
    """E (a-,b-,c-), A (a+,s+,A-), W (b+,s-,S-,B-); every charge 0.

    Every contracted pair carries opposite signs.  The intermediates are
    T1_{bcsA} (-,-,+,-), T2_{cASB} (-,-,-,-) and E'_{ABC} (-,-,-).
    """
    nb, nw, ns = bond, 4, 2
    ops = {
        "E": Operand("E", "abc", "---", 0, (nb, nw, nb), DIST_UNIFORM, 1.0, cid * 16 + 0),
        "A": Operand("A", "asA", "++-", 0, (nb, ns, nb), DIST_UNIFORM, 1.0, cid * 16 + 1),
        "W": Operand("W", "bsSB", "+---", 0, (nw, ns, ns, nw), DIST_UNIFORM, 1.0, cid * 16 + 2),
        "T1": Operand("T1", "bcsA", "--+-", 0, (nw, nb, ns, nb)),
        "T2": Operand("T2", "cASB", "----", 0, (nb, nb, ns, nw)),
        "Ep": Operand("Ep", "ABC", "---", 0, (nb, nw, nb)),
    }
    inputs = ("E", "A", "W")
    if with_r:
        ops["R"] = Operand("R", "ABC", "---", 0, (nb, nw, nb), DIST_NORMAL, 1.0, cid * 16 + 3)
        inputs = inputs + ("R",)
    steps = (
        Contraction("abc,asA->bcsA", "E", "A", "T1"),
        Contraction("bcsA,bsSB->cASB", "T1", "W", "T2"),
        Contraction("cASB,cSC->ABC", "T2", "A", "Ep"),
    )
    return Workload(name, (2, 3), ops, steps, inputs, "Ep")


def mps_env_z2z3() -> Workload:
    return _mps_env("mps_env_z2z3", 64, 2, False)


def mps_env_grad() -> Workload:
    return _mps_env("mps_env_grad", 128, 4, True)


# ---------------------------------------------------------------------------
# The paper's benchmark suite (Table 1 contractions at Table 2 dimensions).
# Block dimension per mode letter as in Table 2; signs are not given there and
# are read as: every contracted pair carries opposite signs, and each operand's
# signs sum to zero over its modes where the order allows (CC tensors ++--,
# matrices +-, MPS tensors ++-); charges 0; values uniform in [-1, 1).
# ---------------------------------------------------------------------------
_SUITE = {
    # label: (G, einsum, u signs, v signs, derived w signs, block dim per letter)
    "cc1a": (8, "ijkl,mnkl->ijmn", "++--", "--++", "++--", dict(i=32, j=32, k=32, l=32, m=16, n=16)),
    "cc2a": (8, "opij,opkm->ijmk", "++--", "--++", "--++", dict(i=32, j=32, k=32, m=16, o=16, p=16)),
    "cc3a": (8, "opmn,opij->ijmn", "++--", "--++", "++--", dict(i=32, j=32, m=16, n=16, o=16, p=16)),
    "cc1b": (16, "ijkl,mnkl->ijmn", "++--", "--++", "++--", dict(i=16, j=16, k=16, l=16, m=8, n=8)),
    "cc2b": (16, "opij,opkm->ijmk", "++--", "--++", "--++", dict(i=16, j=16, k=16, m=8, o=8, p=8)),
    "cc3b": (16, "opmn,opij->ijmn", "++--", "--++", "++--", dict(i=16, j=16, m=8, n=8, o=8, p=8)),
    "mma": (2, "ij,jk->ik", "+-", "+-", "+-", dict(i=10000, j=10000, k=10000)),
    "mmb": (100, "ij,jk->ik", "+-", "+-", "+-", dict(i=2000, j=2000, k=2000)),
    "mpsa": (2, "ijk,klm->ijlm", "++-", "++-", "+++-", dict(i=3000, j=10, k=3000, l=1, m=3000)),
    "mpsb": (5, "ijk,klm->ijlm", "++-", "++-", "+++-", dict(i=700, j=10, k=700, l=1, m=700)),
    "pepsa": (2, "ijkl,klmn->ijmn", "++--", "++--", "++--", dict(i=400, j=400, k=20, l=20, m=20, n=20)),
    "pepsb": (10, "ijkl,klmn->ijmn", "++--", "++--", "++--", dict(i=64, j=64, k=8, l=8, m=8, n=8)),
}


def paper_suite_case(label: str, dims: dict | None = None) -> Workload:
    """One Table 2 case (``dims`` overrides block dimensions, for small test copies)."""
    G, sub, su, sv, sw, d = _SUITE[label]
    d = dict(d, **(dims or {}))
    tu, rest = sub.split(",")
    tv, tw = rest.split("->")
    cid = 32 + sorted(_SUITE).index(label)
    ops = {
        "U": Operand("U", tu, su, 0, tuple(d[m] for m in tu), DIST_UNIFORM, 1.0, cid * 16 + 0),
        "V": Operand("V", tv, sv, 0, tuple(d[m] for m in tv), DIST_UNIFORM, 1.0, cid * 16 + 1),
        "W": Operand("W", tw, sw, 0, tuple(d[m] for m in tw)),
    }
    return Workload("suite_" + label, (G,), ops, (Contraction(sub, "U", "V", "W"),), ("U", "V"), "W")


SUITE_LABELS = tuple(_SUITE)


# ---------------------------------------------------------------------------
# The paper's generic-contraction sweep (Sec. 4): (s, t, v) free and contracted
# mode counts at G = 4, every mode's block dimension N chosen so that the
# contraction costs 80 GFLOP (2 N^(s+t+v) G^(s+t+v-2), N rounded to the nearest
# integer).  Which (s, t, v) the paper plotted is not recoverable; these are
# every pattern with s, t, v in 1..3 and s + t + v <= 6, plus the three
# one-sided order-5 patterns.  Signs: U's free modes +, its contracted modes -;
# V's contracted modes + (opposite to U's), its free modes -; charges 0.
# ---------------------------------------------------------------------------
STV_CASES = ((1, 1, 1), (2, 1, 1), (1, 2, 1), (1, 1, 2), (2, 2, 1), (2, 1, 2), (1, 2, 2),
             (2, 2, 2), (3, 1, 1), (1, 3, 1), (1, 1, 3))


def stv_case(s: int, t: int, v: int, G: int = 4, total_flops: float = 80e9, n: int | None = None) -> Workload:
    """W[I,J] = sum_K U[I,K] V[K,J] with s, t, v modes of block dimension N (``n`` overrides)."""
    order = s + t + v
    if n is None:
        n = max(1, round((total_flops / 2.0 / G ** (order - 2)) ** (1.0 / order)))
    letters = "abcdefghijklmnop"
    I, K, J = letters[:s], letters[s:s + v], letters[s + v:s + v + t]
    tu, tv, tw = I + K, K + J, I + J
    ops = {
        "U": Operand("U", tu, "+" * s + "-" * v, 0, (n,) * len(tu), DIST_UNIFORM, 1.0, 600 + 16 * (9 * s + 3 * t + v)),
        "V": Operand("V", tv, "+" * v + "-" * t, 0, (n,) * len(tv), DIST_UNIFORM, 1.0,
                     601 + 16 * (9 * s + 3 * t + v)),
        # derived: c^W = (c^U_I, -sigma c^V_J) with sigma = -1
        "W": Operand("W", tw, "+" * s + "-" * t, 0, (n,) * len(tw)),
    }
    return Workload(f"stv_{s}{t}{v}", (G,), ops, (Contraction(f"{tu},{tv}->{tw}", "U", "V", "W"),), ("U", "V"), "W")


# ---------------------------------------------------------------------------
# The paper's sensitivity-to-G sweeps (Sec. 4): MM with N = 500 over G = 4..12,
# CC1 over G = 4..12 and PEPS over G = 2..10.  The CC1 dimensions are printed
# for eight mode letters of a six-mode contraction; read as U's four modes
# i, j, k, l at 8 and V's free modes m, n at 16.  PEPS: the boundary-MPS
# bonds i, j at 16, the PEPS bonds k, l, m, n at 4.  Signs as in the suite.
# ---------------------------------------------------------------------------
G_SWEEP = {"mm": tuple(range(4, 13)), "cc1": tuple(range(4, 13)), "peps": tuple(range(2, 11))}
_G_SWEEP_SHAPES = {
    "mm": ("ij,jk->ik", "+-", "+-", "+-", dict(i=500, j=500, k=500)),
    "cc1": ("ijkl,mnkl->ijmn", "++--", "--++", "++--", dict(i=8, j=8, k=8, l=8, m=16, n=16)),
    "peps": ("ijkl,klmn->ijmn", "++--", "++--", "++--", dict(i=16, j=16, k=4, l=4, m=4, n=4)),
}


def g_sweep_case(family: str, G: int, dims: dict | None = None) -> Workload:
    """One point of a G sweep (``dims`` overrides block dimensions, for small test copies)."""
    sub, su, sv, sw, d = _G_SWEEP_SHAPES[family]
    d = dict(d, **(dims or {}))
    tu, rest = sub.split(",")
    tv, tw = rest.split("->")
    cid = 700 + 16 * (3 * list(_G_SWEEP_SHAPES).index(family)) + G
    ops = {
        "U": Operand("U", tu, su, 0, tuple(d[m] for m in tu), DIST_UNIFORM, 1.0, cid * 16 + 0),
        "V": Operand("V", tv, sv, 0, tuple(d[m] for m in tv), DIST_UNIFORM, 1.0, cid * 16 + 1),
        "W": Operand("W", tw, sw, 0, tuple(d[m] for m in tw)),
    }
    return Workload(f"gsweep_{family}_{G}", (G,), ops, (Contraction(sub, "U", "V", "W"),), ("U", "V"), "W")


ALL = {
    "plain_z4": plain_z4,
    "ccd_ladder_z8": ccd_ladder_z8,
    "mps_env_z2z3": mps_env_z2z3,
    "ccd_ladder_z16": ccd_ladder_z16,
    "mps_env_grad": mps_env_grad,
    "ccd_ladder_z8_sub": ccd_ladder_z8_sub,
}


def get(name: str) -> Workload:
    return ALL[name]()


def scaled(wl: Workload, dims_map: dict) -> Workload:
    """A copy of a workload with some block dimensions replaced (for small test cases).

    ``dims_map`` maps a mode letter to its new block dimension; every operand
    carrying that letter changes consistently.
    """
    ops = {}
    for k, op in wl.operands.items():
        dims = tuple(dims_map.get(m, d) for m, d in zip(op.modes, op.dims))
        ops[k] = Operand(op.name, op.modes, op.signs, op.charge, dims, op.dist, op.scale, op.tensor_id,
                         op.sectors)
    return Workload(wl.name + "_scaled", wl.group, ops, wl.steps, wl.inputs, wl.output, wl.seed,
                    dict(wl.extra))
