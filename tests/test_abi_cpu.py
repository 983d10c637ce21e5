"""C-ABI checks that need no GPU: symbols, planner results, error codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import synth
from paper_2007_08056_amd import _lib as L
from tests.seeding import seed

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "symtensor.h")).read()
    declared = set(re.findall(r"\b(symtensor_\w+)\s*\(", header))
    assert declared == set(L.EXPORTED)
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def _desc(signs, charge, dims, dtype=L.SYMT_F64):
    return L.TensorDesc(signs, charge, dims, dtype, None)


def _plan(sub, group, u, v, w=None, compute=0):
    info = L.SymtPlanInfo()
    rc = L.LIB.symtensor_plan(sub.encode(), ctypes.byref(L.make_group(group)), u.ref, v.ref,
                              w.ref if w is not None else None, compute, ctypes.byref(info))
    return rc, info


@pytest.mark.parametrize("name", list(synth.configs.ALL))
def test_plan_matches_oracle_on_workloads(name):
    wl = synth.configs.get(name)
    g = O.Group(wl.group)
    for st in wl.steps:
        ou, ov, ow = (wl.operands[x] for x in (st.u, st.v, st.w))
        su = O.Sym.make(ou.signs, ou.charge, ou.dims, g, sectors=ou.sectors)
        sv = O.Sym.make(ov.signs, ov.charge, ov.dims, g, sectors=ov.sectors)
        rc, info = _plan(st.einsum, wl.group, _sdesc(ou.signs, ou.charge, ou.dims, ou.sectors),
                         _sdesc(ov.signs, ov.charge, ov.dims, ov.sectors),
                         _sdesc(ow.signs, ow.charge, ow.dims, ow.sectors))
        assert rc == 0, L.last_error()
        G, M, K, N = O.aligned_shape(st.einsum, su, sv)
        assert (info.group_size, info.m, info.k, info.n) == (G, M, K, N)
        assert info.flops == O.flop_count(st.einsum, su, sv)
        sw = O.output_symmetry(st.einsum, su, sv)
        assert info.w_signs.decode() == sw.sign_string() and info.w_charge == sw.charge
        assert info.elems_u == np.prod(su.reduced_shape())
        tu = st.einsum.split(",")[0]
        tv = st.einsum.split(",")[1].split("->")[0]
        k_modes = [m for m in tu if m in tv]
        trailing = tu.endswith("".join(k_modes))
        nK = int(np.prod([ou.dims[tu.index(m)] for m in k_modes]))
        whole = trailing and (nK % 16 == 0 or len(k_modes) == 1)
        no_sub = su.sectors is None and sv.sectors is None
        # whole K-steps read U in place on any tile; other layouts (K-major A, runs stepped one
        # by one) only where the product runs on register tiles, which the planner decides
        assert info.fused == 0 if not no_sub else (info.fused == 1 if whole else True)
        # W is written in place whenever no mode is a subgroup mode (real f64 operands here)
        assert info.fused_w == int(no_sub)
        G = info.group_size
        if info.fused:
            # V aligned plus four offset tables of U and W
            assert info.workspace_bytes >= 8 * info.elems_v + 8 * G * (2 * info.m + info.k + info.n)
            assert info.workspace_bytes < 8 * (info.elems_u + info.elems_v + info.elems_w)
        rc, steps = _plan(st.einsum, wl.group, _desc(ou.signs, ou.charge, ou.dims),
                          _desc(ov.signs, ov.charge, ov.dims), _desc(ow.signs, ow.charge, ow.dims),
                          compute=L.SYMT_FLAG_STEPS)
        assert rc == 0 and steps.fused == 0
        assert steps.workspace_bytes >= 8 * (info.elems_u + info.elems_v + info.elems_w)


def test_plan_matches_oracle_on_random_contractions():
    rng = np.random.default_rng(2)
    letters = "abcdefghij"
    for _ in range(200):
        orders = [(2,), (3,), (4,), (2, 3), (2, 2, 2)][rng.integers(5)]
        g = O.Group(orders)
        s, t, v = (int(x) for x in rng.integers(1, 4, 3))
        ls = list(letters[: s + t + v])
        I, K, J = ls[:s], ls[s:s + v], ls[s + v:]
        tu = list(I + K); rng.shuffle(tu)
        tv = list(K + J); rng.shuffle(tv)
        tw = list(I + J); rng.shuffle(tw)
        dims = {m: int(rng.integers(0, 4)) for m in ls}
        cu = {m: int(rng.choice([-1, 1])) for m in tu}
        sigma = int(rng.choice([-1, 1]))
        cv = {m: (sigma * cu[m] if m in K else int(rng.choice([-1, 1]))) for m in tv}
        su = O.Sym(tuple(cu[m] for m in tu), int(rng.integers(g.size)), tuple(dims[m] for m in tu), g)
        sv = O.Sym(tuple(cv[m] for m in tv), int(rng.integers(g.size)), tuple(dims[m] for m in tv), g)
        sub = f"{''.join(tu)},{''.join(tv)}->{''.join(tw)}"
        rc, info = _plan(sub, orders, _desc(su.sign_string(), su.charge, su.dims),
                         _desc(sv.sign_string(), sv.charge, sv.dims))
        assert rc == 0, L.last_error()
        assert (info.group_size, info.m, info.k, info.n) == O.aligned_shape(sub, su, sv)
        assert info.sigma == sigma and (info.s, info.t, info.v) == (s, t, v)
        sw = O.output_symmetry(sub, su, sv)
        assert info.w_signs.decode() == sw.sign_string() and info.w_charge == sw.charge
        # the globally flipped rule is accepted as W, anything else is not
        flip = "".join("+" if c == "-" else "-" for c in sw.sign_string())
        rc2, _ = _plan(sub, orders, _desc(su.sign_string(), su.charge, su.dims),
                       _desc(sv.sign_string(), sv.charge, sv.dims),
                       _desc(flip, g.neg(sw.charge), sw.dims))
        assert rc2 == 0
        if g.size > 2:
            rc3, _ = _plan(sub, orders, _desc(su.sign_string(), su.charge, su.dims),
                           _desc(sv.sign_string(), sv.charge, sv.dims),
                           _desc(sw.sign_string(), g.add(sw.charge, 1), sw.dims))
            assert rc3 == L.SYMT_ESYM


U4 = ("++--", 0, (2, 2, 2, 2))


@pytest.mark.parametrize("sub,code", [
    ("abkl,klij", L.SYMT_EEINSUM),            # no arrow
    ("abkl,klij->abij,x", L.SYMT_EEINSUM),
    ("aakl,klij->abij", L.SYMT_EEINSUM),      # repeated letter
    ("abkl,klaj->abj", L.SYMT_EEINSUM),       # 'a' in all three terms (batch)
    ("abkl,klij->abi", L.SYMT_EEINSUM),       # 'j' only in v (trace)
    ("abkl,klij->abijx", L.SYMT_EEINSUM),     # output letter in no input
    ("ab1l,klij->abij", L.SYMT_EEINSUM),      # not a letter
    ("abkl,abkl->", L.SYMT_EEINSUM),          # full contraction: s = t = 0
])
def test_einsum_errors(sub, code):
    rc, _ = _plan(sub, 4, _desc(*U4), _desc(*U4))
    assert rc == code, L.last_error()


def test_symmetry_and_size_errors():
    good = _desc(*U4)
    assert _plan("abkl,klij->abij", 4, good, good)[0] == 0
    # mixed sign ratio over the two contracted modes
    assert _plan("abkl,klij->abij", 4, good, _desc("+---", 0, (2, 2, 2, 2)))[0] == L.SYMT_ESYM
    # output rule not the derived one
    assert _plan("abkl,klij->abij", 4, good, good, _desc("++-+", 0, (2, 2, 2, 2)))[0] == L.SYMT_ESYM
    assert _plan("abkl,klij->abij", 4, good, good, _desc("++--", 1, (2, 2, 2, 2)))[0] == L.SYMT_ESYM
    # flipped output rule is the same rule
    assert _plan("abkl,klij->abij", 4, good, good, _desc("--++", 0, (2, 2, 2, 2)))[0] == 0
    # bad sign characters / length, charge out of range
    assert _plan("abkl,klij->abij", 4, _desc("++-x", 0, (2, 2, 2, 2)), good)[0] == L.SYMT_ESYM
    assert _plan("abkl,klij->abij", 4, _desc("++-", 0, (2, 2, 2)), good)[0] == L.SYMT_EINVAL
    assert _plan("abkl,klij->abij", 4, _desc("++--", 4, (2, 2, 2, 2)), good)[0] == L.SYMT_ESYM
    # contracted block sizes differ
    assert _plan("abkl,klij->abij", 4, good, _desc("++--", 0, (3, 2, 2, 2)))[0] == L.SYMT_EINVAL
    # output block sizes differ
    assert _plan("abkl,klij->abij", 4, good, good, _desc("++--", 0, (2, 2, 2, 3)))[0] == L.SYMT_EINVAL
    # negative dims, bad dtype, bad compute, bad group
    assert _plan("abkl,klij->abij", 4, _desc("++--", 0, (2, -1, 2, 2)), good)[0] == L.SYMT_EINVAL
    assert _plan("abkl,klij->abij", 4, _desc("++--", 0, (2, 2, 2, 2), dtype=7), good)[0] == L.SYMT_EDTYPE
    assert _plan("abkl,klij->abij", 4, good, good, compute=9)[0] == L.SYMT_EDTYPE
    assert _plan("abkl,klij->abij", 4, good, good, compute=0x200)[0] == L.SYMT_EDTYPE
    assert _plan("abkl,klij->abij", (0,), good, good)[0] == L.SYMT_EINVAL
    bad = L.SymtGroup()
    bad.nfactors = 5
    info = L.SymtPlanInfo()
    assert L.LIB.symtensor_plan(b"abkl,klij->abij", ctypes.byref(bad), good.ref, good.ref, None, 0,
                                ctypes.byref(info)) == L.SYMT_EINVAL


def test_null_arguments():
    info = L.SymtPlanInfo()
    g = L.make_group(4)
    good = _desc(*U4)
    assert L.LIB.symtensor_plan(None, ctypes.byref(g), good.ref, good.ref, None, 0, ctypes.byref(info)) == L.SYMT_EINVAL
    assert L.LIB.symtensor_plan(b"abkl,klij->abij", None, good.ref, good.ref, None, 0, ctypes.byref(info)) == L.SYMT_EINVAL
    assert L.LIB.symtensor_plan(b"abkl,klij->abij", ctypes.byref(g), None, good.ref, None, 0, ctypes.byref(info)) == L.SYMT_EINVAL
    assert L.LIB.symtensor_plan(b"abkl,klij->abij", ctypes.byref(g), good.ref, good.ref, None, 0, None) == L.SYMT_EINVAL
    assert L.last_error() != ""
    # context-taking calls reject a NULL context before touching the device
    assert L.LIB.symtensor_contract(None, b"abkl,klij->abij", ctypes.byref(g), good.ref, good.ref, good.ref,
                                    0, None, 0, None) == L.SYMT_EINVAL
    assert L.LIB.symtensor_sector_gemm(None, 0, 1, 1, 1, 1, None, None, None, None, 0, None) == L.SYMT_EINVAL
    assert L.LIB.symtensor_destroy(None) == 0


def test_workspace_sizes_per_compute_mode():
    u = _desc("++--", 0, (3, 3, 3, 3))
    v = _desc("++--", 0, (3, 3, 2, 2))
    sizes = {}
    for name, code in L.COMPUTE.items():
        for steps in (False, True):
            s = ctypes.c_size_t()
            assert L.LIB.symtensor_workspace_size(b"abcd,cdij->abij", ctypes.byref(L.make_group(4)), u.ref,
                                                  v.ref, None, code | (0x100 if steps else 0),
                                                  ctypes.byref(s)) == 0
            sizes[name, steps] = s.value
    eu, ev, ew = 4 ** 3 * 81, 4 ** 3 * 36, 4 ** 3 * 36
    r = lambda x: (x + 255) // 256 * 256  # noqa: E731
    # three steps: U_al | V_al | W_al
    assert sizes["f64", True] == r(8 * eu) + r(8 * ev) + r(8 * ew)
    assert sizes["f32", True] == r(4 * eu) + r(4 * ev) + r(4 * ew)
    # split-bf16 planes hold K (36 per Q here) at a pitch rounded up to 8: 40
    assert sizes["bf16x3", True] == r(4 * 4 * 36 * 40) + r(4 * 4 * 40 * 16) + r(8 * ew)
    # fused (the contracted block of 9 is stepped on its own; U and V read in place):
    # V_al, then row and column tables of U, W and V (M = K = 36, N = 16 per Q)
    tables = lambda rows, cols: r(8 * 4 * rows) + r(8 * 4 * cols)  # noqa: E731
    info = _plan("abcd,cdij->abij", 4, u, v, compute=L.COMPUTE["f64"])[1]
    assert info.fused == 1 and info.fused_v == 1
    assert sizes["f64", False] == r(8 * ev) + tables(36, 36) + tables(36, 16) + tables(36, 16)
    # binary64 operands under f32 compute (w not given, so taken in binary32): U is
    # aligned (converted) first, then U_al | V_al | tables of U_al, W
    info = _plan("abcd,cdij->abij", 4, u, v, compute=L.COMPUTE["f32"])[1]
    assert info.fused == 0 and info.fused_w == 1 and info.fused_v == 0
    assert sizes["f32", False] == r(4 * eu) + r(4 * ev) + tables(36, 36) + tables(36, 16)
    # with a binary64 w the product cannot write it: three steps
    w64 = _desc("++--", 0, (3, 3, 2, 2))
    info = _plan("abcd,cdij->abij", 4, u, v, w64, compute=L.COMPUTE["f32"])[1]
    assert info.fused == 0 and info.fused_w == 0 and info.workspace_bytes == sizes["f32", True]
    # split-bf16 (a contracted block of 9 is not whole 32-deep steps) writes W in place
    # only where W's columns come in runs of >= 16 (here 2 x 2): three steps
    info = _plan("abcd,cdij->abij", 4, u, v, compute=L.COMPUTE["bf16x3"])[1]
    assert info.fused == 0 and info.fused_w == 0
    assert sizes["bf16x3", False] == sizes["bf16x3", True]
    # ... with runs of 4 x 4: U and V to hi/lo planes, W in place (U planes | V planes | tables)
    v4 = _desc("++--", 0, (3, 3, 4, 4))
    info = _plan("abcd,cdij->abij", 4, u, v4, compute=L.COMPUTE["bf16x3"])[1]
    assert info.fused == 0 and info.fused_w == 1
    # (planes at K pitch 40: U 36 x 40, V 64 x 40 per Q)
    assert info.workspace_bytes == r(4 * 4 * 36 * 40) + r(4 * 4 * 64 * 40) + tables(36, 36) + tables(36, 64)


def test_status_strings():
    for code in range(-8, 1):
        assert L.status_string(code) not in ("", "unknown status")
    assert L.status_string(-99) == "unknown status"


def _gemm_ws(compute, batch, m, k, n):
    out = ctypes.c_size_t()
    rc = L.LIB.symtensor_sector_gemm_workspace_size(compute, batch, m, k, n, ctypes.byref(out))
    return rc, out.value


def test_stream_k_choice_and_workspace(monkeypatch):
    """Stream-K is chosen where whole waves of tiles would idle the device."""
    monkeypatch.delenv("SYMT_GEMM_SK", raising=False)
    monkeypatch.delenv("SYMT_GEMM_TILE", raising=False)
    # CCD ladder over Z_8 (24 virtual, 6 occupied per sector): 1152 tiles of 96 x 96
    # on 768 resident workgroups leave a last wave half full; two f64 pieces per
    # persistent workgroup
    rc, ladder = _gemm_ws(L.COMPUTE["f64"], 8, 4608, 4608, 288)
    assert rc == 0 and ladder == 2 * 768 * 96 * 96 * 8
    # 16384 tiles: whole waves, nothing to recover.
    assert _gemm_ws(L.COMPUTE["f64"], 16, 16384, 16384, 1024) == (0, 0)
    # split-bf16 and empty products never need it
    assert _gemm_ws(L.COMPUTE["bf16x3"], 8, 4608, 4608, 288) == (0, 0)
    assert _gemm_ws(L.COMPUTE["f64"], 8, 0, 4608, 288) == (0, 0)
    assert _gemm_ws(7, 1, 1, 1, 1)[0] == L.SYMT_EDTYPE
    assert _gemm_ws(L.COMPUTE["f64"], 1, -1, 1, 1)[0] == L.SYMT_EINVAL
    # forbidding it drops the workspace; the contraction's workspace carries the same pieces
    u = _desc("++--", 0, (24, 24, 24, 24))
    v = _desc("++--", 0, (24, 24, 6, 6))
    g = L.make_group(8)
    info = L.plan("abcd,cdij->abij", g, u, v, None, L.COMPUTE["f64"])
    assert (info.m, info.k, info.n) == (4608, 4608, 288) and info.fused
    r = lambda x: (x + 255) // 256 * 256  # noqa: E731
    # V_al, then the row and column tables of U, W and (V read in place) V
    assert info.fused_v == 1
    base = r(info.bytes_v_al) + r(8 * 8 * 4608) * 2 + r(8 * 8 * 4608) + r(8 * 8 * 288) + \
        r(8 * 8 * 4608) + r(8 * 8 * 288)
    assert info.workspace_bytes == base + r(ladder)
    monkeypatch.setenv("SYMT_GEMM_SK", "0")
    assert _gemm_ws(L.COMPUTE["f64"], 8, 4608, 4608, 288) == (0, 0)
    assert L.plan("abcd,cdij->abij", g, u, v, None, L.COMPUTE["f64"]).workspace_bytes == base


# ---------------------------------------------------------------------------
# charge tables (symt_tensor.mode_charges)
# ---------------------------------------------------------------------------
def _cdesc(signs, charge, dims, tables):
    return L.TensorDesc(signs, charge, dims, L.SYMT_F64, None, tables)


def test_charge_tables_validation():
    G = 3
    ident = [0, 1, 2]
    a, k, b = [1, 2, 0], [2, 0, 1], [0, 2, 1]
    u = _cdesc("+-", 0, (2, 3), [a, k])
    v = _cdesc("+-", 0, (3, 4), [k, b])
    rc, info = _plan("ak,kb->ab", G, u, v)
    assert rc == 0
    base_rc, base = _plan("ak,kb->ab", G, _desc("+-", 0, (2, 3)), _desc("+-", 0, (3, 4)))
    # the device copy of the tables (forward and inverse per mode of u, v, w) adds workspace
    assert info.workspace_bytes >= base.workspace_bytes + 4 * 2 * G * 6
    # all-identity tables are the same as none
    rc, same = _plan("ak,kb->ab", G, _cdesc("+-", 0, (2, 3), [ident, ident]), _cdesc("+-", 0, (3, 4), [ident, ident]))
    assert rc == 0 and same.workspace_bytes == base.workspace_bytes
    # not a permutation
    assert _plan("ak,kb->ab", G, _cdesc("+-", 0, (2, 3), [[0, 0, 1], k]), v)[0] == L.SYMT_EINVAL
    assert _plan("ak,kb->ab", G, _cdesc("+-", 0, (2, 3), [[0, 1, 3], k]), v)[0] == L.SYMT_EINVAL
    # contracted mode with different tables in u and v
    assert _plan("ak,kb->ab", G, u, _cdesc("+-", 0, (3, 4), [ident, b]))[0] == L.SYMT_ESYM
    # w must carry the derived tables (u's on a, v's on b); NULL stands for identity
    sig = info.w_signs.decode()
    assert _plan("ak,kb->ab", G, u, v, _cdesc(sig, info.w_charge, (2, 4), [a, b]))[0] == 0
    assert _plan("ak,kb->ab", G, u, v, _desc(sig, info.w_charge, (2, 4)))[0] == L.SYMT_ESYM
    assert _plan("ak,kb->ab", G, u, v, _cdesc(sig, info.w_charge, (2, 4), [b, a]))[0] == L.SYMT_ESYM


def test_complex_planning():
    G = 4
    u = _desc("+-", 1, (3, 5), L.SYMT_C128)
    v = _desc("+-", 2, (5, 6), L.SYMT_C64)
    rc, info = _plan("ak,kb->ab", G, u, v)
    assert rc == 0
    # the real representation of C: K and N doubled, 8 real flops per complex multiply-add
    assert (info.m, info.k, info.n) == (3, 10, 12)
    assert info.flops == 8 * G * 3 * 5 * 6
    assert info.bytes_u_al == 8 * G * 3 * 10 and info.bytes_v_al == 8 * G * 10 * 12
    assert info.bytes_w_al == 8 * G * 3 * 12
    assert info.fused == 1          # one contracted mode: a single run of 2 x 5 reals
    rc32, info32 = _plan("ak,kb->ab", G, u, v, compute=1)
    assert rc32 == 0 and info32.bytes_v_al == 4 * G * 10 * 12
    # all complex or all real; split-bf16 takes complex operands in three steps
    # (planes K fastest, the K pitch rounded up to 8 in the workspace: 10 -> 16)
    assert _plan("ak,kb->ab", G, u, _desc("+-", 2, (5, 6)))[0] == L.SYMT_EDTYPE
    rcb, infob = _plan("ak,kb->ab", G, u, v, compute=2)
    assert rcb == 0 and infob.fused == 0 and infob.fused_w == 0
    assert infob.bytes_u_al == 4 * G * 3 * 10 and infob.bytes_v_al == 4 * G * 10 * 12
    r = lambda x: (x + 255) // 256 * 256  # noqa: E731
    assert infob.workspace_bytes == r(4 * G * 3 * 16) + r(4 * G * 16 * 12) + r(8 * G * 3 * 12)
    sig = info.w_signs.decode()
    assert _plan("ak,kb->ab", G, u, v, _desc(sig, info.w_charge, (3, 6), L.SYMT_C128))[0] == 0
    assert _plan("ak,kb->ab", G, u, v, _desc(sig, info.w_charge, (3, 6)))[0] == L.SYMT_EDTYPE
    assert _plan("ak,kb->ab", G, _desc("+-", 1, (3, 5)), _desc("+-", 2, (5, 6)),
                 _desc(sig, info.w_charge, (3, 6), L.SYMT_C64))[0] == L.SYMT_EDTYPE
    assert _plan("ak,kb->ab", G, _desc("+-", 1, (3, 5), 7), v)[0] == L.SYMT_EDTYPE


def _sdesc(signs, charge, dims, sectors, dtype=L.SYMT_F64):
    return L.TensorDesc(signs, charge, dims, dtype, None, None, sectors)


def test_subgroup_sector_counts_planning():
    G = 6
    # a: 3 sectors (c = 2), k: 2 sectors (c = 3), b: 6 sectors
    u = _sdesc("+-", 2, (2, 3), (3, 2))
    v = _sdesc("+-", 3, (3, 4), (2, 6))
    rc, info = _plan("ak,kb->ab", G, u, v)
    assert rc == 0
    # stored-sector radices: I and K have one mode each, so M = n_a, K = n_k, N = n_b
    assert (info.m, info.k, info.n) == (2, 3, 4) and info.fused == 0
    assert info.elems_u == 3 * 2 * 3 and info.elems_v == 2 * 3 * 4
    rc, info2 = _plan("abk,kc->abc", G, _sdesc("++-", 0, (2, 2, 3), (3, 2, 2)), _sdesc("+-", 0, (3, 4), (2, 6)))
    assert rc == 0 and info2.m == 3 * 2 * 2          # a (3 sectors) stored, b implicit
    # counts must divide |G|
    assert _plan("ak,kb->ab", G, _sdesc("+-", 2, (2, 3), (4, 2)), v)[0] == L.SYMT_EINVAL
    # a contracted mode carries one count
    assert _plan("ak,kb->ab", G, u, _sdesc("+-", 3, (3, 4), (3, 6)))[0] == L.SYMT_ESYM
    # w carries the derived counts (NULL stands for |G| everywhere)
    sig = info.w_signs.decode()
    assert _plan("ak,kb->ab", G, u, v, _sdesc(sig, info.w_charge, (2, 4), (3, 6)))[0] == 0
    assert _plan("ak,kb->ab", G, u, v, _desc(sig, info.w_charge, (2, 4)))[0] == L.SYMT_ESYM
    # a cyclic group and no charge tables
    assert _plan("ak,kb->ab", (2, 3), _sdesc("+-", 2, (2, 3), (3, 2)), _sdesc("+-", 3, (3, 4), (2, 6)))[0] \
        == L.SYMT_EUNSUPPORTED
    tab = [[1, 0, 2, 3, 4, 5], [0, 1, 2, 3, 4, 5]]          # a relabelled, k identity
    withtab = L.TensorDesc("+-", 2, (2, 3), L.SYMT_F64, None, tab, (3, 2))
    assert _plan("ak,kb->ab", G, withtab, v)[0] == L.SYMT_EUNSUPPORTED
    # all counts |G| is the plain case
    rc, plain = _plan("ak,kb->ab", G, _sdesc("+-", 2, (2, 16), (6, 6)), _sdesc("+-", 3, (16, 4), (6, 6)))
    assert rc == 0 and plain.fused == 1
    rc, sub = _plan("ak,kb->ab", G, _sdesc("+-", 2, (2, 16), (3, 6)), _sdesc("+-", 3, (16, 4), (6, 6)))
    assert rc == 0 and sub.fused == 0


@pytest.mark.parametrize("G,s,t,v", [(4, 1, 1, 1), (6, 2, 1, 1), (8, 1, 2, 1), (12, 1, 1, 2), (6, 2, 2, 1),
                                     (6, 1, 1, 0), (4, 0, 2, 1), (6, 2, 0, 1), (5, 1, 1, 1)])
def test_live_slices_match_the_oracles_nonzero_slices(G, s, t, v):
    """The planner multiplies only the Q slices where all three deltas can hold:
    exactly those where the oracle's U_al and V_al (random data) are both nonzero."""
    from tests import gpu_helpers as H
    rng = np.random.default_rng(seed(("live", G, s, t, v)))
    for _ in range(4):
        sub, su, sv = H.subgroup_case(rng, G, s, t, v, nmax=2)
        Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
        Ual, Val = O.align_u(sub, Ru, su, sv), O.align_v(sub, Rv, su, sv)
        live = sum(1 for q in range(G) if np.any(Ual[q] != 0) and np.any(Val[q] != 0))
        rc, info = _plan(sub, G, _sdesc(su.sign_string(), su.charge, su.dims, su.sectors),
                         _sdesc(sv.sign_string(), sv.charge, sv.dims, sv.sectors))
        assert rc == 0
        assert info.flops == 2 * live * info.m * info.k * info.n


def test_fused_needs_whole_k_steps_per_run(monkeypatch):
    """The global-to-LDS tiles read a 128-byte K-step (16 f64, 32 f32) from one run of
    contracted indices: f32 needs runs of 32, complex operands count reals.  Other
    runs are stepped one by one on register tiles (here forced to a global-to-LDS
    tile, so the aligned forms are kept)."""
    monkeypatch.setenv("SYMT_GEMM_TILE", "d128x128s2")
    G = 4
    u16, v16 = _desc("+-+-", 0, (3, 5, 4, 4)), _desc("+-+-", 0, (4, 4, 4, 4))
    assert _plan("abkl,klij->abij", G, u16, v16, compute=0)[1].fused == 1
    f16, fv16 = _desc("+-+-", 0, (3, 5, 4, 4), L.SYMT_F32), _desc("+-+-", 0, (4, 4, 4, 4), L.SYMT_F32)
    assert _plan("abkl,klij->abij", G, f16, fv16, compute=1)[1].fused == 0
    # on the register tiles the run of 16 f32 is stepped on its own
    monkeypatch.setenv("SYMT_GEMM_TILE", "128x128")
    assert _plan("abkl,klij->abij", G, f16, fv16, compute=1)[1].fused == 1
    f32, fv32 = _desc("+-+-", 0, (3, 5, 4, 8), L.SYMT_F32), _desc("+-+-", 0, (4, 8, 4, 4), L.SYMT_F32)
    assert _plan("abkl,klij->abij", G, f32, fv32, compute=1)[1].fused == 1
    c16 = _desc("+-+-", 0, (3, 5, 4, 4), L.SYMT_C64)
    cv16 = _desc("+-+-", 0, (4, 4, 4, 4), L.SYMT_C64)
    assert _plan("abkl,klij->abij", G, c16, cv16, compute=1)[1].fused == 1      # 2 x 16 reals
    c8 = _desc("+-+-", 0, (3, 5, 2, 4), L.SYMT_C128)
    cv8 = _desc("+-+-", 0, (2, 4, 4, 4), L.SYMT_C128)
    assert _plan("abkl,klij->abij", G, c8, cv8, compute=0)[1].fused == 1       # 2 x 8 reals
    c8s = _desc("+-+-", 0, (3, 5, 2, 4), L.SYMT_C64)
    cv8s = _desc("+-+-", 0, (2, 4, 4, 4), L.SYMT_C64)
    assert _plan("abkl,klij->abij", G, c8s, cv8s, compute=1)[1].fused == 0
    # one contracted mode: its run is the whole K range, of any length
    assert _plan("ak,kb->ab", G, _desc("+-", 0, (3, 57)), _desc("+-", 0, (57, 5)), compute=0)[1].fused == 1
    assert _plan("ak,kb->ab", G, _desc("+-", 0, (3, 57), L.SYMT_F32), _desc("+-", 0, (57, 5), L.SYMT_F32),
                 compute=1)[1].fused == 1


def test_v_in_place_layout_rules(monkeypatch):
    """The product reads B straight from V's standard form when V's contracted
    modes are affine in U's K order, a K run holds whole K-steps and V's
    trailing output modes form runs of whole 16-byte chunks; otherwise V is
    aligned as before."""
    monkeypatch.delenv("SYMT_GEMM_TILE", raising=False)
    monkeypatch.delenv("SYMT_GEMM_SK", raising=False)
    u = _desc("++--", 0, (24, 24, 24, 24))
    ladder = _plan("abcd,cdij->abij", 8, u, _desc("++--", 0, (24, 24, 6, 6)))[1]
    assert ladder.fused == 1 and ladder.fused_v == 1
    # contracted modes stored in the other order, or split by an output mode
    assert _plan("abcd,dcij->abij", 8, u, _desc("++--", 0, (24, 24, 6, 6)))[1].fused_v == 0
    assert _plan("abcd,cidj->abij", 8, u, _desc("+-+-", 0, (24, 6, 24, 6)))[1].fused_v == 0
    # output run of 6 f64 = 48 bytes is whole chunks; 3 f64 (an odd run) is not
    assert _plan("abcd,cdij->abij", 8, u, _desc("++--", 0, (24, 24, 3, 1)))[1].fused_v == 0
    # K run of 24 f64 rows is not whole 16-row steps
    u24 = _desc("++--", 0, (24, 24, 4, 6))
    assert _plan("abcd,cdij->abij", 8, u24, _desc("++--", 0, (4, 6, 6, 6)))[1].fused_v == 0
    # complex operands; a K run of 4 x 4 = 16 rows is one whole step
    c = _desc("++--", 0, (24, 24, 24, 24), L.SYMT_C128)
    assert _plan("abcd,cdij->abij", 8, c, _desc("++--", 0, (24, 24, 6, 6), L.SYMT_C128))[1].fused_v == 0
    assert _plan("abcd,cdij->abij", 8, _desc("++--", 0, (4, 4, 4, 4)),
                 _desc("++--", 0, (4, 4, 2, 2)))[1].fused_v == 1
    # register tiles read V in place too: a forced one, a small product, binary32
    monkeypatch.setenv("SYMT_GEMM_TILE", "128x48")
    forced = _plan("abcd,cdij->abij", 8, u, _desc("++--", 0, (24, 24, 6, 6)))[1]
    assert forced.fused == 1 and forced.fused_v == 1
    monkeypatch.delenv("SYMT_GEMM_TILE")
    small = _plan("abkl,klij->abij", 4, _desc("++--", 0, (3, 5, 4, 8)), _desc("++--", 0, (4, 8, 2, 6)))[1]
    assert small.fused == 1 and small.fused_v == 1
    u32, v32 = _desc("++--", 0, (24, 24, 24, 24), L.SYMT_F32), _desc("++--", 0, (24, 24, 6, 6), L.SYMT_F32)
    assert _plan("abcd,cdij->abij", 8, u32, v32, compute=1)[1].fused_v == 1
    # switched off: V aligned, no V tables
    monkeypatch.setenv("SYMT_FUSED_V", "0")
    off = _plan("abcd,cdij->abij", 8, u, _desc("++--", 0, (24, 24, 6, 6)))[1]
    assert off.fused == 1 and off.fused_v == 0 and off.workspace_bytes < ladder.workspace_bytes


def test_split_bf16_fused_plans(monkeypatch):
    """The split-bf16 product reads U in place (binary64 or binary32, split into
    hi/lo in registers) when U's trailing contracted block holds whole 32-deep
    K-steps, W is binary64 and the launcher runs register tiles on the shape."""
    monkeypatch.delenv("SYMT_GEMM_TILE", raising=False)
    bf = L.COMPUTE["bf16x3"]
    v = _desc("++--", 0, (24, 24, 6, 6))
    ladder = _plan("abcd,cdij->abij", 8, _desc("++--", 0, (24, 24, 24, 24)), v, compute=bf)[1]
    assert ladder.fused == 1 and ladder.fused_v == 0
    r = lambda x: (x + 255) // 256 * 256  # noqa: E731
    assert ladder.workspace_bytes == r(ladder.bytes_v_al) + r(8 * 8 * 4608) * 2 + r(8 * 8 * 4608) + \
        r(8 * 8 * 288)
    u32, v32 = _desc("++--", 0, (24, 24, 24, 24), L.SYMT_F32), _desc("++--", 0, (24, 24, 6, 6), L.SYMT_F32)
    assert _plan("abcd,cdij->abij", 8, u32, v32, compute=bf)[1].fused == 1
    # a binary32 output (the binary64 sums rounded on the store), a contracted block of
    # 16, a global-to-LDS shape (Z_16 ladder)
    w32 = _desc("++--", 0, (24, 24, 6, 6), L.SYMT_F32)
    assert _plan("abcd,cdij->abij", 8, _desc("++--", 0, (24, 24, 24, 24)), v, w32, compute=bf)[1].fused == 1
    assert _plan("abcd,cdij->abij", 8, _desc("++--", 0, (24, 24, 4, 4)),
                 _desc("++--", 0, (4, 4, 6, 6)), compute=bf)[1].fused == 0
    z16 = _plan("abcd,cdij->abij", 16, _desc("++--", 0, (32, 32, 32, 32)), _desc("++--", 0, (32, 32, 8, 8)),
                compute=bf)[1]
    assert z16.fused == 0 and z16.fused_w == 1      # planes for U and V, W written in place
    monkeypatch.setenv("SYMT_GEMM_TILE", "b128x128k32")
    assert _plan("abcd,cdij->abij", 16, _desc("++--", 0, (32, 32, 32, 32)),
                 _desc("++--", 0, (32, 32, 8, 8)), compute=bf)[1].fused == 1


def test_leading_contracted_modes_plans(monkeypatch):
    """U's contracted modes first: on register tiles A is loaded K-major from U in
    place (fused = 1, no U_al in the workspace); on a global-to-LDS tile U alone is
    aligned (fused = 0, fused_w = 1, U_al first in the workspace); complex too."""
    monkeypatch.delenv("SYMT_GEMM_TILE", raising=False)
    monkeypatch.delenv("SYMT_GEMM_SK", raising=False)
    u, v = _desc("--++", 0, (4, 8, 3, 5)), _desc("++--", 0, (4, 8, 2, 6))
    r = lambda x: (x + 255) // 256 * 256  # noqa: E731
    km = _plan("klab,klij->abij", 4, u, v)[1]
    assert km.fused == 1 and km.fused_w == 1 and km.fused_v == 1
    assert km.workspace_bytes < km.bytes_u_al      # V_al and tables only
    monkeypatch.setenv("SYMT_GEMM_TILE", "d96x96s2")
    ua = _plan("klab,klij->abij", 4, u, v)[1]
    assert ua.fused == 0 and ua.fused_w == 1
    assert ua.workspace_bytes >= r(ua.bytes_u_al) + r(ua.bytes_v_al)
    monkeypatch.delenv("SYMT_GEMM_TILE")
    cu, cv = _desc("--++", 0, (4, 8, 3, 5), L.SYMT_C128), _desc("++--", 0, (4, 8, 2, 6), L.SYMT_C128)
    c = _plan("klab,klij->abij", 4, cu, cv)[1]
    assert c.fused == 1 and c.fused_w == 1 and c.fused_v == 0
    # forced three steps
    st = _plan("klab,klij->abij", 4, u, v, compute=0x100)[1]
    assert st.fused == 0 and st.fused_w == 0


def test_split_k_for_few_tiles_and_long_k(monkeypatch):
    """Register tiles split a long K into runs when a launch has too few tiles to fill the CUs."""
    monkeypatch.delenv("SYMT_GEMM_SK", raising=False)
    monkeypatch.delenv("SYMT_GEMM_TILE", raising=False)
    # the (s, t, v) = (1, 1, 3) sweep case: 4 x (57 x 2963088 x 57); N odd rules out the DMA tiles
    rc, ws = _gemm_ws(L.COMPUTE["f64"], 4, 57, 2963088, 57)
    assert rc == 0 and ws > 0
    monkeypatch.setenv("SYMT_GEMM_SK", "0")
    assert _gemm_ws(L.COMPUTE["f64"], 4, 57, 2963088, 57) == (0, 0)
    monkeypatch.delenv("SYMT_GEMM_SK")
    # short K: nothing to split
    assert _gemm_ws(L.COMPUTE["f64"], 4, 57, 64, 57) == (0, 0)


def test_outer_product_takes_the_sign_ratio_that_matches_the_given_output():
    """v = 0: the rule derived with sigma = +1 describes the outer product's blocks too.

    'a,k->ak' is the gradient dU = dW (x) V of 'ak,k->a' (u +- with Z 2, v + with
    Z 1 over Z_5: sigma = -1, W = + with Z 3); dU must carry u's own rule.
    'k,b->kb' is dV = U (x) dW of 'k,kb->b' (u + with Z 2, v -+ with Z 1).
    """
    g = 5
    rc, info = _plan("a,k->ak", g, _desc("+", 3, (3,)), _desc("+", 1, (4,)))
    assert rc == 0 and info.sigma == -1 and info.w_signs.decode() == "++" and info.w_charge == 4
    rc, info = _plan("a,k->ak", g, _desc("+", 3, (3,)), _desc("+", 1, (4,)), _desc("+-", 2, (3, 4)))
    assert rc == 0, L.last_error()
    assert info.sigma == 1 and info.w_signs.decode() == "+-" and info.w_charge == 2
    # the -1 rule, when given, keeps -1
    rc, info = _plan("a,k->ak", g, _desc("+", 3, (3,)), _desc("+", 1, (4,)), _desc("++", 4, (3, 4)))
    assert rc == 0 and info.sigma == -1
    # dV of 'k,kb->b': forward W = + with Z 3; dV carries v's rule (-+, 1) or its flip (+-, 4)
    for wsig, wz in (("-+", 1), ("+-", 4)):
        rc, info = _plan("k,b->kb", g, _desc("+", 2, (4,)), _desc("+", 3, (3,)), _desc(wsig, wz, (4, 3)))
        assert rc == 0 and info.sigma == 1, L.last_error()
    # a rule neither ratio derives is still rejected
    rc, _ = _plan("a,k->ak", g, _desc("+", 3, (3,)), _desc("+", 1, (4,)), _desc("+-", 3, (3, 4)))
    assert rc == L.SYMT_ESYM


def test_python_plan_cache_follows_the_tuning_variables(monkeypatch):
    """The binding's plan cache keys on the tuning variables as the library's does: the
    Z_8 ladder's workspace holds stream-K pieces by default and none with SYMT_GEMM_SK=0."""
    import torch
    import paper_2007_08056_amd as P
    wl = synth.configs.get("ccd_ladder_z8")
    st = wl.steps[0]
    mk = lambda name: P.SymTensor(torch.empty(wl.reduced_shape(name), dtype=torch.float64),  # noqa: E731
                                  wl.operands[name].signs, wl.operands[name].charge, wl.group)
    u, v = mk(st.u), mk(st.v)
    monkeypatch.delenv("SYMT_GEMM_SK", raising=False)
    with_pieces = P.plan(st.einsum, u, v, "f64").workspace_bytes
    monkeypatch.setenv("SYMT_GEMM_SK", "0")
    without = P.plan(st.einsum, u, v, "f64").workspace_bytes
    monkeypatch.delenv("SYMT_GEMM_SK")
    assert with_pieces > without
    assert P.plan(st.einsum, u, v, "f64").workspace_bytes == with_pieces
