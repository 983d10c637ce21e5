"""GPU parity of every step of the HIP path against the CPU oracle (MI355X).

Each test prints what names its case before touching the GPU.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth
from synth import philox
from tests import gpu_helpers as H
from tests.seeding import seed

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


def _sym_tensor(P, R: np.ndarray, sym: O.Sym, dtype=torch.float64):
    return P.SymTensor(torch.from_numpy(np.ascontiguousarray(R)).to(DEV, dtype), sym.sign_string(),
                       sym.charge, sym.group.orders, sym.charges, sym.sectors)


# ---------------------------------------------------------------------------
# synthetic inputs: GPU generator == NumPy generator, bit for bit
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dist,scale", [(philox.DIST_UNIFORM, 1.0), (philox.DIST_NORMAL, 1.0),
                                        (philox.DIST_NORMAL, 1e-2)])
def test_generator_bit_exact(SG, dist, scale):
    say(f"generator dist={dist} scale={scale}")
    first = (1 << 33) + 12345
    n = 100_003
    ref = philox.values_at(np.arange(first, first + n, dtype=np.int64), 99, 7, dist, scale)
    t = torch.empty(n, dtype=torch.float64, device=DEV)
    SG.fill_(t, 99, 7, dist, scale, first=first)
    assert np.array_equal(H.to_np(t), ref)
    t32 = torch.empty(n, dtype=torch.float32, device=DEV)
    SG.fill_(t32, 99, 7, dist, scale, first=first)
    assert np.array_equal(H.to_np(t32), ref.astype(np.float32))


# ---------------------------------------------------------------------------
# step (b) alone: sector-batched products
# ---------------------------------------------------------------------------
GEMM_SHAPES = [(1, 16, 4, 16), (3, 64, 64, 64), (2, 130, 50, 70), (4, 200, 96, 288), (1, 1, 1, 1),
               (2, 257, 33, 47), (6, 300, 48, 48), (1, 128, 128, 128), (5, 17, 0, 9)]


@pytest.mark.parametrize("shape", GEMM_SHAPES)
@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_sector_gemm_fp(P, shape, compute):
    say(f"sector_gemm {compute} {shape}")
    b, m, k, n = shape
    rng = np.random.default_rng(m * 1000 + n)
    A = rng.standard_normal((b, m, k))
    B = rng.standard_normal((b, k, n))
    dt = torch.float64 if compute == "f64" else torch.float32
    a = torch.from_numpy(A).to(DEV, dt)
    bb = torch.from_numpy(B).to(DEV, dt)
    C = H.to_np(P.sector_gemm(a, bb, compute))
    A = H.to_np(a).astype(np.float64)
    B = H.to_np(bb).astype(np.float64)
    ref = np.matmul(A, B)
    absb = np.matmul(np.abs(A), np.abs(B))
    fac = 2 * H.gamma(max(k, 1), H.U64) if compute == "f64" else 1.05 * H.gamma(max(k, 1), H.U32)
    assert np.all(np.abs(C - ref) <= fac * absb + 1e-300), compute


@pytest.mark.parametrize("tile,shape", [
    (None, (1, 16, 32, 16)), (None, (3, 64, 64, 64)), (None, (2, 130, 56, 70)), (None, (4, 200, 96, 288)),
    (None, (2, 257, 40, 47)), (None, (6, 300, 48, 48)), (None, (1, 128, 256, 128)),
    # global-to-LDS split-bf16 tiles (K a multiple of 32), ragged in M and N, and the default pick
    ("bd256x128s3", (2, 300, 96, 200)), ("bd256x128s3", (1, 512, 64, 256)),
    ("bd128x256s3", (2, 200, 128, 300)), ("bd128x256s3", (3, 130, 32, 70)),
    (None, (2, 600, 256, 384)),
    # wide tiles with one accumulator, ragged in M and N, and their default picks
    ("bw256x256s2", (2, 300, 96, 300)), ("bw256x256s2", (1, 512, 64, 512)), ("bw256x256s2", (3, 130, 32, 70)),
    ("bw256x128s3", (2, 300, 64, 200)), ("bw256x128s3", (3, 257, 32, 129)), ("bw256x128s3", (1, 512, 160, 384)),
    (None, (16, 1024, 64, 1024)), (None, (32, 512, 32, 384)),
    # the 96-wide register tile, ragged in M and N
    ("b128x96k32", (2, 130, 64, 200)), ("b128x96k32", (3, 257, 40, 96)),
])
def test_sector_gemm_bf16x3(P, tile, shape, monkeypatch):
    if tile:
        monkeypatch.setenv("SYMT_GEMM_TILE", tile)
    say(f"sector_gemm bf16x3 tile={tile} {shape}")
    b, m, k, n = shape
    rng = np.random.default_rng(m * 7 + n)
    A = rng.standard_normal((b, m, k)).astype(np.float32)
    B = rng.standard_normal((b, k, n)).astype(np.float32)
    ah, al = O.bf16_split(A)
    bh, bl = O.bf16_split(np.ascontiguousarray(np.swapaxes(B, 1, 2)))   # [b][n][k]
    bits = lambda x: (x.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)  # noqa: E731
    a = torch.from_numpy(np.stack([bits(ah), bits(al)])).to(DEV)
    bb = torch.from_numpy(np.stack([bits(bh), bits(bl)])).to(DEV)
    C = H.to_np(P.sector_gemm(a, bb, "bf16x3"))
    ah64, al64 = ah.astype(np.float64), al.astype(np.float64)
    bh64 = np.swapaxes(bh, 1, 2).astype(np.float64)
    bl64 = np.swapaxes(bl, 1, 2).astype(np.float64)
    ref = np.matmul(ah64, bh64) + np.matmul(ah64, bl64) + np.matmul(al64, bh64)
    absb = (np.matmul(np.abs(ah64), np.abs(bh64)) + np.matmul(np.abs(ah64), np.abs(bl64))
            + np.matmul(np.abs(al64), np.abs(bh64)))
    # binary32 accumulation of the 3k products (one accumulator on the wide tiles)
    assert np.all(np.abs(C - ref) <= 1.02 * H.gamma(3 * k, H.U32) * absb)
    # and the three-term product is within the split bound of the binary32 product
    full = np.matmul(A.astype(np.float64), B.astype(np.float64))
    absf = np.matmul(np.abs(A.astype(np.float64)), np.abs(B.astype(np.float64)))
    assert np.all(np.abs(C - full) <= (3.1 * H.U_BF16_PAIR + 1.03 * H.gamma(3 * k, H.U32)) * absf)


# ---------------------------------------------------------------------------
# steps (a) and (c) alone: bit-exact against Alg. 2 with dense deltas
# ---------------------------------------------------------------------------
ALIGN_CASES = [((4,), 2, 2, 2), ((3,), 1, 1, 1), ((2, 3), 2, 2, 1), ((5,), 1, 3, 2), ((2,), 3, 1, 2),
               ((2, 2), 2, 1, 2), ((1,), 2, 2, 2), ((8,), 1, 1, 1), ((3,), 3, 2, 2)]


def _bf16_planes_of(x64):
    hi, lo = O.bf16_split(x64.astype(np.float32))
    return (hi.view(np.uint32) >> 16).astype(np.uint16), (lo.view(np.uint32) >> 16).astype(np.uint16)


@pytest.mark.parametrize("case", ALIGN_CASES)
def test_align_and_unalign_bit_exact(P, case):
    orders, ns, nt, nv = case
    rng = np.random.default_rng(seed(case))
    for rep in range(3):
        sub, su, sv = H.random_case(rng, orders, ns, nt, nv, nmax=4)
        say(f"align {sub} G={orders} rep={rep} dims_u={su.dims} dims_v={sv.dims}")
        Ru = rng.standard_normal(su.reduced_shape())
        Rv = rng.standard_normal(sv.reduced_shape())
        u = _sym_tensor(P, Ru, su)
        v = _sym_tensor(P, Rv, sv)
        Ual = O.align_u(sub, Ru, su, sv)
        Val = O.align_v(sub, Rv, su, sv)
        assert np.array_equal(H.to_np(P.align(sub, u, v, 0, "f64")), Ual)
        assert np.array_equal(H.to_np(P.align(sub, u, v, 1, "f64")), Val)
        assert np.array_equal(H.to_np(P.align(sub, u, v, 0, "f32")), Ual.astype(np.float32))
        # f32 storage in, f32 aligned out
        u32 = P.SymTensor(u.data.float(), u.signs, u.charge, u.group)
        assert np.array_equal(H.to_np(P.align(sub, u32, v, 0, "f32")), Ual.astype(np.float32))
        # split bf16 planes: U as (2, G, M, K); V transposed (2, G, N, K)
        gu = H.to_np(P.align(sub, u, v, 0, "bf16x3")).view(np.uint16)
        hi, lo = _bf16_planes_of(Ual)
        assert np.array_equal(gu[0], hi) and np.array_equal(gu[1], lo)
        gv = H.to_np(P.align(sub, u, v, 1, "bf16x3")).view(np.uint16)
        hi, lo = _bf16_planes_of(np.ascontiguousarray(np.swapaxes(Val, 1, 2)))
        assert np.array_equal(gv[0], hi) and np.array_equal(gv[1], lo)
        # step (c): random aligned output -> standard form of W
        Wal = rng.standard_normal(np.matmul(Ual, Val).shape)
        ref, sw = O.unalign_w(sub, Wal, su, sv)
        w = P.output_like(sub, u, v)
        P.unalign(sub, u, v, w, torch.from_numpy(Wal).to(DEV), "f64")
        assert np.array_equal(H.to_np(w.data), ref)
        w32 = P.output_like(sub, u, v, dtype=torch.float32)
        P.unalign(sub, u, v, w32, torch.from_numpy(Wal).to(DEV, torch.float32), "f32")
        assert np.array_equal(H.to_np(w32.data), ref.astype(np.float32))


# In-block shapes whose fastest dims are tiny or odd: the transpose tile is
# then a mixed-radix merge of several dims on each side, with ragged tiles.
RAGGED_DIMS = (1, 2, 3, 5, 7, 9, 13, 17, 33, 65, 70)
RAGGED_CASES = [((2, 3), 2, 2, 2), ((3,), 1, 2, 2), ((2,), 2, 1, 3), ((4,), 3, 1, 1), ((1,), 2, 2, 2)]


def _check_align_unalign(P, sub, su, sv, rng):
    Ru = rng.standard_normal(su.reduced_shape())
    Rv = rng.standard_normal(sv.reduced_shape())
    u = _sym_tensor(P, Ru, su)
    v = _sym_tensor(P, Rv, sv)
    Ual = O.align_u(sub, Ru, su, sv)
    Val = O.align_v(sub, Rv, su, sv)
    assert np.array_equal(H.to_np(P.align(sub, u, v, 0, "f64")), Ual)
    assert np.array_equal(H.to_np(P.align(sub, u, v, 1, "f64")), Val)
    assert np.array_equal(H.to_np(P.align(sub, u, v, 0, "f32")), Ual.astype(np.float32))
    gu = H.to_np(P.align(sub, u, v, 0, "bf16x3")).view(np.uint16)
    hi, lo = _bf16_planes_of(Ual)
    assert np.array_equal(gu[0], hi) and np.array_equal(gu[1], lo)
    gv = H.to_np(P.align(sub, u, v, 1, "bf16x3")).view(np.uint16)
    hi, lo = _bf16_planes_of(np.ascontiguousarray(np.swapaxes(Val, 1, 2)))
    assert np.array_equal(gv[0], hi) and np.array_equal(gv[1], lo)
    Wal = rng.standard_normal((Ual.shape[0], Ual.shape[1], Val.shape[2]))
    ref, _ = O.unalign_w(sub, Wal, su, sv)
    w = P.output_like(sub, u, v)
    P.unalign(sub, u, v, w, torch.from_numpy(Wal).to(DEV), "f64")
    assert np.array_equal(H.to_np(w.data), ref)
    w32 = P.output_like(sub, u, v, dtype=torch.float32)
    P.unalign(sub, u, v, w32, torch.from_numpy(Wal).to(DEV, torch.float32), "f32")
    assert np.array_equal(H.to_np(w32.data), ref.astype(np.float32))


@pytest.mark.parametrize("case", RAGGED_CASES)
def test_align_unalign_ragged_inner_dims(P, case):
    orders, ns, nt, nv = case
    rng = np.random.default_rng(seed(("ragged",) + case))
    G = int(np.prod(orders))
    done = 0
    while done < 3:
        sub, su, sv = H.random_case(rng, orders, ns, nt, nv, dim_choices=RAGGED_DIMS)
        tu, rest = sub.split(",")
        tv, tw = rest.split("->")
        dims = dict(zip(tu, su.dims)) | dict(zip(tv, sv.dims))
        sizes = [G ** (len(x) - 1) * int(np.prod([dims[m] for m in x])) for x in (tu, tv, tw)]
        if max(sizes) > 300000:
            continue
        say(f"ragged align {sub} G={orders} dims_u={su.dims} dims_v={sv.dims}")
        _check_align_unalign(P, sub, su, sv, rng)
        done += 1


@pytest.mark.parametrize("orders,sub,cu,du,cv,dv", [
    # a whole matrix block is one run of 90000 elements: cut into ragged chunks
    ((2,), "ij,jk->ik", (1, -1), (300, 300), (1, -1), (300, 300)),
    ((3,), "ij,jk->ik", (1, -1), (200, 150), (1, -1), (150, 170)),
    ((2,), "ijk,klm->ijlm", (1, 1, -1), (100, 3, 100), (1, 1, -1), (100, 1, 100)),
])
def test_align_unalign_long_runs(P, orders, sub, cu, du, cv, dv):
    g = O.Group(orders)
    say(f"long-run align {sub} G={orders} {du} {dv}")
    _check_align_unalign(P, sub, O.Sym(cu, 0, du, g), O.Sym(cv, 0, dv, g), np.random.default_rng(9))


@pytest.mark.parametrize("sub,cu,du,cv,dv", [
    # environment steps of an MPS with physical dim 2 and MPO bond 4 (bond 33)
    ("bcsA,bsSB->cASB", (-1, -1, 1, -1), (4, 33, 2, 33), (1, -1, -1, -1), (4, 2, 2, 4)),
    ("cASB,cSC->ABC", (-1, -1, -1, -1), (33, 33, 2, 4), (1, 1, -1), (33, 2, 33)),
    ("abc,asA->bcsA", (-1, -1, -1), (33, 4, 33), (1, 1, -1), (33, 2, 33)),
])
def test_align_unalign_mps_environment_shapes(P, sub, cu, du, cv, dv):
    g = O.Group((2, 3))
    su, sv = O.Sym(cu, 0, du, g), O.Sym(cv, 0, dv, g)
    say(f"mps-shape align {sub}")
    _check_align_unalign(P, sub, su, sv, np.random.default_rng(5))


# ---------------------------------------------------------------------------
# whole path on random contractions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ALIGN_CASES)
def test_contract_random_vs_oracle(P, case):
    orders, ns, nt, nv = case
    rng = np.random.default_rng(seed(case))
    for rep in range(2):
        sub, su, sv = H.random_case(rng, orders, ns, nt, nv, nmax=5)
        say(f"contract {sub} G={orders} rep={rep}")
        Ru = rng.standard_normal(su.reduced_shape())
        Rv = rng.standard_normal(sv.reduced_shape())
        ref, sw = O.contract_blocks(sub, Ru, su, Rv, sv)
        absref, _ = O.contract_blocks(sub, np.abs(Ru), su, np.abs(Rv), sv)
        k = H.contracted_extent(sub, su)
        u = _sym_tensor(P, Ru, su)
        vv = _sym_tensor(P, Rv, sv)
        for compute in ("f64", "f32", "bf16x3"):
            info = P.plan(sub, u, vv, compute)
            w = P.output_like(sub, u, vv)
            P.contract_into(sub, u, vv, w, compute)
            got = H.to_np(w.data)
            assert w.signs == sw.sign_string() and w.charge == sw.charge
            assert np.all(np.abs(got - ref) <= H.bound_factor(compute, k) * absref + 1e-300), compute
            if compute == "f64":
                assert H.rel_err(got, ref) <= 1e-12
                # zero pattern of the full tensor is identical
                assert np.array_equal(O.expand(got, sw) == 0, O.expand(ref, sw) == 0)


def test_degenerate_shapes(P):
    rng = np.random.default_rng(11)
    g = O.Group(3)
    # an empty contracted block dim: W is all zeros
    su = O.Sym.make("+-", 0, (3, 0), g)
    sv = O.Sym.make("+-", 0, (0, 2), g)
    say("degenerate: empty contracted dim")
    u = _sym_tensor(P, np.zeros(su.reduced_shape()), su)
    v = _sym_tensor(P, np.zeros(sv.reduced_shape()), sv)
    w = P.output_like("ij,jk->ik", u, v)
    w.data.fill_(7.0)
    P.contract_into("ij,jk->ik", u, v, w)
    assert np.all(H.to_np(w.data) == 0.0)
    # an empty output
    su = O.Sym.make("+-", 0, (0, 2), g)
    sv = O.Sym.make("+-", 0, (2, 2), g)
    say("degenerate: empty output")
    u = _sym_tensor(P, np.zeros(su.reduced_shape()), su)
    v = _sym_tensor(P, rng.standard_normal(sv.reduced_shape()), sv)
    w = P.output_like("ij,jk->ik", u, v)
    P.contract_into("ij,jk->ik", u, v, w)
    assert w.data.numel() == 0
    # the trivial group is a plain product
    say("degenerate: trivial group")
    g1 = O.Group(1)
    su = O.Sym.make("++-", 0, (5, 3, 7), g1)
    sv = O.Sym.make("+-", 0, (7, 4), g1)
    Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
    w = P.output_like("abk,kc->acb", _sym_tensor(P, Ru, su), _sym_tensor(P, Rv, sv))
    P.contract_into("abk,kc->acb", _sym_tensor(P, Ru, su), _sym_tensor(P, Rv, sv), w)
    ref = np.einsum("abk,kc->acb", Ru.reshape(5, 3, 7), Rv.reshape(7, 4))
    np.testing.assert_allclose(H.to_np(w.data).reshape(ref.shape), ref, rtol=1e-13, atol=1e-13)


def test_misaligned_views_take_the_scalar_path(P):
    rng = np.random.default_rng(12)
    g = O.Group(4)
    su = O.Sym.make("++--", 1, (2, 3, 2, 2), g)
    sv = O.Sym.make("++--", 2, (2, 2, 3, 1), g)
    Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
    say("misaligned views")
    # views starting one element into a larger buffer: 8-byte but not 16-byte aligned
    bu = torch.zeros(Ru.size + 1, dtype=torch.float64, device=DEV)
    bu[1:] = torch.from_numpy(Ru.ravel()).to(DEV)
    bv = torch.zeros(Rv.size + 1, dtype=torch.float64, device=DEV)
    bv[1:] = torch.from_numpy(Rv.ravel()).to(DEV)
    u = P.SymTensor(bu[1:].view(su.reduced_shape()), "++--", 1, (4,))
    v = P.SymTensor(bv[1:].view(sv.reduced_shape()), "++--", 2, (4,))
    bw = torch.zeros(1 + int(np.prod(O.output_symmetry("abkl,klij->abij", su, sv).reduced_shape())),
                     dtype=torch.float64, device=DEV)
    sw = O.output_symmetry("abkl,klij->abij", su, sv)
    w = P.SymTensor(bw[1:].view(sw.reduced_shape()), sw.sign_string(), sw.charge, (4,))
    P.contract_into("abkl,klij->abij", u, v, w)
    ref, _ = O.contract_blocks("abkl,klij->abij", Ru, su, Rv, sv)
    assert H.rel_err(H.to_np(w.data), ref) <= 1e-13


def test_error_paths_on_device(P):
    from paper_2007_08056_amd import _lib as L
    rng = np.random.default_rng(13)
    g = O.Group(4)
    su = O.Sym.make("++--", 0, (2, 2, 2, 2), g)
    u = _sym_tensor(P, rng.standard_normal(su.reduced_shape()), su)
    v = _sym_tensor(P, rng.standard_normal(su.reduced_shape()), su)
    w = P.output_like("abkl,klij->abij", u, v)
    say("errors: workspace too small")
    with pytest.raises(L.SymtError) as e:
        info = P.plan("abkl,klij->abij", u, v)
        ws = torch.empty(info.workspace_bytes - 1, dtype=torch.uint8, device=DEV)
        import ctypes
        gg = L.make_group(4)
        L.check(L.LIB.symtensor_contract(L.context(0), b"abkl,klij->abij", ctypes.byref(gg), u.desc().ref,
                                         v.desc().ref, w.desc().ref, 0, ctypes.c_void_p(ws.data_ptr()),
                                         ws.numel(), None), L.context(0))
    assert e.value.code == L.SYMT_EWORKSPACE
    say("errors: output aliases an input")
    w_alias = P.SymTensor(u.data, "++--", 0, (4,))
    with pytest.raises(L.SymtError) as e:
        P.contract_into("abkl,klij->abij", u, v, w_alias)
    assert e.value.code == L.SYMT_EALIAS
    say("errors: mixed signs")
    v_bad = P.SymTensor(v.data, "+---", 0, (4,))
    with pytest.raises(L.SymtError) as e:
        P.contract_into("abkl,klij->abij", u, v_bad, w)
    assert e.value.code == L.SYMT_ESYM
    say("errors: an input inside the workspace")
    info = P.plan("abkl,klij->abij", u, v, w=w)
    ws = torch.zeros(info.workspace_bytes + 4096, dtype=torch.uint8, device=DEV)
    inside = ws[: u.data.numel() * 8].view(torch.float64).view(u.data.shape)
    inside.copy_(u.data)
    for uu, vv in ((P.SymTensor(inside, "++--", 0, (4,)), v), (u, P.SymTensor(inside, "++--", 0, (4,)))):
        with pytest.raises(L.SymtError) as e:
            P.contract_into("abkl,klij->abij", uu, vv, w, workspace=ws)
        assert e.value.code == L.SYMT_EALIAS
    # nothing was written by the failed calls
    before = w.data.clone()
    with pytest.raises(L.SymtError):
        P.contract_into("abkl,klij->abij", u, v_bad, w)
    torch.cuda.synchronize()
    assert torch.equal(before, w.data)


def test_plan_cache_reuses_plans_with_new_data(P, monkeypatch):
    """Calls with the same descriptors and new data (a cached plan) and with a
    tuning variable changed (a new plan) all match the oracle."""
    rng = np.random.default_rng(14)
    g = O.Group(4)
    sub = "abkl,klij->abij"
    su = O.Sym.make("++--", 1, (3, 5, 4, 4), g)
    sv = O.Sym.make("++--", 2, (4, 4, 2, 3), g)
    for tile in ("", "128x48", ""):
        if tile:
            monkeypatch.setenv("SYMT_GEMM_TILE", tile)
        else:
            monkeypatch.delenv("SYMT_GEMM_TILE", raising=False)
        for _ in range(2):
            Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
            u, v = _sym_tensor(P, Ru, su), _sym_tensor(P, Rv, sv)
            w = P.output_like(sub, u, v)
            P.contract_into(sub, u, v, w)
            ref, _ = O.contract_blocks(sub, Ru, su, Rv, sv)
            assert H.rel_err(H.to_np(w.data), ref) <= 1e-12, tile


# ---------------------------------------------------------------------------
# fused product: A read from U's standard form, C written into W's
# ---------------------------------------------------------------------------
FUSED_CASES = [
    ("abkl,klij->abij", (4,), "++--", "++--", (3, 5, 4, 4), (4, 4, 2, 3)),
    ("abkl,klij->abji", (3,), "+-+-", "-+++", (2, 7, 8, 2), (8, 2, 4, 1)),
    ("ak,kb->ab", (5,), "+-", "++", (33, 16), (16, 20)),
    ("ak,kb->ba", (2, 3), "--", "-+", (17, 32), (32, 8)),
    ("xykcd,kcdz->zxy", (2,), "+-+--", "-++-", (3, 3, 2, 2, 4), (2, 2, 4, 8)),
    ("abcd,cdij->abij", (8,), "++--", "++--", (5, 6, 4, 4), (4, 4, 3, 2)),
    ("abkl,klij->abij", (4,), "++--", "++--", (3, 5, 4, 8), (4, 8, 2, 3)),
    ("akl,klb->ab", (3,), "+-+", "-++", (7, 2, 16), (2, 16, 12)),
]


def _fusable(compute, sub, du):
    # every product tile reads one K-step from one contiguous run of K: 16 reals,
    # and 32 f32 on the global-to-LDS tiles; a single contracted mode is one run
    tu, rest = sub.split(",")
    tv = rest.split("->")[0]
    k_modes = [m for m in tu if m in tv]
    nK = int(np.prod([d for m, d in zip(tu, du) if m in tv]))
    return nK % (16 if compute == "f64" else 32) == 0 or len(k_modes) == 1


@pytest.mark.parametrize("case", FUSED_CASES)
@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_fused_product_equals_steps_and_oracle(P, case, compute):
    sub, orders, cu, cv, du, dv = case
    rng = np.random.default_rng(len(sub) * 31 + sum(du))
    g = O.Group(orders)
    su = O.Sym.make(cu, int(rng.integers(g.size)), du, g)
    sv = O.Sym.make(cv, int(rng.integers(g.size)), dv, g)
    say(f"fused {sub} G={orders} {compute}")
    Ru = rng.standard_normal(su.reduced_shape())
    Rv = rng.standard_normal(sv.reduced_shape())
    dt = torch.float64 if compute == "f64" else torch.float32
    u = _sym_tensor(P, Ru, su, dt)
    v = _sym_tensor(P, Rv, sv, dt)
    whole = _fusable(compute, sub, du)
    # runs that are not whole K-steps are stepped one by one on register tiles
    # (fused as well, but summed in other groups than the three-step path)
    assert P.plan(sub, u, v, compute).fused == 1 or not whole
    assert P.plan(sub, u, v, compute, steps=True).fused == 0
    w_f = P.output_like(sub, u, v, dtype=dt)
    w_s = P.output_like(sub, u, v, dtype=dt)
    P.contract_into(sub, u, v, w_f, compute)
    P.contract_into(sub, u, v, w_s, compute, steps=True)
    if whole:
        assert torch.equal(w_f.data, w_s.data)
    ref, sw = O.contract_blocks(sub, H.to_np(u.data).astype(np.float64), su,
                                H.to_np(v.data).astype(np.float64), sv)
    absref, _ = O.contract_blocks(sub, np.abs(Ru), su, np.abs(Rv), sv)
    k = H.contracted_extent(sub, su)
    fac = 2 * H.gamma(k, H.U64) if compute == "f64" else 1.05 * H.gamma(k, H.U32) + H.gamma(k, H.U64)
    assert np.all(np.abs(H.to_np(w_f.data) - ref) <= fac * absref + 1e-300)
    assert np.all(np.abs(H.to_np(w_s.data) - ref) <= fac * absref + 1e-300)
    # U starting 8 bytes into a buffer: the fused product loads A one element at a time
    buf = torch.zeros(u.data.numel() + 1, dtype=dt, device=DEV)
    buf[1:] = u.data.reshape(-1)
    u_off = P.SymTensor(buf[1:].view(u.data.shape), u.signs, u.charge, u.group)
    w_o = P.output_like(sub, u, v, dtype=dt)
    P.contract_into(sub, u_off, v, w_o, compute)
    if whole:
        assert torch.equal(w_o.data, w_s.data)
    else:
        assert np.all(np.abs(H.to_np(w_o.data) - ref) <= fac * absref + 1e-300)


# Contracted blocks that are not whole K-steps (odd runs, as in the paper's
# unbalanced (s, t, v) patterns): each run is stepped on its own on register tiles,
# U and V read in place, W written in place.
RUN_CASES = [
    ("abcd,bcde->ae", (4,), "++--", "-++-", (5, 3, 5, 7), (3, 5, 7, 5)),
    ("abcd,cde->abe", (3,), "+-+-", "-++", (4, 5, 3, 5), (3, 5, 6)),
    ("abc,bcde->ade", (2, 2), "+++", "--+-", (6, 5, 3), (5, 3, 4, 5)),
    ("abc,cde->abde", (5,), "++-", "+-+", (3, 4, 7), (7, 3, 5)),
    ("ak,kb->ab", (2,), "+-", "++", (9, 3001), (3001, 7)),          # one long run, split K
    ("abkl,klij->abij", (4,), "++--", "++--", (3, 5, 3, 3), (3, 3, 2, 3)),
    # runs of 24: whole 16-byte vectors (binary64 V columns in pairs as well)
    ("abcd,bcde->ae", (4,), "++--", "-++-", (5, 2, 3, 4), (2, 3, 4, 6)),
]


@pytest.mark.parametrize("case", RUN_CASES)
@pytest.mark.parametrize("compute", ["f64", "f32"])
@pytest.mark.parametrize("tile", ["", "128x48", "64x96", "128x128", "rows"])
def test_fused_product_steps_each_run(P, case, compute, tile, monkeypatch):
    """Run-by-run K-steps: U and V read in place and W written in place whatever the
    run length, within the product's bound of the oracle (as is the three-step
    path), with and without charge tables, and run-to-run identical."""
    sub, orders, cu, cv, du, dv = case
    if tile:
        monkeypatch.setenv("SYMT_GEMM_TILE", tile)
    else:
        monkeypatch.delenv("SYMT_GEMM_TILE", raising=False)
    monkeypatch.delenv("SYMT_GEMM_SK", raising=False)
    rng = np.random.default_rng(seed("runs", sub, orders))
    g = O.Group(orders)
    su0 = O.Sym.make(cu, int(rng.integers(g.size)), du, g)
    sv0 = O.Sym.make(cv, int(rng.integers(g.size)), dv, g)
    dt = torch.float64 if compute == "f64" else torch.float32
    for tables in (False, True):
        su, sv = _with_tables(rng, sub, su0, sv0) if tables else (su0, sv0)
        say(f"run-stepped {sub} G={orders} {compute} tile={tile or 'default'} tables={tables}")
        Ru = rng.standard_normal(su.reduced_shape())
        Rv = rng.standard_normal(sv.reduced_shape())
        u = _sym_tensor(P, Ru, su, dt)
        v = _sym_tensor(P, Rv, sv, dt)
        info = P.plan(sub, u, v, compute)
        assert info.fused == 1 and info.fused_v == 1
        w_f = P.output_like(sub, u, v, dtype=dt)
        w_s = P.output_like(sub, u, v, dtype=dt)
        P.contract_into(sub, u, v, w_f, compute)
        P.contract_into(sub, u, v, w_s, compute, steps=True)
        U64, V64 = H.to_np(u.data).astype(np.float64), H.to_np(v.data).astype(np.float64)
        ref, _ = O.contract_blocks(sub, U64, su, V64, sv)
        absref, _ = O.contract_blocks(sub, np.abs(U64), su, np.abs(V64), sv)
        k = H.contracted_extent(sub, su)
        fac = 2 * H.gamma(k, H.U64) if compute == "f64" else 1.05 * H.gamma(k, H.U32) + H.gamma(k, H.U64)
        for w in (w_f, w_s):
            assert np.all(np.abs(H.to_np(w.data) - ref) <= fac * absref + 1e-300)
        # the same launch twice gives the same bits
        w_2 = P.output_like(sub, u, v, dtype=dt)
        P.contract_into(sub, u, v, w_2, compute)
        assert torch.equal(w_2.data, w_f.data)


# U's contracted modes first (the paper's CC2 / CC3 layouts), or runs that do not
# suit a global-to-LDS tile: U is aligned first, the product reads U_al through
# affine tables, V in place where it can, and writes W in place.
UA_CASES = [
    ("klab,klij->abij", (4,), "--++", "++--", (4, 8, 3, 5), (4, 8, 2, 6)),
    ("opij,opkm->ijmk", (8,), "--++", "++--", (4, 4, 3, 5), (4, 4, 2, 3)),
    ("opmn,opij->ijmn", (2, 3), "+-+-", "-+-+", (4, 8, 3, 2), (4, 8, 5, 3)),
    ("kab,kij->abij", (3,), "-++", "+--", (16, 7, 5), (16, 3, 4)),
    ("abkl,klij->abij", (4,), "++--", "++--", (3, 5, 4, 6), (4, 6, 2, 4)),     # runs of 24
    ("klab,klij->abij", (2,), "--++", "++--", (4, 8, 16, 16), (4, 8, 16, 16)),  # 512 x 64 x 512
    # the chain's E' = T2 A: M chunks of 4 (B) under a strided K (c, S)
    ("cASB,cSC->ABC", (2, 3), "----", "++-", (8, 8, 2, 4), (8, 2, 8)),
    # the chain's dA = T2 dE': no M chunks (S strided), K = (A, B) ending in runs of 4 (B)
    ("cASB,ABC->cSC", (2, 3), "----", "---", (8, 8, 2, 4), (8, 4, 8)),
]


def _w_col_run(sub, du, dv):
    """Contiguous run of W's aligned columns (V's output modes, in V's order) in W."""
    tu, rest = sub.split(",")
    tv, tw = rest.split("->")
    dims = {m: d for m, d in list(zip(tu, du)) + list(zip(tv, dv))}
    stride, acc = {}, 1
    for m in reversed(tw):
        stride[m] = acc
        acc *= dims[m]
    run = 1
    for m in reversed([m for m in tv if m in tw]):
        if stride[m] != run:
            break
        run *= dims[m]
    return run


@pytest.mark.parametrize("case", UA_CASES)
@pytest.mark.parametrize("compute", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("tile,sk", [("", ""), ("d96x96s2", "0"), ("d96x96s2", "1"), ("d128x64s3", "1"),
                                     ("d128x128s2", "0"), ("d128x96s2", "1"),
                                     ("128x48", "0"), ("64x96", "0"), ("rows", "")])
def test_fused_product_on_aligned_u(P, case, compute, tile, sk, monkeypatch):
    """U's contracted modes leading (or runs that do not suit a global-to-LDS
    tile): read K-major in place on register tiles and on 128-row global-to-LDS
    tiles where U's last modes come in 16-byte chunks, else U aligned first on
    global-to-LDS tiles; V in place where its layout allows, W in place (split-bf16: U
    and V on hi/lo planes, W in place): bit-identical to the three-step path on
    the same tile and within the product's bound of the oracle, with and without
    charge tables."""
    sub, orders, cu, cv, du, dv = case
    for name, val in (("SYMT_GEMM_TILE", tile), ("SYMT_GEMM_SK", sk)):
        if val:
            monkeypatch.setenv(name, val)
        else:
            monkeypatch.delenv(name, raising=False)
    rng = np.random.default_rng(seed("aligned-u", sub, orders))
    g = O.Group(orders)
    su0 = O.Sym.make(cu, int(rng.integers(g.size)), du, g)
    sv0 = O.Sym.make(cv, int(rng.integers(g.size)), dv, g)
    dt = torch.float32 if compute == "f32" else torch.float64
    for tables in (False, True):
        su, sv = _with_tables(rng, sub, su0, sv0) if tables else (su0, sv0)
        say(f"aligned-u {sub} G={orders} {compute} tile={tile or 'default'} sk={sk} tables={tables}")
        Ru = rng.standard_normal(su.reduced_shape())
        Rv = rng.standard_normal(sv.reduced_shape())
        u = _sym_tensor(P, Ru, su, dt)
        v = _sym_tensor(P, Rv, sv, dt)
        info = P.plan(sub, u, v, compute)
        # runs of 24 on register tiles are stepped run by run (summed in other groups);
        # U with leading contracted modes on register tiles is read K-major in place
        tu, tv = sub.split(",")[0], sub.split(",")[1].split("->")[0]
        trailing = tu.endswith("".join(m for m in tu if m in tv))
        stepped = info.fused == 1 and trailing
        assert not stepped or (sub.startswith("abkl") and compute != "bf16x3")
        # split-bf16 writes W in place only where W's columns come in runs of >= 16
        assert info.fused_w == int(compute != "bf16x3" or _w_col_run(sub, du, dv) >= 16)
        w_f = P.output_like(sub, u, v, dtype=dt)
        w_s = P.output_like(sub, u, v, dtype=dt)
        P.contract_into(sub, u, v, w_f, compute)
        P.contract_into(sub, u, v, w_s, compute, steps=True)
        w_o = None
        if not stepped:
            assert torch.equal(w_f.data, w_s.data)
            # U one element into a buffer (not 16-byte aligned): one-element loads, same
            # bits (a 128-row global-to-LDS tile reads K-major A in place only from an
            # aligned U: one element off, a register tile takes over, summing the
            # stream-K pieces in another order, so only the bound applies there)
            buf = torch.zeros(u.data.numel() + 1, dtype=dt, device=DEV)
            buf[1:] = u.data.reshape(-1)
            u_off = P.SymTensor(buf[1:].view(u.data.shape), u.signs, u.charge, u.group, u.mode_charges)
            w_o = P.output_like(sub, u, v, dtype=dt)
            P.contract_into(sub, u_off, v, w_o, compute)
            if not tile.startswith("d128"):
                assert torch.equal(w_o.data, w_s.data)
        if compute == "bf16x3":    # binary32 W: the same sums, rounded on the store
            w32_f = P.output_like(sub, u, v, dtype=torch.float32)
            assert P.plan(sub, u, v, compute, w=w32_f).fused_w == info.fused_w
            P.contract_into(sub, u, v, w32_f, compute)
            assert torch.equal(w32_f.data, w_s.data.to(torch.float32))
        U64, V64 = H.to_np(u.data).astype(np.float64), H.to_np(v.data).astype(np.float64)
        ref, _ = O.contract_blocks(sub, U64, su, V64, sv)
        absref, _ = O.contract_blocks(sub, np.abs(U64), su, np.abs(V64), sv)
        k = H.contracted_extent(sub, su)
        fac = H.bound_factor(compute, k)
        assert np.all(np.abs(H.to_np(w_f.data) - ref) <= fac * absref + 1e-300)
        if w_o is not None:
            assert np.all(np.abs(H.to_np(w_o.data) - ref) <= fac * absref + 1e-300)


@pytest.mark.parametrize("sub,orders,cu,cv,du,dv", [UA_CASES[0], UA_CASES[2], FUSED_CASES[0]])
@pytest.mark.parametrize("udt,vdt", [("f64", "f64"), ("f64", "f32"), ("f32", "f64")])
def test_fused_products_with_mixed_storage(P, sub, orders, cu, cv, du, dv, udt, vdt):
    """f32 compute on operands stored in binary64 (converted by their transforms, or
    read as binary32 in place where stored so) with a binary32 W written in place:
    identical to the three-step path and within the f32 bound of the oracle."""
    rng = np.random.default_rng(seed("mixed", sub, udt, vdt))
    g = O.Group(orders)
    su = O.Sym.make(cu, int(rng.integers(g.size)), du, g)
    sv = O.Sym.make(cv, int(rng.integers(g.size)), dv, g)
    say(f"mixed storage {sub} u={udt} v={vdt}")
    dtype = {"f64": torch.float64, "f32": torch.float32}
    Ru = rng.standard_normal(su.reduced_shape())
    Rv = rng.standard_normal(sv.reduced_shape())
    u = _sym_tensor(P, Ru, su, dtype[udt])
    v = _sym_tensor(P, Rv, sv, dtype[vdt])
    w_f = P.output_like(sub, u, v, dtype=torch.float32)
    w_s = P.output_like(sub, u, v, dtype=torch.float32)
    info = P.plan(sub, u, v, "f32", w=w_f)
    assert info.fused_w == 1
    P.contract_into(sub, u, v, w_f, "f32")
    P.contract_into(sub, u, v, w_s, "f32", steps=True)
    assert torch.equal(w_f.data, w_s.data)
    U64, V64 = H.to_np(u.data).astype(np.float64), H.to_np(v.data).astype(np.float64)
    ref, _ = O.contract_blocks(sub, U64, su, V64, sv)
    absref, _ = O.contract_blocks(sub, np.abs(U64), su, np.abs(V64), sv)
    k = H.contracted_extent(sub, su)
    assert np.all(np.abs(H.to_np(w_f.data) - ref) <= H.bound_factor("f32", k) * absref + 1e-300)


# split-bf16 fused product: U's trailing contracted block a multiple of 32
BF_FUSED_CASES = [
    ("abkl,klij->abij", (4,), "++--", "++--", (3, 5, 4, 8), (4, 8, 2, 6)),
    ("ak,kb->ab", (5,), "+-", "++", (33, 64), (64, 20)),
    ("abkl,klij->abji", (3,), "+-+-", "-+++", (2, 7, 8, 4), (8, 4, 2, 1)),
    ("akl,klb->ab", (2, 3), "+-+", "-++", (7, 2, 16), (2, 16, 12)),
    ("xykcd,kcdz->zxy", (2,), "+-+--", "-++-", (3, 3, 2, 2, 8), (2, 2, 8, 5)),
    ("abkl,klij->abij", (4,), "++--", "++--", (3, 5, 4, 4), (4, 4, 2, 3)),   # run 16: not fused
]


@pytest.mark.parametrize("case", BF_FUSED_CASES)
@pytest.mark.parametrize("udt", ["f64", "f32"])
@pytest.mark.parametrize("tile", ["", "b128x64k32", "b128x96k32", "b128x128k32", "b128x256k32"])
def test_fused_split_bf16_product(P, case, udt, tile, monkeypatch):
    """Split-bf16 product reading U in place (hi/lo split in registers) and writing W
    in place: bit-identical to the three-step path (which writes hi/lo planes),
    within the split-bf16 bound of the oracle; also for a U that is not 16-byte
    aligned (one-element loads)."""
    sub, orders, cu, cv, du, dv = case
    if tile:
        monkeypatch.setenv("SYMT_GEMM_TILE", tile)
    else:
        monkeypatch.delenv("SYMT_GEMM_TILE", raising=False)
    rng = np.random.default_rng(len(sub) * 13 + sum(du))
    g = O.Group(orders)
    su = O.Sym.make(cu, int(rng.integers(g.size)), du, g)
    sv = O.Sym.make(cv, int(rng.integers(g.size)), dv, g)
    say(f"fused split-bf16 {sub} G={orders} u={udt} tile={tile or 'default'}")
    dt = torch.float64 if udt == "f64" else torch.float32
    Ru = rng.standard_normal(su.reduced_shape())
    Rv = rng.standard_normal(sv.reduced_shape())
    u = _sym_tensor(P, Ru, su, dt)
    v = _sym_tensor(P, Rv, sv, dt)
    tu = sub.split(",")[0]
    nK = int(np.prod([d for m, d in zip(tu, du) if m in sub.split(",")[1].split("->")[0]]))
    assert P.plan(sub, u, v, "bf16x3").fused == int(nK % 32 == 0)
    w_f = P.output_like(sub, u, v, dtype=torch.float64)
    w_s = P.output_like(sub, u, v, dtype=torch.float64)
    P.contract_into(sub, u, v, w_f, "bf16x3")
    P.contract_into(sub, u, v, w_s, "bf16x3", steps=True)
    assert torch.equal(w_f.data, w_s.data)
    U64, V64 = H.to_np(u.data).astype(np.float64), H.to_np(v.data).astype(np.float64)
    ref, _ = O.contract_blocks(sub, U64, su, V64, sv)
    absref, _ = O.contract_blocks(sub, np.abs(U64), su, np.abs(V64), sv)
    k = H.contracted_extent(sub, su)
    assert np.all(np.abs(H.to_np(w_f.data) - ref) <= H.bound_factor("bf16x3", k) * absref + 1e-300)
    buf = torch.zeros(u.data.numel() + 1, dtype=dt, device=DEV)
    buf[1:] = u.data.reshape(-1)
    u_off = P.SymTensor(buf[1:].view(u.data.shape), u.signs, u.charge, u.group)
    w_o = P.output_like(sub, u, v, dtype=torch.float64)
    P.contract_into(sub, u_off, v, w_o, "bf16x3")
    assert torch.equal(w_o.data, w_s.data)
    # a binary32 W takes the same sums rounded once, on the store
    w32_f = P.output_like(sub, u, v, dtype=torch.float32)
    w32_s = P.output_like(sub, u, v, dtype=torch.float32)
    assert P.plan(sub, u, v, "bf16x3", w=w32_f).fused == int(nK % 32 == 0)
    P.contract_into(sub, u, v, w32_f, "bf16x3")
    P.contract_into(sub, u, v, w32_s, "bf16x3", steps=True)
    assert torch.equal(w32_f.data, w32_s.data)
    assert torch.equal(w32_f.data, w_s.data.to(torch.float32))


# split-bf16 contractions on the wide tiles: the aligned planes interleaved by
# 32-deep K-steps (K = 32 and 64; M and N ragged against the 256-row tiles)
IL_CASES = [
    ("abcd,cdij->abij", (8,), "++--", "++--", (3, 5, 2, 2), (2, 2, 4, 9)),
    ("abkl,klij->abij", (4,), "++--", "++--", (9, 8, 4, 4), (4, 4, 5, 13)),
]


@pytest.mark.parametrize("case", IL_CASES)
@pytest.mark.parametrize("tile", ["bw256x256s2", "bw256x128s3"])
@pytest.mark.parametrize("steps", [False, True])
def test_interleaved_split_bf16_planes(P, case, tile, steps, monkeypatch):
    """Split-bf16 planes interleaved by K-steps (U aligned first, or the three-step
    path): bit-identical to the plane-after-plane layout on the same wide tile
    (the same sums in the same order), and within the split-bf16 bound of the
    oracle."""
    sub, orders, cu, cv, du, dv = case
    monkeypatch.setenv("SYMT_GEMM_TILE", tile)
    monkeypatch.delenv("SYMT_BF16_IL", raising=False)
    rng = np.random.default_rng(sum(du) * 7 + len(sub))
    g = O.Group(orders)
    su = O.Sym.make(cu, int(rng.integers(g.size)), du, g)
    sv = O.Sym.make(cv, int(rng.integers(g.size)), dv, g)
    say(f"interleaved split-bf16 planes {sub} G={orders} tile={tile} steps={steps}")
    u = _sym_tensor(P, rng.standard_normal(su.reduced_shape()), su, torch.float64)
    v = _sym_tensor(P, rng.standard_normal(sv.reduced_shape()), sv, torch.float64)
    info = P.plan(sub, u, v, "bf16x3")
    assert info.k % 32 == 0 and info.fused == 0
    w_il = P.output_like(sub, u, v, dtype=torch.float64)
    P.contract_into(sub, u, v, w_il, "bf16x3", steps=steps)
    monkeypatch.setenv("SYMT_BF16_IL", "0")
    w_pp = P.output_like(sub, u, v, dtype=torch.float64)
    P.contract_into(sub, u, v, w_pp, "bf16x3", steps=steps)
    assert torch.equal(w_il.data, w_pp.data)
    U64, V64 = H.to_np(u.data), H.to_np(v.data)
    ref, _ = O.contract_blocks(sub, U64, su, V64, sv)
    absref, _ = O.contract_blocks(sub, np.abs(U64), su, np.abs(V64), sv)
    k = H.contracted_extent(sub, su)
    assert np.all(np.abs(H.to_np(w_il.data) - ref) <= H.bound_factor("bf16x3", k) * absref + 1e-300)


@pytest.mark.parametrize("case", IL_CASES)
@pytest.mark.parametrize("wdt", ["f64", "f32"])
def test_wide_split_bf16_reads_u_in_place(P, case, wdt, monkeypatch):
    """The 256 x 256 wide split-bf16 tile reading binary32 U in place (split into
    hi/lo as its fragments are read): bit-identical to the three-step path (U on
    interleaved planes), to the same contraction with U at an odd element offset
    (aligned first) and with the in-place read switched off, and within the
    split-bf16 bound of the oracle."""
    sub, orders, cu, cv, du, dv = case
    monkeypatch.setenv("SYMT_GEMM_TILE", "bw256x256s2")
    monkeypatch.delenv("SYMT_BF16_IL", raising=False)
    monkeypatch.delenv("SYMT_BF16_FA", raising=False)
    rng = np.random.default_rng(sum(dv) * 11 + len(wdt))
    g = O.Group(orders)
    su = O.Sym.make(cu, int(rng.integers(g.size)), du, g)
    sv = O.Sym.make(cv, int(rng.integers(g.size)), dv, g)
    say(f"wide split-bf16 U in place {sub} G={orders} w={wdt}")
    u = _sym_tensor(P, rng.standard_normal(su.reduced_shape()), su, torch.float32)
    v = _sym_tensor(P, rng.standard_normal(sv.reduced_shape()), sv, torch.float32)
    wt = torch.float64 if wdt == "f64" else torch.float32
    w_fa = P.output_like(sub, u, v, dtype=wt)
    P.contract_into(sub, u, v, w_fa, "bf16x3")
    w_st = P.output_like(sub, u, v, dtype=wt)
    P.contract_into(sub, u, v, w_st, "bf16x3", steps=True)
    assert torch.equal(w_fa.data, w_st.data)
    buf = torch.zeros(u.data.numel() + 1, dtype=torch.float32, device=DEV)
    buf[1:] = u.data.reshape(-1)
    u_off = P.SymTensor(buf[1:].view(u.data.shape), u.signs, u.charge, u.group)
    w_o = P.output_like(sub, u, v, dtype=wt)
    P.contract_into(sub, u_off, v, w_o, "bf16x3")
    assert torch.equal(w_o.data, w_st.data)
    monkeypatch.setenv("SYMT_BF16_FA", "0")
    w_pl = P.output_like(sub, u, v, dtype=wt)
    P.contract_into(sub, u, v, w_pl, "bf16x3")
    assert torch.equal(w_pl.data, w_st.data)
    U64, V64 = H.to_np(u.data).astype(np.float64), H.to_np(v.data).astype(np.float64)
    ref, _ = O.contract_blocks(sub, U64, su, V64, sv)
    absref, _ = O.contract_blocks(sub, np.abs(U64), su, np.abs(V64), sv)
    k = H.contracted_extent(sub, su)
    w64 = H.to_np(w_fa.data).astype(np.float64)
    # (a binary32 W adds one rounding of each sum)
    extra = 0.0 if wdt == "f64" else H.U32
    assert np.all(np.abs(w64 - ref) <= H.bound_factor("bf16x3", k) * absref + extra * np.abs(ref) + 1e-300)


@pytest.mark.parametrize("steps", [False, True])
@pytest.mark.parametrize("tile", ["bw256x256s2", "bw256x128s3"])
def test_wide_split_bf16_pads_k_to_whole_steps(P, steps, tile, monkeypatch):
    """K = 280 on a wide split-bf16 tile: the planes take a zero pad to 288 (whole
    32-deep K-steps, interleaved) instead of leaving the wide tiles out; the
    U-aligned-first and three-step paths give the same bits, within the
    oracle's bound."""
    sub, orders, cu, cv, du, dv = "ak,kb->ab", (5,), "+-", "++", (300, 280), (280, 260)
    monkeypatch.setenv("SYMT_GEMM_TILE", tile)
    monkeypatch.delenv("SYMT_BF16_IL", raising=False)
    rng = np.random.default_rng(280 + len(tile))
    g = O.Group(orders)
    su = O.Sym.make(cu, int(rng.integers(g.size)), du, g)
    sv = O.Sym.make(cv, int(rng.integers(g.size)), dv, g)
    say(f"wide split-bf16 K pad {sub} tile={tile} steps={steps}")
    u = _sym_tensor(P, rng.standard_normal(su.reduced_shape()), su, torch.float64)
    v = _sym_tensor(P, rng.standard_normal(sv.reduced_shape()), sv, torch.float64)
    assert P.plan(sub, u, v, "bf16x3").k == 280
    w = P.output_like(sub, u, v, dtype=torch.float64)
    P.contract_into(sub, u, v, w, "bf16x3", steps=steps)
    w_other = P.output_like(sub, u, v, dtype=torch.float64)
    P.contract_into(sub, u, v, w_other, "bf16x3", steps=not steps)
    assert torch.equal(w.data, w_other.data)
    U64, V64 = H.to_np(u.data), H.to_np(v.data)
    ref, _ = O.contract_blocks(sub, U64, su, V64, sv)
    absref, _ = O.contract_blocks(sub, np.abs(U64), su, np.abs(V64), sv)
    k = H.contracted_extent(sub, su)
    assert np.all(np.abs(H.to_np(w.data) - ref) <= H.bound_factor("bf16x3", k) * absref + 1e-300)


# V read in place: contracted modes first in V, in U's K order; K runs of 32
# rows; V's trailing output run a multiple of 16 bytes (f64; the last case's run
# of 6 is not for f32)
VIP_CASES = [
    ("abkl,klij->abij", (4,), "++--", "++--", (3, 5, 4, 8), (4, 8, 2, 6)),
    ("ak,kb->ab", (5,), "+-", "++", (33, 32), (32, 20)),
    ("abkl,klij->abji", (3,), "+-+-", "-+++", (2, 7, 4, 8), (4, 8, 2, 4)),
    ("akl,klb->ab", (2, 3), "+-+", "-++", (7, 2, 16), (2, 16, 12)),
    ("abcd,cdij->abij", (8,), "++--", "++--", (5, 6, 4, 8), (4, 8, 3, 2)),
    ("ak,kb->ab", (2,), "+-", "++", (16, 4096), (4096, 12)),     # few tiles, long K: split K
]


@pytest.mark.parametrize("case", VIP_CASES)
@pytest.mark.parametrize("compute", ["f64", "f32"])
@pytest.mark.parametrize("tile,sk", [("d96x96s2", "0"), ("d96x96s2", "1"), ("d128x64s3", "0"),
                                     ("d128x64s3", "1"), ("d128x128s2", "1"), ("128x48", "0"),
                                     ("64x96", "0"), ("128x128", ""), ("rows", ""), ("", "")])
def test_fused_product_reads_v_in_place(P, case, compute, tile, sk, monkeypatch):
    """Products reading B from V's standard form through its row and column
    tables, on global-to-LDS tiles (stream-K on and off), register tiles and
    split K: bit-identical to the three-step path on the same tile, within the
    product's bound of the oracle, with and without charge tables; a V that is
    not 16-byte aligned is aligned first and gives the same bits."""
    sub, orders, cu, cv, du, dv = case
    for name, val in (("SYMT_GEMM_TILE", tile), ("SYMT_GEMM_SK", sk)):
        if val:
            monkeypatch.setenv(name, val)
        else:
            monkeypatch.delenv(name, raising=False)
    rng = np.random.default_rng(len(sub) * 17 + sum(dv))
    g = O.Group(orders)
    su0 = O.Sym.make(cu, int(rng.integers(g.size)), du, g)
    sv0 = O.Sym.make(cv, int(rng.integers(g.size)), dv, g)
    dt = torch.float64 if compute == "f64" else torch.float32
    # V's trailing output run must hold whole 16-byte chunks (4 binary32)
    run_ok = compute == "f64" or dv[-1] * (dv[-2] if len(sub.split(",")[1].split("->")[0]) > 2 else 1) % 4 == 0
    for tables in (False, True):
        su, sv = _with_tables(rng, sub, su0, sv0) if tables else (su0, sv0)
        say(f"v in place {sub} G={orders} {compute} tile={tile} sk={sk} tables={tables}")
        Ru = rng.standard_normal(su.reduced_shape())
        Rv = rng.standard_normal(sv.reduced_shape())
        u = _sym_tensor(P, Ru, su, dt)
        v = _sym_tensor(P, Rv, sv, dt)
        info = P.plan(sub, u, v, compute)
        assert info.fused == 1
        assert info.fused_v == int(run_ok)
        w_f = P.output_like(sub, u, v, dtype=dt)
        w_s = P.output_like(sub, u, v, dtype=dt)
        P.contract_into(sub, u, v, w_f, compute)
        P.contract_into(sub, u, v, w_s, compute, steps=True)
        assert torch.equal(w_f.data, w_s.data)
        ref, _ = O.contract_blocks(sub, H.to_np(u.data).astype(np.float64), su,
                                   H.to_np(v.data).astype(np.float64), sv)
        absref, _ = O.contract_blocks(sub, np.abs(H.to_np(u.data).astype(np.float64)), su,
                                      np.abs(H.to_np(v.data).astype(np.float64)), sv)
        k = H.contracted_extent(sub, su)
        fac = 2 * H.gamma(k, H.U64) if compute == "f64" else 1.05 * H.gamma(k, H.U32) + H.gamma(k, H.U64)
        assert np.all(np.abs(H.to_np(w_f.data) - ref) <= fac * absref + 1e-300)
        # V starting one element into a buffer: not 16-byte aligned, so V_al is written
        buf = torch.zeros(v.data.numel() + 1, dtype=dt, device=DEV)
        buf[1:] = v.data.reshape(-1)
        v_off = P.SymTensor(buf[1:].view(v.data.shape), v.signs, v.charge, v.group, v.mode_charges)
        w_o = P.output_like(sub, u, v, dtype=dt)
        P.contract_into(sub, u, v_off, w_o, compute)
        assert torch.equal(w_o.data, w_s.data)


@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_row_streaming_product(P, compute, monkeypatch):
    """The row-streaming product (K and N at most 64): forced on small and
    ragged shapes (K and N of 1, not multiples of 4 or 16, and 64; one row;
    many slices) and taken by default on tall ones, within the product's bound
    of an FP64 matmul and run-to-run identical."""
    monkeypatch.delenv("SYMT_GEMM_SK", raising=False)
    cases = [("rows", (1, 1, 1, 1)), ("rows", (3, 5, 3, 7)), ("rows", (2, 33, 64, 64)), ("rows", (5, 100, 17, 1)),
             ("rows", (1, 16, 32, 4)), ("rows", (7, 61, 48, 48)), ("rows", (300, 3, 8, 16)),
             ("", (6, 3000, 48, 48)), ("", (1, 40000, 13, 50)), ("", (2, 9000, 64, 33))]
    for tile, shape in cases:
        if tile:
            monkeypatch.setenv("SYMT_GEMM_TILE", tile)
        else:
            monkeypatch.delenv("SYMT_GEMM_TILE", raising=False)
        b, m, k, n = shape
        say(f"row product {compute} tile={tile or 'default'} {shape}")
        rng = np.random.default_rng(m * 7 + n + k)
        dt = torch.float64 if compute == "f64" else torch.float32
        a = torch.from_numpy(rng.standard_normal((b, m, k))).to(DEV, dt)
        bb = torch.from_numpy(rng.standard_normal((b, k, n))).to(DEV, dt)
        C = H.to_np(P.sector_gemm(a, bb, compute))
        A64, B64 = H.to_np(a).astype(np.float64), H.to_np(bb).astype(np.float64)
        ref = np.matmul(A64, B64)
        absb = np.matmul(np.abs(A64), np.abs(B64))
        fac = 2 * H.gamma(k, H.U64) if compute == "f64" else 1.05 * H.gamma(k, H.U32)
        assert np.all(np.abs(C - ref) <= fac * absb + 1e-300), (compute, shape)
        assert np.array_equal(H.to_np(P.sector_gemm(a, bb, compute)), C)


@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_long_k_product(P, compute, monkeypatch):
    """The long-K product (M and N at most 64): forced on small and ragged shapes
    (M, N of 1 and 64, K of 3 and not a multiple of 16, one and many slices)
    and taken by default on long K, within the product's bound of an FP64
    matmul and run-to-run identical (ranges summed in order)."""
    monkeypatch.delenv("SYMT_GEMM_SK", raising=False)
    cases = [("tallk", (1, 1, 1, 1)), ("tallk", (2, 16, 3, 16)), ("tallk", (3, 17, 5000, 33)),
             ("tallk", (2, 64, 1030, 64)), ("tallk", (1, 5, 4097, 1)), ("tallk", (700, 3, 40, 2)),
             ("", (6, 48, 20000, 48)), ("", (1, 64, 300000, 64)), ("", (2, 9, 1024, 50))]
    for tile, shape in cases:
        if tile:
            monkeypatch.setenv("SYMT_GEMM_TILE", tile)
        else:
            monkeypatch.delenv("SYMT_GEMM_TILE", raising=False)
        b, m, k, n = shape
        say(f"long-K product {compute} tile={tile or 'default'} {shape}")
        rng = np.random.default_rng(m * 5 + n + k)
        dt = torch.float64 if compute == "f64" else torch.float32
        a = torch.from_numpy(rng.standard_normal((b, m, k))).to(DEV, dt)
        bb = torch.from_numpy(rng.standard_normal((b, k, n))).to(DEV, dt)
        C = H.to_np(P.sector_gemm(a, bb, compute))
        A64, B64 = H.to_np(a).astype(np.float64), H.to_np(bb).astype(np.float64)
        ref = np.matmul(A64, B64)
        absb = np.matmul(np.abs(A64), np.abs(B64))
        fac = 2 * H.gamma(k, H.U64) if compute == "f64" else 1.05 * H.gamma(k, H.U32)
        assert np.all(np.abs(C - ref) <= fac * absb + 1e-300), (compute, shape)
        assert np.array_equal(H.to_np(P.sector_gemm(a, bb, compute)), C)


@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_long_k_lds_variant(P, compute, monkeypatch):
    """The long-K product's global-to-LDS variant (K in whole 16-deep groups,
    N in whole 16-byte chunks): within the product's bound of an FP64 matmul on
    ragged M and N (rows and chunks clamped), one group, more slices than
    ranges, every LDS swizzle of B (rows of 32, 36, 48 and 64 columns), and
    run-to-run identical.  (Its bits equal the register variant's: see the
    in-place long-K cases, whose fused and three-step paths take different
    variants.)"""
    monkeypatch.setenv("SYMT_GEMM_TILE", "tallk")
    monkeypatch.delenv("SYMT_GEMM_SK", raising=False)
    dt = torch.float64 if compute == "f64" else torch.float32
    for shape in [(6, 48, 20000, 48), (2, 1, 512, 4), (5, 33, 1600, 20), (3, 64, 4096, 64),
                  (1, 64, 16, 64), (700, 3, 48, 4), (2, 17, 2048, 36), (4, 48, 3072, 32)]:
        b, m, k, n = shape
        say(f"long-K global-to-LDS {compute} {shape}")
        rng = np.random.default_rng(m * 7 + n + k)
        a = torch.from_numpy(rng.standard_normal((b, m, k))).to(DEV, dt)
        bb = torch.from_numpy(rng.standard_normal((b, k, n))).to(DEV, dt)
        C = H.to_np(P.sector_gemm(a, bb, compute))
        A64, B64 = H.to_np(a).astype(np.float64), H.to_np(bb).astype(np.float64)
        ref = np.matmul(A64, B64)
        absb = np.matmul(np.abs(A64), np.abs(B64))
        fac = 2 * H.gamma(k, H.U64) if compute == "f64" else 1.05 * H.gamma(k, H.U32)
        assert np.all(np.abs(C - ref) <= fac * absb + 1e-300), (compute, shape)
        assert np.array_equal(H.to_np(P.sector_gemm(a, bb, compute)), C)


ROW_CASES = [
    # W's rows contiguous (its last modes from U): lanes store along rows
    ("cASB,bsSB->bcsA", (2, 3), "----", "+---", (6, 16, 2, 4), (4, 2, 2, 4)),
    ("ak,kb->ba", (2, 3), "--", "-+", (17, 32), (32, 8)),
    # W's columns contiguous: lanes store along columns
    ("bcsA,bsSB->cASB", (2, 3), "--+-", "+---", (4, 6, 2, 16), (4, 2, 2, 4)),
    ("abkl,klij->abij", (4,), "++--", "++--", (3, 5, 4, 4), (4, 4, 2, 6)),
    # odd K and N
    ("akl,klb->ab", (3,), "+-+", "-++", (7, 3, 5), (3, 5, 13)),
]


# Long K with M and N at most 64 (a gradient with respect to a small operand).
TALLK_CASES = [
    # (K in whole 16-deep groups of U's and V's runs: the global-to-LDS variant on both paths)
    ("bcsA,cASB->bsSB", (2, 3), "--+-", "----", (4, 16, 2, 16), (16, 16, 2, 4)),
    ("ak,kb->ab", (5,), "+-", "++", (7, 3000), (3000, 9)),
    ("klab,klc->abc", (3,), "++-+", "--+", (40, 30, 2, 3), (40, 30, 5)),
    # U's contracted modes lead: the register variant in place, the global-to-LDS
    # variant on U_al (three steps); the two must give the same bits
    ("klab,klc->abc", (3,), "++-+", "--+", (40, 32, 2, 4), (40, 32, 4)),
    ("ak,kb->ab", (5,), "+-", "++", (7, 3200), (3200, 10)),
]


@pytest.mark.parametrize("case", [("rows", c) for c in ROW_CASES] + [("tallk", c) for c in TALLK_CASES])
@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_short_products_in_place(P, case, compute, monkeypatch):
    """The row-streaming product (K, N <= 64) and the long-K product (M, N <=
    64) forced on fused contractions (U and V read in place where they can, W
    written in place; row-streaming lanes along W's contiguous index):
    bit-identical to the three-step path on the same kernel (the transposed
    MFMA forms the same products in the same K order), within the product's
    bound of the oracle, with and without charge tables."""
    tile, (sub, orders, cu, cv, du, dv) = case
    monkeypatch.setenv("SYMT_GEMM_TILE", tile)
    monkeypatch.delenv("SYMT_GEMM_SK", raising=False)
    rng = np.random.default_rng(seed("rows", sub, orders))
    g = O.Group(orders)
    su0 = O.Sym.make(cu, int(rng.integers(g.size)), du, g)
    sv0 = O.Sym.make(cv, int(rng.integers(g.size)), dv, g)
    dt = torch.float64 if compute == "f64" else torch.float32
    for tables in (False, True):
        su, sv = _with_tables(rng, sub, su0, sv0) if tables else (su0, sv0)
        say(f"{tile} in place {sub} G={orders} {compute} tables={tables}")
        Ru = rng.standard_normal(su.reduced_shape())
        Rv = rng.standard_normal(sv.reduced_shape())
        u = _sym_tensor(P, Ru, su, dt)
        v = _sym_tensor(P, Rv, sv, dt)
        info = P.plan(sub, u, v, compute)
        assert info.fused_w == 1
        w_f = P.output_like(sub, u, v, dtype=dt)
        w_s = P.output_like(sub, u, v, dtype=dt)
        P.contract_into(sub, u, v, w_f, compute)
        P.contract_into(sub, u, v, w_s, compute, steps=True)
        assert torch.equal(w_f.data, w_s.data)
        ref, _ = O.contract_blocks(sub, H.to_np(u.data).astype(np.float64), su,
                                   H.to_np(v.data).astype(np.float64), sv)
        absref, _ = O.contract_blocks(sub, np.abs(H.to_np(u.data).astype(np.float64)), su,
                                      np.abs(H.to_np(v.data).astype(np.float64)), sv)
        k = H.contracted_extent(sub, su)
        fac = 2 * H.gamma(k, H.U64) if compute == "f64" else 1.05 * H.gamma(k, H.U32) + H.gamma(k, H.U64)
        assert np.all(np.abs(H.to_np(w_f.data) - ref) <= fac * absref + 1e-300)


def test_cached_offset_tables_across_streams_and_alignments(P):
    """A plan's offset tables are built once on the context (on the stream of
    its first call) and reused: a first call whose V is not 16-byte aligned
    (V aligned first, four tables used), then calls reading V in place (six
    tables) on a second stream, then on the first again, with new data each
    time, with and without charge tables: every call bit-identical to the
    three-step path and within the product's bound of the oracle."""
    sub, orders, cu, cv = "abkl,klij->abij", (4,), "++--", "++--"
    du, dv = (3, 7, 4, 8), (4, 8, 5, 6)          # shapes no other test plans
    rng = np.random.default_rng(91)
    g = O.Group(orders)
    su0 = O.Sym.make(cu, 1, du, g)
    sv0 = O.Sym.make(cv, 3, dv, g)
    side = torch.cuda.Stream(device=DEV)
    for tables in (False, True):
        su, sv = _with_tables(rng, sub, su0, sv0) if tables else (su0, sv0)
        for call, (stream, aligned) in enumerate(((None, False), (side, True), (None, True), (side, False))):
            say(f"cached tables tables={tables} call={call} side={stream is not None} aligned_v={aligned}")
            Ru = rng.standard_normal(su.reduced_shape())
            Rv = rng.standard_normal(sv.reduced_shape())
            u = _sym_tensor(P, Ru, su)
            v = _sym_tensor(P, Rv, sv)
            if not aligned:
                buf = torch.zeros(v.data.numel() + 1, dtype=torch.float64, device=DEV)
                buf[1:] = v.data.reshape(-1)
                v = P.SymTensor(buf[1:].view(v.data.shape), v.signs, v.charge, v.group, v.mode_charges)
            info = P.plan(sub, u, v, "f64")
            assert info.fused == 1 and info.fused_v == 1
            w_f = P.output_like(sub, u, v)
            w_s = P.output_like(sub, u, v)
            if stream is not None:
                stream.wait_stream(torch.cuda.current_stream(DEV))
                with torch.cuda.stream(stream):
                    P.contract_into(sub, u, v, w_f, "f64")
                torch.cuda.current_stream(DEV).wait_stream(stream)
            else:
                P.contract_into(sub, u, v, w_f, "f64")
            P.contract_into(sub, u, v, w_s, "f64", steps=True)
            torch.cuda.synchronize(DEV)
            assert torch.equal(w_f.data, w_s.data), call
            ref, _ = O.contract_blocks(sub, Ru, su, Rv, sv)
            absref, _ = O.contract_blocks(sub, np.abs(Ru), su, np.abs(Rv), sv)
            k = H.contracted_extent(sub, su)
            assert np.all(np.abs(H.to_np(w_f.data) - ref) <= 2 * H.gamma(k, H.U64) * absref + 1e-300), call


@pytest.mark.parametrize("tile,sk", [("d128x128s2", "0"), ("d128x96s2", "0"), ("d128x64s3", "0"),
                                     ("d96x96s3", "0"), ("128x48", "0"), ("64x96", "0"),
                                     ("d128x128s2", "1"), ("d128x96s2", "1"), ("d128x64s3", "1"),
                                     ("d96x96s3", "1"), ("d96x96s2", "0"), ("d96x96s2", "1")])
@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_sector_gemm_every_tile_on_ragged_shapes(P, tile, sk, compute, monkeypatch):
    """Each tile shape, forced, on shapes that leave partial tiles in M and N;
    sk = "1" forces stream-K, whose tiles are cut into 1 to 8 pieces here."""
    monkeypatch.setenv("SYMT_GEMM_TILE", tile)
    monkeypatch.setenv("SYMT_GEMM_SK", sk)
    for shape in ((2, 130, 64, 68), (3, 257, 96, 196), (1, 16, 32, 4), (2, 200, 512, 100)):
        b, m, k, n = shape
        say(f"sector_gemm tile={tile} sk={sk} {compute} {shape}")
        rng = np.random.default_rng(m + n + k)
        dt = torch.float64 if compute == "f64" else torch.float32
        a = torch.from_numpy(rng.standard_normal((b, m, k))).to(DEV, dt)
        bb = torch.from_numpy(rng.standard_normal((b, k, n))).to(DEV, dt)
        C = H.to_np(P.sector_gemm(a, bb, compute))
        A64, B64 = H.to_np(a).astype(np.float64), H.to_np(bb).astype(np.float64)
        ref = np.matmul(A64, B64)
        absb = np.matmul(np.abs(A64), np.abs(B64))
        fac = 2 * H.gamma(k, H.U64) if compute == "f64" else 1.05 * H.gamma(k, H.U32)
        assert np.all(np.abs(C - ref) <= fac * absb), (tile, compute, shape)
        # the same launch again gives the same bits (pieces are summed in K order)
        assert np.array_equal(H.to_np(P.sector_gemm(a, bb, compute)), C)



# ---------------------------------------------------------------------------
# charge tables: every sector label of a mode carries a permuted charge
# ---------------------------------------------------------------------------
def _with_tables(rng, sub, su, sv):
    tu, rest = sub.split(",")
    tv, _ = rest.split("->")
    G = su.group.size
    tab = {m: tuple(int(x) for x in rng.permutation(G)) for m in set(tu) | set(tv)}
    return (O.Sym.make(su.signs, su.charge, su.dims, su.group, [tab[m] for m in tu]),
            O.Sym.make(sv.signs, sv.charge, sv.dims, sv.group, [tab[m] for m in tv]))


@pytest.mark.parametrize("case", [((4,), 2, 2, 2), ((3,), 1, 1, 1), ((2, 3), 2, 1, 2), ((5,), 1, 2, 1),
                                  ((8,), 2, 2, 2)])
def test_contract_with_charge_tables_vs_oracle(P, case):
    orders, ns, nt, nv = case
    rng = np.random.default_rng(seed(("charges",) + case))
    for rep in range(2):
        sub, su0, sv0 = H.random_case(rng, orders, ns, nt, nv, nmax=5)
        su, sv = _with_tables(rng, sub, su0, sv0)
        say(f"charge tables {sub} G={orders} rep={rep}")
        Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
        ref, sw = O.contract_blocks(sub, Ru, su, Rv, sv)
        absref, _ = O.contract_blocks(sub, np.abs(Ru), su, np.abs(Rv), sv)
        k = H.contracted_extent(sub, su)
        u, v = _sym_tensor(P, Ru, su), _sym_tensor(P, Rv, sv)
        for compute in ("f64", "f32", "bf16x3"):
            info = P.plan(sub, u, v, compute)
            w = P.output_like(sub, u, v)
            assert w.mode_charges == sw.charges
            P.contract_into(sub, u, v, w, compute)
            got = H.to_np(w.data)
            assert np.all(np.abs(got - ref) <= H.bound_factor(compute, k) * absref + 1e-300), compute
            if compute == "f64":
                assert H.rel_err(got, ref) <= 1e-12
                ws = P.output_like(sub, u, v)
                P.contract_into(sub, u, v, ws, compute, steps=True)
                assert torch.equal(ws.data, w.data)          # fused (where it applies) == three steps


def test_charge_tables_fused_path_and_gradient(P):
    """A fused-layout contraction (trailing contracted modes) with tables, and its backward."""
    rng = np.random.default_rng(31)
    g = O.Group((4,))
    su0 = O.Sym.make("++--", 1, (3, 2, 4, 4), g)
    sv0 = O.Sym.make("++--", 2, (4, 4, 2, 3), g)
    sub = "abkl,klij->abij"
    su, sv = _with_tables(rng, sub, su0, sv0)
    Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
    u, v = _sym_tensor(P, Ru, su), _sym_tensor(P, Rv, sv)
    assert P.plan(sub, u, v, "f64").fused
    ud = u.data.clone().requires_grad_(True)
    vd = v.data.clone().requires_grad_(True)
    w = P.einsum(sub, P.SymTensor(ud, u.signs, u.charge, u.group, u.mode_charges),
                 P.SymTensor(vd, v.signs, v.charge, v.group, v.mode_charges))
    ref, sw = O.contract_blocks(sub, Ru, su, Rv, sv)
    assert H.rel_err(H.to_np(w.data), ref) <= 1e-12
    Rg = rng.standard_normal(sw.reduced_shape())
    (w.data * torch.from_numpy(Rg).to(DEV)).sum().backward()
    # dU = dW . V over J; dV = U . dW over I, with the same tables
    gu_ref, _ = O.contract_blocks("abij,klij->abkl", Rg, sw, Rv, sv)
    gv_ref, _ = O.contract_blocks("abkl,abij->klij", Ru, su, Rg, sw)
    assert H.rel_err(H.to_np(ud.grad), gu_ref) <= 1e-12
    assert H.rel_err(H.to_np(vd.grad), gv_ref) <= 1e-12


@pytest.mark.parametrize("tile", ["bw256x256s2", "bw256x128s3"])
def test_charge_tables_on_wide_split_bf16_tiles(P, tile, monkeypatch):
    """Charge tables with the wide split-bf16 tiles: U (binary32) read in place on the
    256 x 256 tile, or aligned onto interleaved planes on the 256 x 128 one; the same
    bits as the three-step path, within the oracle's bound."""
    monkeypatch.setenv("SYMT_GEMM_TILE", tile)
    rng = np.random.default_rng(47 + len(tile))
    g = O.Group((8,))
    sub = "abcd,cdij->abij"
    su0 = O.Sym.make("++--", 3, (3, 5, 2, 2), g)
    sv0 = O.Sym.make("++--", 5, (2, 2, 4, 9), g)
    su, sv = _with_tables(rng, sub, su0, sv0)
    say(f"charge tables on wide split-bf16 tile {tile}")
    Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
    u, v = _sym_tensor(P, Ru, su, torch.float32), _sym_tensor(P, Rv, sv, torch.float32)
    w = P.output_like(sub, u, v, dtype=torch.float64)
    P.contract_into(sub, u, v, w, "bf16x3")
    ws = P.output_like(sub, u, v, dtype=torch.float64)
    P.contract_into(sub, u, v, ws, "bf16x3", steps=True)
    assert torch.equal(w.data, ws.data)
    U64, V64 = H.to_np(u.data).astype(np.float64), H.to_np(v.data).astype(np.float64)
    ref, _ = O.contract_blocks(sub, U64, su, V64, sv)
    absref, _ = O.contract_blocks(sub, np.abs(U64), su, np.abs(V64), sv)
    k = H.contracted_extent(sub, su)
    assert np.all(np.abs(H.to_np(w.data) - ref) <= H.bound_factor("bf16x3", k) * absref + 1e-300)


def test_charge_tables_rejected_by_standalone_align(P):
    rng = np.random.default_rng(3)
    g = O.Group((3,))
    su, sv = _with_tables(rng, "ak,kb->ab", O.Sym.make("+-", 0, (2, 3), g), O.Sym.make("+-", 0, (3, 2), g))
    u = _sym_tensor(P, rng.standard_normal(su.reduced_shape()), su)
    v = _sym_tensor(P, rng.standard_normal(sv.reduced_shape()), sv)
    with pytest.raises(P._lib.SymtError) as e:
        P.align("ak,kb->ab", u, v, 0)
    assert e.value.code == P._lib.SYMT_EUNSUPPORTED


# ---------------------------------------------------------------------------
# s, t or v = 0: Q pinned to one value, the product on a single slice
# ---------------------------------------------------------------------------
DEGENERATE = ["a,b->ab", "ab,c->abc", "ab,cd->acbd",        # v = 0: outer products
              "k,kb->b", "kl,klij->ij", "lk,klb->b",         # s = 0
              "ak,k->a", "abk,k->ab", "akl,lk->a"]           # t = 0


def _degenerate_case(rng, sub, orders, nmax=5):
    g = O.Group(orders)
    tu, rest = sub.split(",")
    tv, tw = rest.split("->")
    dims = {m: int(rng.integers(1, nmax + 1)) for m in set(tu + tv)}
    cu = {m: int(rng.choice([-1, 1])) for m in tu}
    sigma = int(rng.choice([-1, 1]))
    cv = {m: (sigma * cu[m] if m in tu else int(rng.choice([-1, 1]))) for m in tv}
    su = O.Sym.make([cu[m] for m in tu], int(rng.integers(g.size)), [dims[m] for m in tu], g)
    sv = O.Sym.make([cv[m] for m in tv], int(rng.integers(g.size)), [dims[m] for m in tv], g)
    return su, sv


@pytest.mark.parametrize("sub", DEGENERATE)
@pytest.mark.parametrize("orders", [(4,), (2, 3)])
def test_degenerate_contractions_vs_oracle(P, sub, orders):
    rng = np.random.default_rng(seed(("degenerate", sub, orders)))
    for with_tables in (False, True):
        su, sv = _degenerate_case(rng, sub, orders)
        if with_tables:
            su, sv = _with_tables(rng, sub, su, sv)
        say(f"degenerate {sub} G={orders} tables={with_tables}")
        Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
        ref, sw = O.contract_blocks(sub, Ru, su, Rv, sv)
        absref, _ = O.contract_blocks(sub, np.abs(Ru), su, np.abs(Rv), sv)
        k = H.contracted_extent(sub, su) if "," in sub and set(sub.split(",")[0]) & set(sub.split(",")[1].split("->")[0]) else 1
        u, v = _sym_tensor(P, Ru, su), _sym_tensor(P, Rv, sv)
        assert P.plan(sub, u, v).flops == O.flop_count(sub, su, sv)
        for compute in ("f64", "f32", "bf16x3"):
            info = P.plan(sub, u, v, compute)
            w = P.output_like(sub, u, v)
            w.data.fill_(7.0)                      # every element must be overwritten
            assert w.signs == sw.sign_string() and w.charge == sw.charge
            P.contract_into(sub, u, v, w, compute)
            got = H.to_np(w.data)
            assert np.all(np.abs(got - ref) <= H.bound_factor(compute, k) * absref + 1e-300), compute
            if compute == "f64":
                assert H.rel_err(got, ref) <= 1e-12 or np.max(np.abs(ref)) == 0
                assert np.array_equal(O.expand(got, sw) == 0, O.expand(ref, sw) == 0)
        if not with_tables:
            # steps (a) and (c) alone, bit-exact against Alg. 2 with dense deltas (zero Q slices included)
            Ual, Val = O.align_u(sub, Ru, su, sv), O.align_v(sub, Rv, su, sv)
            for op, ref_al in ((0, Ual), (1, Val)):
                # into a NaN-filled buffer: the slices that must be zero are written too
                for compute, dt in (("f64", torch.float64), ("f32", torch.float32)):
                    buf = torch.full(ref_al.shape, float("nan"), dtype=dt, device=DEV)
                    got_al = H.to_np(P.align(sub, u, v, op, compute, out=buf))
                    assert np.array_equal(got_al, ref_al.astype(got_al.dtype)), (op, compute)
            Wal = np.matmul(Ual, Val)
            ref_w, _ = O.unalign_w(sub, Wal, su, sv)
            w = P.output_like(sub, u, v)
            w.data.fill_(3.0)
            P.unalign(sub, u, v, w, torch.from_numpy(Wal).to(DEV), "f64")
            assert np.array_equal(H.to_np(w.data), ref_w)


# ---------------------------------------------------------------------------
# U(1) emulated by Z_G with per-mode charge tables (Sec. 3): the library's
# result, expanded, is the dense U(1) einsum at the labels that carry U(1)
# charges and zero elsewhere.  The reference is np.einsum on dense U(1)
# tensors built with integer charges, independent of the oracle's contraction.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("sub", ["ij,jk->ik", "ijk,klm->ijlm", "abcd,cdij->abij", "ak,k->a", "a,b->ab"])
def test_u1_emulation_vs_dense_u1_einsum(P, sub):
    from tests import u1_cases as U1
    rng = np.random.default_rng(seed(("u1-gpu", sub)))
    for g_extra in (0, 3):
        c = U1.random_case(rng, sub, g_extra, nmax=4)
        say(f"u1 {sub} G={c['G']}")
        u, v = _sym_tensor(P, c["Ru"], c["su"]), _sym_tensor(P, c["Rv"], c["sv"])
        sw = O.output_symmetry(sub, c["su"], c["sv"])
        absref = np.einsum(sub, np.abs(c["Tu"]), np.abs(c["Tv"]))
        k = P.plan(sub, u, v).k + int(np.prod([d for m, d in zip(sub.split(",")[0], c["Tu"].shape)
                                                 if m in sub.split(",")[1].split("->")[0]]))
        for compute in ("f64", "f32", "bf16x3"):
            w = P.output_like(sub, u, v)
            w.data.fill_(7.0)
            P.contract_into(sub, u, v, w, compute)
            phys, rest = U1.physical_part(O.expand(H.to_np(w.data), sw), c["Pw"], c["nw"])
            assert rest == 0.0, compute
            assert np.all(np.abs(phys - c["ref"]) <= H.bound_factor(compute, k) * absref + 1e-300), compute


# ---------------------------------------------------------------------------
# Complex operands (Sec. 2.2 allows tensors over C): the product runs on the
# real representation of C.  Results against the complex oracle; the aligned
# forms bit-exact against Alg. 2 with dense deltas (U_al and W_al are the
# complex forms viewed as interleaved reals; V_al's even real rows hold V, its
# odd rows i V); gradients against dense complex autograd on the CPU.
# ---------------------------------------------------------------------------
COMPLEX_CASES = [((4,), 1, 1, 1), ((3,), 2, 1, 2), ((2, 3), 1, 2, 1), ((5,), 2, 2, 1),
                 ((4,), 1, 1, 0), ((3,), 0, 2, 1), ((3,), 2, 0, 1)]


def _cplx(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("orders,s,t,v", COMPLEX_CASES)
def test_complex_contractions_vs_oracle(P, orders, s, t, v):
    rng = np.random.default_rng(seed(("cplx-gpu", orders, s, t, v)))
    for with_tables in (False, True):
        sub, su, sv = H.random_case(rng, orders, s, t, v, nmax=5)
        if with_tables:
            su, sv = _with_tables(rng, sub, su, sv)
        say(f"complex {sub} G={orders} tables={with_tables}")
        Ru, Rv = _cplx(rng, su.reduced_shape()), _cplx(rng, sv.reduced_shape())
        ref, sw = O.contract_blocks(sub, Ru, su, Rv, sv)
        absref, _ = O.contract_blocks(sub, np.abs(Ru), su, np.abs(Rv), sv)
        u, v_ = _sym_tensor(P, Ru, su, torch.complex128), _sym_tensor(P, Rv, sv, torch.complex128)
        info = P.plan(sub, u, v_)
        assert info.flops == 4 * O.flop_count(sub, su, sv)      # 8 real flops per complex multiply-add
        k = info.k                                              # real terms per output component
        for compute in ("f64", "f32", "bf16x3"):
            w = P.output_like(sub, u, v_)
            assert w.data.dtype == torch.complex128
            w.data.fill_(7.0 + 7.0j)
            P.contract_into(sub, u, v_, w, compute)
            got = H.to_np(w.data)
            # each component is a real sum of 2 K terms bounded by |u||v| (Cauchy-Schwarz);
            # split-bf16 and f32 round the inputs to binary32 first
            for part in (np.real, np.imag):
                assert np.all(np.abs(part(got) - part(ref)) <= H.bound_factor(compute, k) * absref + 1e-300), compute
            if compute == "f64":
                assert H.rel_err(got, ref) <= 1e-12 or np.max(np.abs(ref)) == 0
        if not with_tables:
            Ual, Val = O.align_u(sub, Ru, su, sv), O.align_v(sub, Rv, su, sv)
            bu = torch.full((Ual.shape[0], Ual.shape[1], 2 * Ual.shape[2]), float("nan"), dtype=torch.float64, device=DEV)
            gu = H.to_np(P.align(sub, u, v_, 0, "f64", out=bu))
            assert np.array_equal(gu.view(np.complex128), Ual)
            bv = torch.full((Val.shape[0], 2 * Val.shape[1], 2 * Val.shape[2]), float("nan"), dtype=torch.float64,
                            device=DEV)
            gv = H.to_np(P.align(sub, u, v_, 1, "f64", out=bv))
            assert np.array_equal(np.ascontiguousarray(gv[:, 0::2, :]).view(np.complex128), Val)
            assert np.array_equal(np.ascontiguousarray(gv[:, 1::2, :]).view(np.complex128), 1j * Val)
            Wal = np.matmul(Ual, Val)
            ref_w, _ = O.unalign_w(sub, Wal, su, sv)
            w = P.output_like(sub, u, v_)
            w.data.fill_(3.0)
            P.unalign(sub, u, v_, w, torch.from_numpy(np.ascontiguousarray(Wal).view(np.float64)).to(DEV), "f64")
            assert np.array_equal(H.to_np(w.data), ref_w)


def test_complex_split_bf16_on_global_to_lds_tiles(P):
    """Complex operands under split-bf16 at a size that takes the global-to-LDS
    tiles (M >= 256, N >= 512 reals) with a contracted extent that is not a
    multiple of 8 (77 complex = 154 reals, padded to 160): within the product's
    bound of the oracle, componentwise."""
    rng = np.random.default_rng(seed(("cplx-bf16", 77)))
    g = O.Group((4,))
    sub = "ak,kb->ab"
    su, sv = O.Sym.make("+-", 1, (300, 77), g), O.Sym.make("++", 3, (77, 300), g)
    Ru, Rv = _cplx(rng, su.reduced_shape()), _cplx(rng, sv.reduced_shape())
    u, v = _sym_tensor(P, Ru, su, torch.complex128), _sym_tensor(P, Rv, sv, torch.complex128)
    info = P.plan(sub, u, v, "bf16x3")
    assert (info.m, info.k, info.n) == (300, 154, 600) and info.fused == 0
    say("complex split-bf16 ak,kb->ab G=4 (300 x 77 x 300)")
    w = P.output_like(sub, u, v)
    w.data.fill_(7.0 + 7.0j)
    P.contract_into(sub, u, v, w, "bf16x3")
    got = H.to_np(w.data)
    # the oracle on binary32-rounded inputs (the split starts from binary32)
    R32u = Ru.real.astype(np.float32) + 1j * Ru.imag.astype(np.float32)
    R32v = Rv.real.astype(np.float32) + 1j * Rv.imag.astype(np.float32)
    ref, _ = O.contract_blocks(sub, R32u.astype(np.complex128), su, R32v.astype(np.complex128), sv)
    absref, _ = O.contract_blocks(sub, np.abs(Ru), su, np.abs(Rv), sv)
    for part in (np.real, np.imag):
        assert np.all(np.abs(part(got) - part(ref)) <= H.bound_factor("bf16x3", info.k) * absref + 1e-300)


@pytest.mark.parametrize("orders,s,t,v", [((3,), 1, 1, 1), ((2, 2), 2, 1, 1), ((4,), 1, 1, 0)])
def test_complex_gradients_vs_dense_autograd(P, orders, s, t, v):
    rng = np.random.default_rng(seed(("cplx-grad", orders, s, t, v)))
    sub, su, sv = H.random_case(rng, orders, s, t, v, nmax=4)
    say(f"complex gradient {sub} G={orders}")
    Ru, Rv = _cplx(rng, su.reduced_shape()), _cplx(rng, sv.reduced_shape())
    sw = O.output_symmetry(sub, su, sv)
    Rr = _cplx(rng, sw.reduced_shape())
    ud = torch.from_numpy(Ru).to(DEV).requires_grad_(True)
    vd = torch.from_numpy(Rv).to(DEV).requires_grad_(True)
    w = P.einsum(sub, P.SymTensor(ud, su.sign_string(), su.charge, su.group.orders),
                 P.SymTensor(vd, sv.sign_string(), sv.charge, sv.group.orders))
    loss = (w.data * torch.from_numpy(Rr).to(DEV)).sum().real
    loss.backward()
    du = torch.from_numpy(O.expand(Ru, su)).requires_grad_(True)
    dv = torch.from_numpy(O.expand(Rv, sv)).requires_grad_(True)
    dloss = (torch.einsum(sub, du, dv) * torch.from_numpy(O.expand(Rr, sw))).sum().real
    dloss.backward()
    assert abs(loss.item() - dloss.item()) <= 1e-12 * max(1.0, abs(dloss.item()))
    for got, dense, sym in ((ud.grad, du.grad, su), (vd.grad, dv.grad, sv)):
        ref, zero_ok = O.reduce_full(dense.numpy(), sym)
        assert zero_ok
        assert H.rel_err(H.to_np(got), ref) <= 1e-12


# ---------------------------------------------------------------------------
# Subgroup modes (Sec. 2.2, Eq. symtsr with c_i = +-G/H_i): against the oracle
# in three precisions; stored tuples of W without a block come out zero; the
# standalone transforms bit-exact against Alg. 2 with dense deltas (aligned
# blocks without a standard block are zero); complex operands; gradients.
# ---------------------------------------------------------------------------
SUBGROUP_CASES = [(4, 1, 1, 1), (6, 2, 1, 1), (8, 1, 2, 1), (12, 1, 1, 2), (6, 2, 2, 1),
                  (6, 1, 1, 0), (4, 0, 2, 1), (6, 2, 0, 1)]


@pytest.mark.parametrize("G,s,t,v", SUBGROUP_CASES)
def test_subgroup_contractions_vs_oracle(P, G, s, t, v):
    rng = np.random.default_rng(seed(("subgroup-gpu", G, s, t, v)))
    for trial in range(3):
        sub, su, sv = H.subgroup_case(rng, G, s, t, v, nmax=5)
        say(f"subgroup {sub} G={G} sectors {su.sectors} {sv.sectors}")
        Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
        ref, sw = O.contract_blocks(sub, Ru, su, Rv, sv)
        absref, _ = O.contract_blocks(sub, np.abs(Ru), su, np.abs(Rv), sv)
        u, v_ = _sym_tensor(P, Ru, su), _sym_tensor(P, Rv, sv)
        Gs, M, K, N = O.aligned_shape(sub, su, sv)
        info = P.plan(sub, u, v_)
        # a mode with fewer than |G| sectors takes the three-step path
        has_sub = any(h < G for x in (su, sv) if x.sectors for h in x.sectors)
        assert (info.m, info.k, info.n) == (M, K, N) and (info.fused == 0 or not has_sub)
        dead = H.dead_stored_tuples(sw)
        for compute in ("f64", "f32", "bf16x3"):
            w = P.output_like(sub, u, v_)
            assert w.sectors == sw.sectors
            w.data.fill_(7.0)
            P.contract_into(sub, u, v_, w, compute)
            got = H.to_np(w.data)
            assert np.all(np.abs(got - ref) <= H.bound_factor(compute, K) * absref + 1e-300), compute
            assert all(np.all(got[st] == 0) for st in dead), compute
            if compute == "f64":
                assert H.rel_err(got, ref) <= 1e-12 or np.max(np.abs(ref)) == 0
        if trial == 0:
            Ual, Val = O.align_u(sub, Ru, su, sv), O.align_v(sub, Rv, su, sv)
            for op, ref_al in ((0, Ual), (1, Val)):
                buf = torch.full(ref_al.shape, float("nan"), dtype=torch.float64, device=DEV)
                assert np.array_equal(H.to_np(P.align(sub, u, v_, op, "f64", out=buf)), ref_al), op
            Wal = np.matmul(Ual, Val)
            ref_w, _ = O.unalign_w(sub, Wal, su, sv)
            w = P.output_like(sub, u, v_)
            w.data.fill_(3.0)
            P.unalign(sub, u, v_, w, torch.from_numpy(Wal).to(DEV), "f64")
            assert np.array_equal(H.to_np(w.data), ref_w)
        if trial == 1:
            Cu = Ru + 1j * rng.standard_normal(su.reduced_shape())
            Cv = Rv + 1j * rng.standard_normal(sv.reduced_shape())
            cref, _ = O.contract_blocks(sub, Cu, su, Cv, sv)
            w = P.output_like(sub, _sym_tensor(P, Cu, su, torch.complex128), _sym_tensor(P, Cv, sv, torch.complex128))
            P.contract_into(sub, _sym_tensor(P, Cu, su, torch.complex128), _sym_tensor(P, Cv, sv, torch.complex128), w)
            assert H.rel_err(H.to_np(w.data), cref) <= 1e-12 or np.max(np.abs(cref)) == 0


@pytest.mark.parametrize("G,s,t,v", [(6, 1, 1, 1), (4, 2, 1, 1)])
def test_subgroup_gradients_vs_dense_autograd(P, G, s, t, v):
    rng = np.random.default_rng(seed(("subgroup-grad", G, s, t, v)))
    sub, su, sv = H.subgroup_case(rng, G, s, t, v, nmax=4)
    say(f"subgroup gradient {sub} G={G}")
    Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
    sw = O.output_symmetry(sub, su, sv)
    Rr = rng.standard_normal(sw.reduced_shape())
    ud = torch.from_numpy(Ru).to(DEV).requires_grad_(True)
    vd = torch.from_numpy(Rv).to(DEV).requires_grad_(True)
    w = P.einsum(sub, P.SymTensor(ud, su.sign_string(), su.charge, G, None, su.sectors),
                 P.SymTensor(vd, sv.sign_string(), sv.charge, G, None, sv.sectors))
    (w.data * torch.from_numpy(Rr).to(DEV)).sum().backward()
    du = torch.from_numpy(O.expand(Ru, su)).requires_grad_(True)
    dv = torch.from_numpy(O.expand(Rv, sv)).requires_grad_(True)
    (torch.einsum(sub, du, dv) * torch.from_numpy(O.expand(Rr, sw))).sum().backward()
    for got, dense, sym in ((ud.grad, du.grad, su), (vd.grad, dv.grad, sv)):
        ref, zero_ok = O.reduce_full(dense.numpy(), sym)
        assert zero_ok
        g = H.to_np(got)
        for st in H.dead_stored_tuples(sym):
            g[st] = 0.0          # entries without a block carry no gradient meaning
        assert H.rel_err(g, ref) <= 1e-12


@pytest.mark.parametrize("case", [FUSED_CASES[0], FUSED_CASES[2], FUSED_CASES[5], FUSED_CASES[6]])
@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_complex_fused_product_equals_steps_and_oracle(P, case, compute):
    """Complex operands on the fused product: A read as interleaved reals from U's
    standard form (K runs of 2 nK reals), C scattered into W's pairs."""
    sub, orders, cu, cv, du, dv = case
    rng = np.random.default_rng(len(sub) * 37 + sum(du))
    g = O.Group(orders)
    su = O.Sym.make(cu, int(rng.integers(g.size)), du, g)
    sv = O.Sym.make(cv, int(rng.integers(g.size)), dv, g)
    say(f"complex fused {sub} G={orders} {compute}")
    Ru, Rv = _cplx(rng, su.reduced_shape()), _cplx(rng, sv.reduced_shape())
    dt = torch.complex128 if compute == "f64" else torch.complex64
    u, v = _sym_tensor(P, Ru, su, dt), _sym_tensor(P, Rv, sv, dt)
    tu, rest = sub.split(",")
    nK = int(np.prod([d for m, d in zip(tu, du) if m in rest.split("->")[0]]))
    single = sum(m in rest.split("->")[0] for m in tu) == 1
    assert P.plan(sub, u, v, compute).fused == int((2 * nK) % (16 if compute == "f64" else 32) == 0 or single)
    w_f = P.output_like(sub, u, v, dtype=dt)
    w_s = P.output_like(sub, u, v, dtype=dt)
    P.contract_into(sub, u, v, w_f, compute)
    P.contract_into(sub, u, v, w_s, compute, steps=True)
    assert torch.equal(w_f.data, w_s.data)
    ref, sw = O.contract_blocks(sub, H.to_np(u.data).astype(np.complex128), su,
                                H.to_np(v.data).astype(np.complex128), sv)
    absref, _ = O.contract_blocks(sub, np.abs(Ru), su, np.abs(Rv), sv)
    k = 2 * H.contracted_extent(sub, su)
    got = H.to_np(w_f.data).astype(np.complex128)
    for part in (np.real, np.imag):
        assert np.all(np.abs(part(got) - part(ref)) <= H.bound_factor(compute, k) * absref + 1e-300)


@pytest.mark.parametrize("case", UA_CASES[:4])
@pytest.mark.parametrize("compute", ["f64", "f32"])
@pytest.mark.parametrize("tile", ["", "128x48", "d96x96s2"])
def test_complex_products_with_leading_contracted_modes(P, case, compute, tile, monkeypatch):
    """Complex operands whose contracted modes lead in U: A loaded K-major as
    interleaved reals on register tiles, or U aligned first on global-to-LDS
    tiles; W's pairs written in place.  Bit-identical to the three-step path and
    within the product's bound of the oracle."""
    sub, orders, cu, cv, du, dv = case
    if tile:
        monkeypatch.setenv("SYMT_GEMM_TILE", tile)
    else:
        monkeypatch.delenv("SYMT_GEMM_TILE", raising=False)
    monkeypatch.delenv("SYMT_GEMM_SK", raising=False)
    rng = np.random.default_rng(seed("complex-leading", sub, orders))
    g = O.Group(orders)
    su = O.Sym.make(cu, int(rng.integers(g.size)), du, g)
    sv = O.Sym.make(cv, int(rng.integers(g.size)), dv, g)
    say(f"complex leading {sub} G={orders} {compute} tile={tile or 'default'}")
    Ru, Rv = _cplx(rng, su.reduced_shape()), _cplx(rng, sv.reduced_shape())
    dt = torch.complex128 if compute == "f64" else torch.complex64
    u, v = _sym_tensor(P, Ru, su, dt), _sym_tensor(P, Rv, sv, dt)
    info = P.plan(sub, u, v, compute)
    assert info.fused_w == 1
    w_f = P.output_like(sub, u, v, dtype=dt)
    w_s = P.output_like(sub, u, v, dtype=dt)
    P.contract_into(sub, u, v, w_f, compute)
    P.contract_into(sub, u, v, w_s, compute, steps=True)
    assert torch.equal(w_f.data, w_s.data)
    ref, _ = O.contract_blocks(sub, H.to_np(u.data).astype(np.complex128), su,
                               H.to_np(v.data).astype(np.complex128), sv)
    absref, _ = O.contract_blocks(sub, np.abs(Ru), su, np.abs(Rv), sv)
    k = 2 * H.contracted_extent(sub, su)
    got = H.to_np(w_f.data).astype(np.complex128)
    for part in (np.real, np.imag):
        assert np.all(np.abs(part(got) - part(ref)) <= H.bound_factor(compute, k) * absref + 1e-300)


# ---------------------------------------------------------------------------
# Split K on the register tiles: few tiles and a long K (odd N rules out the
# global-to-LDS tiles), partial tiles summed in order by k_split_sum.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("compute", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(2, 40, 60000, 33), (3, 7, 20000, 5), (1, 130, 9000, 17)])
def test_sector_gemm_split_k(P, compute, shape):
    b, m, k, n = shape
    assert P.sector_gemm_workspace_size(compute, b, m, k, n) > 0
    say(f"split-K sector product {shape} {compute}")
    g = torch.Generator().manual_seed(b * m + k + n)
    dt = torch.float64 if compute == "f64" else torch.float32
    a = torch.rand(b, m, k, generator=g, dtype=torch.float64) * 2 - 1
    bb = torch.rand(b, k, n, generator=g, dtype=torch.float64) * 2 - 1
    ref = torch.bmm(a.to(dt).double(), bb.to(dt).double())
    absref = torch.bmm(a.to(dt).double().abs(), bb.to(dt).double().abs())
    c = P.sector_gemm(a.to(DEV, dt), bb.to(DEV, dt), compute)
    c2 = P.sector_gemm(a.to(DEV, dt), bb.to(DEV, dt), compute)
    assert torch.equal(c, c2)                      # the sum of the splits does not depend on scheduling
    err = (c.double().cpu() - ref).abs()
    assert torch.all(err <= H.bound_factor(compute, k) * absref + 1e-300)


def test_fused_split_k_contraction(P):
    """Fused product on register tiles (U misaligned by one element) with split K."""
    rng = np.random.default_rng(5)
    g = O.Group(3)
    su = O.Sym.make("+-", 1, (5, 4096), g)
    sv = O.Sym.make("++", 2, (4096, 8), g)
    sub = "ak,kb->ab"
    Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
    u = _sym_tensor(P, Ru, su)
    v = _sym_tensor(P, Rv, sv)
    buf = torch.zeros(u.data.numel() + 1, dtype=torch.float64, device=DEV)
    buf[1:] = u.data.reshape(-1)
    u_off = P.SymTensor(buf[1:].view(u.data.shape), u.signs, u.charge, u.group)
    assert P.plan(sub, u_off, v).fused == 1
    say("fused split-K contraction")
    w_f = P.output_like(sub, u, v)
    w_s = P.output_like(sub, u, v)
    P.contract_into(sub, u_off, v, w_f)
    P.contract_into(sub, u, v, w_s, steps=True)
    ref, sw = O.contract_blocks(sub, Ru, su, Rv, sv)
    absref, _ = O.contract_blocks(sub, np.abs(Ru), su, np.abs(Rv), sv)
    k = H.contracted_extent(sub, su)
    for w in (w_f, w_s):
        got = H.to_np(w.data)
        assert H.rel_err(got, ref) <= 1e-12
        assert np.all(np.abs(got - ref) <= H.bound_factor("f64", k) * absref + 1e-300)
