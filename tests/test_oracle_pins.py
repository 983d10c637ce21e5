"""Pins of the CPU oracle against things other than its own formulas (no GPU).

Each test ties the oracle to the paper's printed maps, a brute-force search, a
textbook identity, a library routine or a closed form.  The "planted mistake"
tests at the end show that plausible bugs in the oracle fail these pins.
"""
import itertools
import os

import numpy as np
import pytest

import oracle as O
import synth
from synth import philox
from tests.seeding import seed

RNG = np.random.default_rng(12345)


# ---------------------------------------------------------------------------
# Input generator
# ---------------------------------------------------------------------------
def test_philox_known_answers(golden_dir):
    rows = [ln.split() for ln in open(os.path.join(golden_dir, "philox4x32_10_kat.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        vals = [int(x, 16) for x in r]
        out = philox.philox4x32_10(*vals[:6])
        assert [int(o) for o in out] == vals[6:]


def test_uniform_values_exact_and_in_range():
    e = np.arange(0, 20000, dtype=np.int64)
    x = philox.values_at(e, 7, 3, philox.DIST_UNIFORM)
    assert x.min() >= -1.0 and x.max() < 1.0
    # exactness: recompute from the raw words with Python integers
    for i in (0, 1, 12345, 19999):
        w = philox.philox4x32_10(i & 0xFFFFFFFF, i >> 32, 0, 0, 7, 3)
        k = ((int(w[1]) << 32) | int(w[0])) >> 11
        assert x[i] == k / 2.0 ** 52 - 1.0
    assert abs(x.mean()) < 0.02 and abs(x.var() - 1.0 / 3.0) < 0.01


def test_normal_values_exact_moments():
    e = np.arange(0, 50000, dtype=np.int64)
    x = philox.values_at(e, 11, 5, philox.DIST_NORMAL)
    for i in (0, 7, 49999):
        s = 0
        for d in range(3):
            s += sum(int(v) for v in philox.philox4x32_10(i, 0, d, 0, 11, 5))
        assert x[i] == s / 2.0 ** 32 - 6.0
    assert abs(x.mean()) < 0.02 and abs(x.var() - 1.0) < 0.03
    y = philox.values_at(e[:100], 11, 5, philox.DIST_NORMAL, 1e-2)
    assert np.array_equal(y, x[:100] * np.float64(1e-2))


def test_host_generator_is_bit_identical_to_numpy():
    """The C twin (synth/csrc/philox_host.c) gives the NumPy generator's bits."""
    from synth import host
    if not host.available():
        pytest.skip("synth/libphilox_host.so is not built")
    e = np.concatenate([np.arange(0, 5000), RNG.integers(0, 2 ** 40, 5000)]).astype(np.int64)
    for dist in (philox.DIST_UNIFORM, philox.DIST_NORMAL):
        for scale in (1.0, 1e-2):
            assert np.array_equal(host.values_at(e, 20070805, 17, dist, scale),
                                  philox.values_at(e, 20070805, 17, dist, scale))
    got = host.fill((7, 11), 3, 4, philox.DIST_NORMAL, 1.0, first=1000)
    assert np.array_equal(got.ravel(), philox.values_at(np.arange(1000, 1077), 3, 4, philox.DIST_NORMAL))


# ---------------------------------------------------------------------------
# Group arithmetic
# ---------------------------------------------------------------------------
def test_cyclic_group_is_addition_mod_g():
    for G in (1, 2, 5, 8):
        g = O.Group(G)
        for a in range(G):
            for b in range(G):
                assert g.add(a, b) == (a + b) % G
                assert g.sub(a, b) == (a - b) % G
            assert g.neg(a) == (-a) % G


def test_z2xz3_isomorphic_to_z6_by_crt():
    g = O.Group((2, 3))
    phi = {e: (3 * g.digits(e)[0] + 4 * g.digits(e)[1]) % 6 for e in range(6)}
    assert sorted(phi.values()) == list(range(6))
    for a in range(6):
        for b in range(6):
            assert phi[g.add(a, b)] == (phi[a] + phi[b]) % 6
            assert phi[g.neg(a)] == (-phi[a]) % 6


def test_implicit_sector_is_the_unique_brute_force_solution():
    for orders in ((3,), (4,), (2, 3), (2, 2)):
        g = O.Group(orders)
        G = g.size
        for N in (1, 2, 3, 4):
            for _ in range(10):
                signs = tuple(int(s) for s in RNG.choice([-1, 1], N))
                Z = int(RNG.integers(G))
                sym = O.Sym(signs, Z, (1,) * N, g)
                for pos in range(N):
                    known = tuple(int(x) for x in RNG.integers(G, size=N - 1))
                    sols = []
                    for cand in range(G):
                        secs = list(known)
                        secs.insert(pos, cand)
                        # brute-force rule check, digit by digit
                        ok = all(sum(c * g.digits(s)[f] for c, s in zip(signs, secs)) % orders[f]
                                 == g.digits(Z)[f] for f in range(len(orders)))
                        if ok:
                            sols.append(cand)
                    assert sols == [O.implicit_sector(sym, known, position=pos)]


# ---------------------------------------------------------------------------
# The paper's worked example (Sec. 2.1) at G = 3
# ---------------------------------------------------------------------------
def _example_rows(golden_dir, kind):
    out = []
    for ln in open(os.path.join(golden_dir, "sec21_example_maps_z3.txt")):
        p = ln.split()
        if p and p[0] == kind:
            k = p.index("->")
            out.append(([int(x) for x in p[1:k]], [int(x) for x in p[k + 1:]]))
    return out


def test_example_maps_file_is_its_generators_output(golden_dir):
    """tests/golden/make_sec21_example_maps.py (the paper's printed maps, evaluated) wrote the file."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_maps", os.path.join(golden_dir, "make_sec21_example_maps.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(os.path.join(golden_dir, "sec21_example_maps_z3.txt")) as f:
        assert f.read() == mod.HEADER + "\n".join(mod.lines()) + "\n"


def test_standard_form_maps_of_the_example(golden_dir):
    g = O.Group(3)
    w = O.Sym.make("++--", 0, (1, 1, 1, 1), g)
    rows = _example_rows(golden_dir, "std")
    assert len(rows) == 27
    for (A, I, J), (B,) in rows:
        assert O.implicit_sector(w, (A, I, J), position=1) == B
    for (A, B, I, K), (J, L) in _example_rows(golden_dir, "alg1"):
        assert O.implicit_sector(w, (A, B, I)) == J        # w's last mode
        assert O.implicit_sector(w, (A, B, K)) == L        # u_abkl has the same rule


def test_aligned_form_maps_of_the_example(golden_dir):
    """Alignment deltas reproduce Sec. 2.1's maps with Q_alg = -Q_example (Q = sum c^U_K K)."""
    g = O.Group(3)
    su = O.Sym.make("++--", 0, (1, 1, 1, 1), g)
    sv = O.Sym.make("++--", 0, (1, 1, 1, 1), g)
    d1, d2, d3 = O.alignment_deltas("abkl,klij->abij", su, sv)
    rows = _example_rows(golden_dir, "aligned")
    assert len(rows) == 81
    for (Q, A, J, L), (B, I, K) in rows:
        q = (-Q) % 3
        assert d1[A, B, q] == 1 and d1[A].sum(axis=0)[q] == 1     # B = Q - A, unique
        assert d3[I, J, q] == 1 and d3[:, J, q].sum() == 1         # I = Q - J, unique
        assert d2[K, L, q] == 1 and d2[:, L, q].sum() == 1         # K = Q - L, unique


def test_footnote_rank3_reduced_form():
    """Sec. 2.1 footnote: r_{i,I,j,J,k} = t_{i,I,j,J,k,I+J} for I + J - K == 0."""
    G, n = 3, 2
    g = O.Group(G)
    sym = O.Sym.make("++-", 0, (n, n, n), g)
    T = np.zeros((G * n,) * 3)
    for I, J, K in itertools.product(range(G), repeat=3):
        if (I + J - K) % G == 0:
            T[I * n:(I + 1) * n, J * n:(J + 1) * n, K * n:(K + 1) * n] = RNG.standard_normal((n, n, n))
    R, zero_ok = O.reduce_full(T, sym)
    assert zero_ok
    for I, J in itertools.product(range(G), repeat=2):
        K = (I + J) % G
        assert np.array_equal(R[I, J], T[I * n:(I + 1) * n, J * n:(J + 1) * n, K * n:(K + 1) * n])
    assert np.array_equal(O.expand(R, sym), T)


# ---------------------------------------------------------------------------
# The five forms agree; brute force on tiny inputs
# ---------------------------------------------------------------------------
def _random_case(rng, orders, s, t, v, nmax=2, sigma=None):
    g = O.Group(orders)
    G = g.size
    letters = iter("abcdefghijklmnop")
    I = [next(letters) for _ in range(s)]
    K = [next(letters) for _ in range(v)]
    J = [next(letters) for _ in range(t)]
    tu = list(I + K)
    rng.shuffle(tu)
    tv = list(K + J)
    rng.shuffle(tv)
    tw = list(I + J)
    rng.shuffle(tw)
    dims = {m: int(rng.integers(1, nmax + 1)) for m in I + K + J}
    sign_u = {m: int(rng.choice([-1, 1])) for m in tu}
    sigma = int(rng.choice([-1, 1])) if sigma is None else sigma
    sign_v = {m: (sigma * sign_u[m] if m in K else int(rng.choice([-1, 1]))) for m in tv}
    su = O.Sym(tuple(sign_u[m] for m in tu), int(rng.integers(G)), tuple(dims[m] for m in tu), g)
    sv = O.Sym(tuple(sign_v[m] for m in tv), int(rng.integers(G)), tuple(dims[m] for m in tv), g)
    sub = f"{''.join(tu)},{''.join(tv)}->{''.join(tw)}"
    Ru = rng.standard_normal(su.reduced_shape())
    Rv = rng.standard_normal(sv.reduced_shape())
    return sub, Ru, su, Rv, sv


@pytest.mark.parametrize("orders", [(2,), (3,), (2, 2)])
@pytest.mark.parametrize("stv", [(1, 1, 1), (2, 1, 1), (1, 2, 1), (1, 1, 2), (2, 1, 2)])
def test_forms_agree_with_brute_force(orders, stv):
    rng = np.random.default_rng(seed((orders, stv)))
    s, t, v = stv
    for sigma in (-1, 1):
        sub, Ru, su, Rv, sv = _random_case(rng, orders, s, t, v, sigma=sigma)
        Rb, swb, zb = O.contract_bruteforce(sub, Ru, su, Rv, sv)
        assert zb, "brute-force output violates the derived conservation rule"
        Rd, swd, zd = O.contract_dense(sub, Ru, su, Rv, sv)
        Rk, swk = O.contract_blocks(sub, Ru, su, Rv, sv)
        Ra, swa, *_ = O.contract_irrep_aligned(sub, Ru, su, Rv, sv)
        assert zd
        for R in (Rd, Rk, Ra):
            np.testing.assert_allclose(R, Rb, rtol=1e-13, atol=1e-13)
        # every allowed block is generically nonzero: the derived rule is not too strict
        Wf = O.expand(Rb, swb)
        nz = 0
        for secs in itertools.product(range(su.group.size), repeat=swb.order):
            if O.allowed(swb, secs):
                sl = tuple(slice(S * n, (S + 1) * n) for S, n in zip(secs, swb.dims))
                nz += int(np.any(Wf[sl] != 0))
        assert nz == su.group.size ** (swb.order - 1)


def test_larger_random_contractions_dense_blocks_aligned():
    rng = np.random.default_rng(99)
    for orders, stv in (((4,), (2, 2, 2)), ((2, 3), (2, 2, 1)), ((5,), (1, 3, 2)), ((3,), (3, 1, 2))):
        sub, Ru, su, Rv, sv = _random_case(rng, orders, *stv, nmax=3)
        Rd, sw, zd = O.contract_dense(sub, Ru, su, Rv, sv)
        Rk, _ = O.contract_blocks(sub, Ru, su, Rv, sv)
        Ra, _, Ual, Val, Wal = O.contract_irrep_aligned(sub, Ru, su, Rv, sv)
        assert zd
        np.testing.assert_allclose(Rk, Rd, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(Ra, Rd, rtol=1e-12, atol=1e-12)
        G, M, Kd, N = O.aligned_shape(sub, su, sv)
        assert Ual.shape == (G, M, Kd) and Val.shape == (G, Kd, N) and Wal.shape == (G, M, N)
        # the alignment is a bijection of stored elements: same multiset of values
        assert np.array_equal(np.sort(Ual.ravel()), np.sort(np.asarray(Ru).ravel()))
        assert np.array_equal(np.sort(Val.ravel()), np.sort(np.asarray(Rv).ravel()))


def test_sampled_form_matches_dense():
    rng = np.random.default_rng(5)
    sub, Ru, su, Rv, sv = _random_case(rng, (4,), 2, 2, 2, nmax=3)
    Rd, sw, _ = O.contract_dense(sub, Ru, su, Rv, sv)
    Wf = O.expand(Rd, sw)
    pos = np.stack([rng.integers(0, d, 40) for d in Wf.shape], axis=1)
    got = O.sample_contract(sub, su, sv, O.reduced_value_fn(Ru, su), O.reduced_value_fn(Rv, sv), pos)
    np.testing.assert_allclose(got, Wf[tuple(pos.T)], rtol=1e-12, atol=1e-13)


def _all_full_positions(sw):
    return np.array(list(itertools.product(*[range(d) for d in sw.full_shape()])), dtype=np.int64)


@pytest.mark.parametrize("orders", [(2,), (3,), (2, 2)])
@pytest.mark.parametrize("stv", [(1, 1, 1), (2, 1, 1), (1, 2, 1), (1, 1, 2), (2, 1, 2), (1, 2, 2)])
def test_sampled_allowed_form_matches_brute_force_everywhere(orders, stv):
    """The allowed-sector sampled form equals Eq. ctr summed term by term at every output element."""
    rng = np.random.default_rng(seed(("allowed", orders, stv)))
    for sigma in (-1, 1):
        sub, Ru, su, Rv, sv = _random_case(rng, orders, *stv, sigma=sigma)
        Rb, sw, zb = O.contract_bruteforce(sub, Ru, su, Rv, sv)
        assert zb
        full = O.expand(Rb, sw)
        pos = _all_full_positions(sw)
        got = O.sample_contract_allowed(sub, su, sv, O.reduced_value_fn(Ru, su), O.reduced_value_fn(Rv, sv),
                                        pos, chunk=7)
        np.testing.assert_allclose(got, full[tuple(pos.T)], rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("sub", ["a,b->ab", "ab,cd->acbd", "k,kb->b", "lk,klb->b", "ak,k->a", "akl,lk->a"])
def test_sampled_allowed_form_degenerate_tables_subgroups_complex(sub):
    rng = np.random.default_rng(seed(("allowed-deg", sub)))
    g = O.Group((4,))
    tu, rest = sub.split(",")
    tv, tw = rest.split("->")
    for variant in ("tables", "subgroups", "complex"):
        dims = {m: int(rng.integers(1, 3)) for m in set(tu + tv)}
        cu = {m: int(rng.choice([-1, 1])) for m in tu}
        sigma = int(rng.choice([-1, 1]))
        cv = {m: (sigma * cu[m] if m in tu else int(rng.choice([-1, 1]))) for m in tv}
        tab = ({m: tuple(int(x) for x in rng.permutation(g.size)) for m in set(tu + tv)}
               if variant == "tables" else None)
        hs = {m: int(rng.choice([1, 2, 4])) for m in set(tu + tv)} if variant == "subgroups" else None
        su = O.Sym.make([cu[m] for m in tu], int(rng.integers(g.size)), [dims[m] for m in tu], g,
                        [tab[m] for m in tu] if tab else None, [hs[m] for m in tu] if hs else None)
        sv = O.Sym.make([cv[m] for m in tv], int(rng.integers(g.size)), [dims[m] for m in tv], g,
                        [tab[m] for m in tv] if tab else None, [hs[m] for m in tv] if hs else None)
        Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
        dt = np.float64
        if variant == "complex":
            Ru = Ru + 1j * rng.standard_normal(su.reduced_shape())
            Rv = Rv + 1j * rng.standard_normal(sv.reduced_shape())
            dt = np.complex128
        Rb, sw, zb = O.contract_bruteforce(sub, Ru, su, Rv, sv)
        assert zb
        full = O.expand(Rb, sw)
        pos = _all_full_positions(sw)
        got = O.sample_contract_allowed(sub, su, sv, O.reduced_value_fn(Ru, su), O.reduced_value_fn(Rv, sv),
                                        pos, dtype=dt)
        np.testing.assert_allclose(got, full[tuple(pos.T)], rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------------------
# Special cases that reduce to textbook or library routines
# ---------------------------------------------------------------------------
def test_trivial_group_is_plain_einsum():
    rng = np.random.default_rng(3)
    g = O.Group(1)
    su = O.Sym.make("+-+", 0, (3, 4, 5), g)
    sv = O.Sym.make("-+", 0, (5, 2), g)
    Ru = rng.standard_normal(su.reduced_shape())
    Rv = rng.standard_normal(sv.reduced_shape())
    sub = "abk,kj->ajb"
    ref = np.einsum(sub, Ru.reshape(3, 4, 5), Rv.reshape(5, 2))
    for R in (O.contract_dense(sub, Ru, su, Rv, sv)[0], O.contract_blocks(sub, Ru, su, Rv, sv)[0],
              O.contract_irrep_aligned(sub, Ru, su, Rv, sv)[0]):
        np.testing.assert_allclose(R.reshape(ref.shape), ref, rtol=1e-13, atol=1e-13)


def test_matrix_product_is_block_diagonal_gemm():
    import scipy.linalg
    rng = np.random.default_rng(4)
    G, n = 5, 3
    g = O.Group(G)
    su = O.Sym.make("+-", 0, (n, n), g)
    sv = O.Sym.make("+-", 0, (n, n), g)
    Ru = rng.standard_normal(su.reduced_shape())
    Rv = rng.standard_normal(sv.reduced_shape())
    ref = scipy.linalg.block_diag(*Ru) @ scipy.linalg.block_diag(*Rv)
    for R, sw in (O.contract_dense("ij,jk->ik", Ru, su, Rv, sv)[:2],
                  O.contract_blocks("ij,jk->ik", Ru, su, Rv, sv),
                  O.contract_irrep_aligned("ij,jk->ik", Ru, su, Rv, sv)[:2]):
        np.testing.assert_allclose(O.expand(R, sw), ref, rtol=1e-13, atol=1e-13)


def test_product_group_equals_z6_after_crt_relabelling():
    rng = np.random.default_rng(6)
    g23, g6 = O.Group((2, 3)), O.Group(6)
    phi = np.array([(3 * g23.digits(e)[0] + 4 * g23.digits(e)[1]) % 6 for e in range(6)])
    sub = "abc,asA->bcsA"
    su = O.Sym.make("---", 2, (2, 1, 2), g23)
    sv = O.Sym.make("++-", 5, (2, 1, 2), g23)
    Ru = rng.standard_normal(su.reduced_shape())
    Rv = rng.standard_normal(sv.reduced_shape())

    def relabel(R, order):
        out = np.empty_like(R)
        for secs in itertools.product(range(6), repeat=order - 1):
            out[tuple(phi[list(secs)])] = R[secs]
        return out

    su6 = O.Sym(su.signs, int(phi[su.charge]), su.dims, g6)
    sv6 = O.Sym(sv.signs, int(phi[sv.charge]), sv.dims, g6)
    W23, sw23 = O.contract_blocks(sub, Ru, su, Rv, sv)
    W6, sw6 = O.contract_blocks(sub, relabel(Ru, 3), su6, relabel(Rv, 3), sv6)
    assert sw6.charge == phi[sw23.charge]
    np.testing.assert_allclose(W6, relabel(W23, 4), rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------------------
# Costs (paper Sec. 2.1, Alg. 2's product step, Table 1)
# ---------------------------------------------------------------------------
def test_flop_counts_closed_forms():
    for G, n in ((4, 4), (8, 3), (3, 5)):
        g = O.Group(G)
        s4 = O.Sym.make("++--", 0, (n,) * 4, g)
        assert O.flop_count("abkl,klij->abij", s4, s4) == 2 * n ** 6 * G ** 4     # Sec. 2.1
        s2 = O.Sym.make("+-", 0, (n, n), g)
        assert O.flop_count("ij,jk->ik", s2, s2) == 2 * G * n ** 3                 # Table 1, MM
        s3 = O.Sym.make("++-", 0, (n, n, n), g)
        s3v = O.Sym.make("+--", 0, (n, n, n), g)
        assert O.flop_count("ijk,klm->ijlm", s3, s3v) == 2 * G ** 3 * n ** 5       # Table 1, MPS
    # plain_z4 workload: 2 n^6 G^4 = 2 097 152
    s = O.Sym.make("++--", 0, (4,) * 4, O.Group(4))
    assert O.flop_count("abkl,klij->abij", s, s) == 2_097_152


def test_flop_count_equals_brute_force_count_of_nonzero_terms():
    rng = np.random.default_rng(8)
    for orders, stv in (((3,), (1, 1, 1)), ((2,), (2, 1, 2)), ((2, 2), (1, 2, 1)), ((3,), (2, 2, 1))):
        sub, Ru, su, Rv, sv = _random_case(rng, orders, *stv)
        tu, tv, tw, I, K, J = O.parse_einsum(sub)
        size = {}
        for t, sym in ((tu, su), (tv, sv)):
            for p, m in enumerate(t):
                size[m] = sym.group.size * sym.dims[p]
        count = 0
        for wi in itertools.product(*[range(size[m]) for m in tw]):
            idx = dict(zip(tw, wi))
            for ki in itertools.product(*[range(size[m]) for m in K]):
                idx.update(zip(K, ki))
                cu = tuple(idx[m] // su.dims[p] for p, m in enumerate(tu))
                cv = tuple(idx[m] // sv.dims[p] for p, m in enumerate(tv))
                count += O.allowed(su, cu) and O.allowed(sv, cv)
        assert 2 * count == O.flop_count(sub, su, sv)


# ---------------------------------------------------------------------------
# Workload definitions are consistent with the derived output rule
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(synth.configs.ALL))
def test_workload_output_signs_are_the_derived_ones(name):
    wl = synth.configs.get(name)
    g = O.Group(wl.group)
    for st in wl.steps:
        ou, ov, ow = (wl.operands[x] for x in (st.u, st.v, st.w))
        su = O.Sym.make(ou.signs, ou.charge, ou.dims, g, sectors=ou.sectors)
        sv = O.Sym.make(ov.signs, ov.charge, ov.dims, g, sectors=ov.sectors)
        sw = O.Sym.make(ow.signs, ow.charge, ow.dims, g, sectors=ow.sectors)
        assert O.same_symmetry(O.output_symmetry(st.einsum, su, sv), sw)


# ---------------------------------------------------------------------------
# bfloat16 rounding against the library conversion
# ---------------------------------------------------------------------------
def test_bf16_round_matches_torch():
    import torch
    x = np.concatenate([RNG.standard_normal(20000), RNG.standard_normal(2000) * 1e-30,
                        RNG.standard_normal(2000) * 1e30]).astype(np.float32)
    # ties: values exactly half-way between two bf16 numbers
    ties = (np.arange(1, 2000, dtype=np.uint32) << 16 | np.uint32(0x8000)).view(np.float32)
    x = np.concatenate([x, ties, -ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(O.bf16_round(x), ref)
    hi, lo = O.bf16_split(x[:20000])
    assert np.array_equal(O.bf16_round(hi), hi) and np.array_equal(O.bf16_round(lo), lo)
    err = np.abs(x[:20000].astype(np.float64) - hi - lo) / np.abs(x[:20000])
    assert err.max() <= 2.0 ** -16


# ---------------------------------------------------------------------------
# Planted mistakes: each must make at least one pin fail
# ---------------------------------------------------------------------------
def _pins_pass(monkeypatch_ctx=None):
    rng = np.random.default_rng(77)
    try:
        for orders, stv in (((3,), (1, 1, 1)), ((2, 2), (2, 1, 1)), ((3,), (1, 2, 2))):
            for sigma in (-1, 1):
                sub, Ru, su, Rv, sv = _random_case(rng, orders, *stv, sigma=sigma)
                Rb, _, zb = O.contract_bruteforce(sub, Ru, su, Rv, sv)
                Rd, _, zd = O.contract_dense(sub, Ru, su, Rv, sv)
                Rk, _ = O.contract_blocks(sub, Ru, su, Rv, sv)
                Ra, *_ = O.contract_irrep_aligned(sub, Ru, su, Rv, sv)
                if not (zb and zd):
                    return False
                for R in (Rd, Rk, Ra):
                    if not np.allclose(R, Rb, rtol=1e-12, atol=1e-12):
                        return False
                sw = O.output_symmetry(sub, su, sv)
                pos = _all_full_positions(sw)
                got = O.sample_contract_allowed(sub, su, sv, O.reduced_value_fn(Ru, su),
                                                O.reduced_value_fn(Rv, sv), pos)
                if not np.allclose(got, O.expand(Rb, sw)[tuple(pos.T)], rtol=1e-12, atol=1e-12):
                    return False
    except (AssertionError, ValueError, IndexError):
        return False
    return True


def test_pins_pass_unmodified():
    assert _pins_pass()


def test_planted_sign_error_in_output_rule_is_caught(monkeypatch):
    import oracle.symcontract as S
    real = S.output_symmetry

    def wrong(sub, su, sv):
        w = real(sub, su, sv)
        return S.Sym(w.signs, w.group.add(w.charge, 1), w.dims, w.group)   # Z^U + sigma Z^V + 1
    monkeypatch.setattr(S, "output_symmetry", wrong)
    assert not _pins_pass()


def test_planted_dropped_coefficient_in_implicit_sector_is_caught(monkeypatch):
    import oracle.symcontract as S

    def wrong(sym, known, position=None):
        g = sym.group
        p = sym.order - 1 if position is None else position
        others = [c for m, c in enumerate(sym.signs) if m != p]
        return g.sub(sym.charge, g.total(others, known))      # forgets to multiply by c_p
    monkeypatch.setattr(S, "implicit_sector", wrong)
    assert not _pins_pass()


def test_planted_wrong_q_sign_in_delta3_is_caught(monkeypatch):
    import oracle.symcontract as S
    real = S.alignment_deltas

    def wrong(sub, su, sv):
        d1, d2, d3 = real(sub, su, sv)
        tu, tv, tw, I, K, J = S.parse_einsum(sub)
        d3w = S.kron_delta(su.group, [sv.signs[tv.index(m)] for m in J], +1, sv.charge)  # ignores sigma
        return d1, d2, d3w
    monkeypatch.setattr(S, "alignment_deltas", wrong)
    assert not _pins_pass()


def test_planted_transposed_block_product_is_caught(monkeypatch):
    import oracle.symcontract as S
    real_einsum = np.einsum

    def wrong(*args, **kw):
        out = real_einsum(*args, **kw)
        if isinstance(args[0], str) and "->" in args[0] and out.ndim >= 2 and out.shape[0] == out.shape[1]:
            out = np.swapaxes(out, 0, 1)
        return out
    monkeypatch.setattr(S.np, "einsum", wrong)
    assert not _pins_pass()


# ---------------------------------------------------------------------------
# Charge tables: sector label L of mode m carries charge chi_m(L).  A tensor
# with tables is the identity-table tensor with each mode's sector blocks
# permuted, so every form must commute with relabelling.
# ---------------------------------------------------------------------------
def _random_tables(rng, order, G):
    return tuple(tuple(int(x) for x in rng.permutation(G)) for _ in range(order))


def _relabel_reduced(R, sym):
    """Identity-table reduced form of the same tensor: stored axes indexed by charge."""
    inv = [np.argsort(np.asarray(sym.table(m))) for m in range(sym.order - 1)]
    return np.asarray(R)[np.ix_(*inv)] if inv else np.asarray(R)


def _relabel_full(T, sym):
    """Full tensor with each mode's sector blocks moved from label to charge position."""
    out = np.asarray(T)
    for m in range(sym.order):
        n = sym.dims[m]
        perm = np.empty(sym.group.size * n, dtype=np.int64)
        for L in range(sym.group.size):
            c = sym.table(m)[L]
            perm[c * n:(c + 1) * n] = np.arange(L * n, (L + 1) * n)
        out = np.take(out, perm, axis=m)
    return out


def _plain(sym):
    return O.Sym(sym.signs, sym.charge, sym.dims, sym.group)


@pytest.mark.parametrize("orders", [(3,), (4,), (2, 3), (5,)])
def test_charge_tables_expand_is_a_relabelling(orders):
    rng = np.random.default_rng(sum(orders) * 13)
    g = O.Group(orders)
    for order in (1, 2, 3, 4):
        sym = O.Sym.make(tuple(rng.choice([-1, 1], order)), int(rng.integers(g.size)),
                         tuple(int(d) for d in rng.integers(1, 3, order)), g,
                         _random_tables(rng, order, g.size))
        R = rng.standard_normal(sym.reduced_shape())
        full = O.expand(R, sym)
        ref = O.expand(_relabel_reduced(R, sym), _plain(sym))
        assert np.array_equal(_relabel_full(full, sym), ref)
        back, zero_ok = O.reduce_full(full, sym)
        assert zero_ok and np.array_equal(back, R)


@pytest.mark.parametrize("orders,s,t,v", [((3,), 1, 1, 1), ((4,), 2, 1, 1), ((2, 3), 1, 2, 1), ((3,), 2, 2, 2)])
def test_charge_tables_contraction_commutes_with_relabelling(orders, s, t, v):
    rng = np.random.default_rng(s * 100 + t * 10 + v + len(orders))
    g = O.Group(orders)
    for sigma in (-1, 1):
        sub, _, su0, _, sv0 = _random_case(rng, orders, s, t, v, sigma=sigma)
        tu, rest = sub.split(",")
        tv, tw = rest.split("->")
        # shared tables on the contracted modes, independent ones elsewhere
        tab = {m: tuple(int(x) for x in rng.permutation(g.size)) for m in set(tu) | set(tv)}
        su = O.Sym.make(su0.signs, su0.charge, su0.dims, g, [tab[m] for m in tu])
        sv = O.Sym.make(sv0.signs, sv0.charge, sv0.dims, g, [tab[m] for m in tv])
        Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
        sw = O.output_symmetry(sub, su, sv)
        assert all(sw.table(p) == tab[m] for p, m in enumerate(tw))
        blocks, _ = O.contract_blocks(sub, Ru, su, Rv, sv)
        dense, _, zero_ok = O.contract_dense(sub, Ru, su, Rv, sv)
        aligned = O.contract_irrep_aligned(sub, Ru, su, Rv, sv)[0]
        assert zero_ok
        assert np.allclose(blocks, dense, rtol=1e-12, atol=1e-12)
        assert np.allclose(aligned, dense, rtol=1e-12, atol=1e-12)
        # relabelled operands through the identity-table path give the relabelled output
        ref, swp = O.contract_blocks(sub, _relabel_reduced(Ru, su), _plain(su), _relabel_reduced(Rv, sv), _plain(sv))
        assert np.allclose(_relabel_reduced(blocks, sw), ref, rtol=1e-12, atol=1e-12)


def test_charge_tables_bruteforce_tiny():
    rng = np.random.default_rng(77)
    g = O.Group((3,))
    tab = {m: tuple(int(x) for x in rng.permutation(3)) for m in "abk"}
    su = O.Sym.make((1, -1), 1, (2, 1), g, [tab["a"], tab["k"]])
    sv = O.Sym.make((1, 1), 2, (1, 2), g, [tab["k"], tab["b"]])
    Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
    brute, sw, zero_ok = O.contract_bruteforce("ak,kb->ab", Ru, su, Rv, sv)
    blocks, _ = O.contract_blocks("ak,kb->ab", Ru, su, Rv, sv)
    assert zero_ok and np.allclose(brute, blocks, rtol=1e-13, atol=1e-13)


def test_charge_tables_mismatch_on_contracted_mode_is_rejected():
    g = O.Group((3,))
    su = O.Sym.make((1, -1), 0, (2, 2), g, [(0, 1, 2), (1, 2, 0)])
    sv = O.Sym.make((1, -1), 0, (2, 2), g, [(0, 1, 2), (0, 1, 2)])
    with pytest.raises(ValueError):
        O.contract_blocks("ak,kb->ab", np.zeros(su.reduced_shape()), su, np.zeros(sv.reduced_shape()), sv)


def test_planted_mistake_tables_ignored_in_implicit_sector(monkeypatch):
    """Solving the implicit sector as if labels were charges must break the relabelling pin."""
    rng = np.random.default_rng(5)
    g = O.Group((4,))
    sym = O.Sym.make((1, -1, 1), 1, (1, 2, 1), g, _random_tables(rng, 3, 4))
    R = rng.standard_normal(sym.reduced_shape())
    good = O.expand(R, sym)

    def wrong(sym_, known, position=None):
        gg = sym_.group
        p = sym_.order - 1 if position is None else position
        others = [c for m, c in enumerate(sym_.signs) if m != p]
        return gg.times(sym_.signs[p], gg.sub(sym_.charge, gg.total(others, known)))
    monkeypatch.setattr(O.symcontract, "implicit_sector", wrong)
    bad = O.expand(R, sym)
    assert not np.array_equal(bad, good)
    assert not np.array_equal(_relabel_full(bad, sym), O.expand(_relabel_reduced(R, sym), _plain(sym)))


# ---------------------------------------------------------------------------
# s, t or v = 0: one delta pins Q to a single value (the case noted after Alg. 2)
# ---------------------------------------------------------------------------
DEGENERATE = ["a,b->ab", "ab,c->abc", "ab,cd->acbd",        # v = 0: outer products
              "k,kb->b", "kl,klij->ij", "lk,klb->b",         # s = 0
              "ak,k->a", "abk,k->ab", "akl,lk->a"]           # t = 0


@pytest.mark.parametrize("sub", DEGENERATE)
@pytest.mark.parametrize("orders", [(3,), (2, 2)])
def test_degenerate_contractions_all_forms_agree(sub, orders):
    rng = np.random.default_rng(seed((sub, orders)))
    g = O.Group(orders)
    tu, rest = sub.split(",")
    tv, tw = rest.split("->")
    for with_tables in (False, True):
        dims = {m: int(rng.integers(1, 3)) for m in set(tu + tv)}
        cu = {m: int(rng.choice([-1, 1])) for m in tu}
        sigma = int(rng.choice([-1, 1]))
        cv = {m: (sigma * cu[m] if m in tu else int(rng.choice([-1, 1]))) for m in tv}
        tab = {m: tuple(int(x) for x in rng.permutation(g.size)) for m in set(tu + tv)} if with_tables else None
        su = O.Sym.make([cu[m] for m in tu], int(rng.integers(g.size)), [dims[m] for m in tu], g,
                        [tab[m] for m in tu] if tab else None)
        sv = O.Sym.make([cv[m] for m in tv], int(rng.integers(g.size)), [dims[m] for m in tv], g,
                        [tab[m] for m in tv] if tab else None)
        Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
        brute, sw, zero_ok = O.contract_bruteforce(sub, Ru, su, Rv, sv)
        assert zero_ok
        blocks, sw2 = O.contract_blocks(sub, Ru, su, Rv, sv)
        dense, _, _ = O.contract_dense(sub, Ru, su, Rv, sv)
        aligned = O.contract_irrep_aligned(sub, Ru, su, Rv, sv)[0]
        assert sw2 == sw
        for got in (blocks, dense, aligned):
            assert np.allclose(got, brute, rtol=1e-13, atol=1e-13)
        # allowed-block products: closed form vs a count of nonzero terms
        G = g.size
        nz = 0
        for us in itertools.product(range(G), repeat=su.order):
            if not O.allowed(su, us):
                continue
            sec = dict(zip(tu, us))
            for vs in itertools.product(range(G), repeat=sv.order):
                if all(sec.get(m, x) == x for m, x in zip(tv, vs)) and O.allowed(sv, vs):
                    nz += 1
        n = int(np.prod([dims[m] for m in set(tu + tv)]))
        assert O.flop_count(sub, su, sv) == 2 * n * nz


def test_degenerate_output_of_order_zero_is_rejected():
    g = O.Group((3,))
    su = O.Sym.make("+-", 0, (2, 2), g)
    sv = O.Sym.make("-+", 0, (2, 2), g)
    with pytest.raises(ValueError):
        O.contract_blocks("kl,kl->", np.zeros(su.reduced_shape()), su, np.zeros(sv.reduced_shape()), sv)


# ---------------------------------------------------------------------------
# U(1) emulated by a cyclic group (Sec. 3): dense U(1) tensors with integer
# charge conservation, embedded in Z_G by per-mode charge tables, contract to
# the embedding of the dense U(1) einsum; wrapped-around blocks stay zero.
# ---------------------------------------------------------------------------
U1_SUBS = ["ij,jk->ik", "ijk,klm->ijlm", "abcd,cdij->abij", "ak,k->a", "a,b->ab", "bk,ka->ab"]


@pytest.mark.parametrize("sub", U1_SUBS)
@pytest.mark.parametrize("g_extra", [0, 3])
def test_u1_emulation_matches_dense_u1_einsum(sub, g_extra):
    from tests import u1_cases as U1
    rng = np.random.default_rng(seed(("u1", sub, g_extra)))
    for _ in range(3):
        c = U1.random_case(rng, sub, g_extra)
        for form in (O.contract_blocks, O.contract_irrep_aligned, O.contract_dense):
            Rw, sw = form(sub, c["Ru"], c["su"], c["Rv"], c["sv"])[:2]
            phys, rest = U1.physical_part(O.expand(Rw, sw), c["Pw"], c["nw"])
            assert rest == 0.0, form.__name__
            np.testing.assert_allclose(phys, c["ref"], rtol=0, atol=1e-12 * max(1.0, np.abs(c["ref"]).max()))


def test_u1_emulation_needs_one_label_per_charge():
    # with G below a mode's number of charges two charges share a label: not representable
    from tests import u1_cases as U1
    rng = np.random.default_rng(7)
    T = U1.dense_u1(rng, [1, -1], 0, [0, 0], [3, 3], [1, 1])
    with pytest.raises(Exception):
        U1.embed(T, [1, -1], 0, [0, 0], [3, 3], [1, 1], 2)


# ---------------------------------------------------------------------------
# Complex tensors (Sec. 2.2 defines tensors over R or C).  Pins: the complex
# contraction is the bilinear combination of four real ones (checked against
# the real forms pinned above), np.einsum on the expanded complex operands
# agrees, and Alg. 2 with dense deltas agrees.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("orders,s,t,v", [((3,), 1, 1, 1), ((4,), 2, 1, 2), ((2, 3), 1, 2, 1), ((5,), 2, 2, 1),
                                          ((4,), 1, 1, 0), ((3,), 0, 2, 1)])
def test_complex_contraction_is_four_real_ones(orders, s, t, v):
    rng = np.random.default_rng(seed(("complex", orders, s, t, v)))
    for _ in range(2):
        sub, _, su, _, sv = _random_case(rng, orders, s, t, v, nmax=3)
        Ur, Ui = rng.standard_normal(su.reduced_shape()), rng.standard_normal(su.reduced_shape())
        Vr, Vi = rng.standard_normal(sv.reduced_shape()), rng.standard_normal(sv.reduced_shape())
        real = lambda a, b: O.contract_blocks(sub, a, su, b, sv)[0]  # noqa: E731
        ref = (real(Ur, Vr) - real(Ui, Vi)) + 1j * (real(Ur, Vi) + real(Ui, Vr))
        U, V = Ur + 1j * Ui, Vr + 1j * Vi
        scale = max(1.0, np.abs(ref).max())
        for form in (O.contract_blocks, O.contract_dense, O.contract_irrep_aligned):
            Rw, sw = form(sub, U, su, V, sv)[:2]
            assert np.iscomplexobj(Rw)
            np.testing.assert_allclose(Rw, ref, rtol=0, atol=1e-12 * scale)
        Wd = np.einsum(sub, O.expand(U, su), O.expand(V, sv))
        np.testing.assert_allclose(O.expand(ref, O.output_symmetry(sub, su, sv)), Wd, rtol=0, atol=1e-12 * scale)


def test_complex_bruteforce_and_samples_tiny():
    rng = np.random.default_rng(31)
    sub, _, su, _, sv = _random_case(rng, (3,), 1, 1, 1, nmax=2)
    U = rng.standard_normal(su.reduced_shape()) + 1j * rng.standard_normal(su.reduced_shape())
    V = rng.standard_normal(sv.reduced_shape()) + 1j * rng.standard_normal(sv.reduced_shape())
    Rb, sw, ok = O.contract_bruteforce(sub, U, su, V, sv)
    assert ok
    np.testing.assert_allclose(Rb, O.contract_blocks(sub, U, su, V, sv)[0], rtol=0, atol=1e-12)
    full = O.expand(Rb, sw)
    pos = np.array(list(itertools.product(*[range(d) for d in full.shape]))[:20])
    got = O.sample_contract(sub, su, sv, O.reduced_value_fn(U, su), O.reduced_value_fn(V, sv), pos,
                            dtype=np.complex128)
    np.testing.assert_allclose(got, full[tuple(pos.T)], rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# Subgroup modes (Sec. 2.2, Eq. symtsr with c_i = +-G/H_i): mode i has H_i | G
# sectors.  Pins: with one H for every mode the tensor is a Z_H tensor with
# charge Z / (G/H) (the pinned Z_H oracle); mixed H_i against brute force over
# full indices (Eq. ctr summed term by term) and np.einsum on the expanded
# operands; the zero pattern of the output; flops against a count of terms.
# ---------------------------------------------------------------------------
def _divisors(G):
    return [h for h in range(1, G + 1) if G % h == 0]


def _subgroup_case(rng, G, s, t, v, nmax=2, uniform_h=None):
    g = O.Group(G)
    letters = iter("abcdefghijklmnop")
    I = [next(letters) for _ in range(s)]
    K = [next(letters) for _ in range(v)]
    J = [next(letters) for _ in range(t)]
    tu = list(I + K); rng.shuffle(tu)
    tv = list(K + J); rng.shuffle(tv)
    tw = list(I + J); rng.shuffle(tw)
    hs = {m: (uniform_h or int(rng.choice(_divisors(G)))) for m in I + K + J}
    dims = {m: int(rng.integers(1, nmax + 1)) for m in I + K + J}
    cu = {m: int(rng.choice([-1, 1])) for m in tu}
    sigma = int(rng.choice([-1, 1]))
    cv = {m: (sigma * cu[m] if m in K else int(rng.choice([-1, 1]))) for m in tv}

    def reach(term, c):
        # a total charge that some sector combination reaches
        return sum(c[m] * (G // hs[m]) * int(rng.integers(hs[m])) for m in term) % G
    su = O.Sym.make([cu[m] for m in tu], reach(tu, cu), [dims[m] for m in tu], g, sectors=[hs[m] for m in tu])
    sv = O.Sym.make([cv[m] for m in tv], reach(tv, cv), [dims[m] for m in tv], g, sectors=[hs[m] for m in tv])
    return f"{''.join(tu)},{''.join(tv)}->{''.join(tw)}", su, sv


@pytest.mark.parametrize("G,H", [(4, 2), (6, 3), (6, 2), (8, 4), (12, 6)])
@pytest.mark.parametrize("stv", [(1, 1, 1), (2, 1, 1), (1, 2, 2)])
def test_uniform_subgroup_is_the_smaller_cyclic_group(G, H, stv):
    rng = np.random.default_rng(seed(("subgroup-uniform", G, H, stv)))
    sub, su, sv = _subgroup_case(rng, G, *stv, uniform_h=H)
    d = G // H
    assert su.charge % d == 0 and sv.charge % d == 0
    small = lambda sym: O.Sym.make(sym.signs, sym.charge // d, sym.dims, O.Group(H))  # noqa: E731
    Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
    assert su.reduced_shape() == small(su).reduced_shape()
    Rw, sw = O.contract_blocks(sub, Ru, su, Rv, sv)
    Rh, swh = O.contract_blocks(sub, Ru, small(su), Rv, small(sv))
    np.testing.assert_allclose(Rw, Rh, rtol=0, atol=1e-12)
    assert sw.charge == swh.charge * d and sw.signs == swh.signs
    Ra = O.contract_irrep_aligned(sub, Ru, su, Rv, sv)[0]
    np.testing.assert_allclose(Ra, Rh, rtol=0, atol=1e-12)


@pytest.mark.parametrize("G", [4, 6, 8])
@pytest.mark.parametrize("stv", [(1, 1, 1), (2, 1, 1), (1, 1, 2), (1, 2, 1), (1, 1, 0), (0, 2, 1)])
def test_mixed_subgroups_all_forms_agree_with_brute_force(G, stv):
    rng = np.random.default_rng(seed(("subgroup-mixed", G, stv)))
    for _ in range(3):
        sub, su, sv = _subgroup_case(rng, G, *stv)
        Ru, Rv = rng.standard_normal(su.reduced_shape()), rng.standard_normal(sv.reduced_shape())
        Rb, sw, zero_ok = O.contract_bruteforce(sub, Ru, su, Rv, sv)
        assert zero_ok
        Wd = np.einsum(sub, O.expand(Ru, su), O.expand(Rv, sv))
        np.testing.assert_allclose(O.expand(Rb, sw), Wd, rtol=0, atol=1e-12)
        for form in (O.contract_dense, O.contract_blocks, O.contract_irrep_aligned):
            R, swf = form(sub, Ru, su, Rv, sv)[:2]
            assert O.same_symmetry(swf, sw)
            np.testing.assert_allclose(O.expand(R, sw), O.expand(Rb, sw), rtol=0, atol=1e-12)
        # flops: 2 x the number of nonzero scalar terms of Eq. ctr
        U, V = O.expand(np.ones(su.reduced_shape()), su), O.expand(np.ones(sv.reduced_shape()), sv)
        assert O.flop_count(sub, su, sv) == 2 * int(round(np.einsum(sub, U, V).sum()))


def test_subgroup_dead_blocks_and_rules():
    # Z_4 with a Z_2 mode (c = 2): a + 2b == 1 has solutions only for odd a
    su = O.Sym.make("++", 1, (1, 1), O.Group(4), sectors=(4, 2))
    assert O.implicit_sector(su, (0,)) is None and O.implicit_sector(su, (2,)) is None
    assert O.implicit_sector(su, (1,)) == 0 and O.implicit_sector(su, (3,)) == 1
    R = np.arange(4.0).reshape(4, 1, 1) + 1
    full = O.expand(R, su)
    assert full.shape == (4, 2) and full[0].sum() == 0 and full[2].sum() == 0
    assert full[1, 0] == 2 and full[3, 1] == 4
    with pytest.raises(ValueError):
        O.Sym.make("++", 0, (1, 1), O.Group(4), sectors=(4, 3))
    with pytest.raises(ValueError):
        O.Sym.make("++", 0, (1, 1), O.Group((2, 2)), sectors=(4, 2))
