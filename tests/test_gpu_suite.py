"""The paper's benchmark suite (Table 1 contractions at Table 2 dimensions) on the GPU.

Small copies (every block dimension shrunk, the group kept) are compared with
the loop-over-blocks oracle in three precisions; the full Table 2 sizes are
contracted in f64, f32 and split-bf16 and checked on sampled outputs against
the oracle's allowed-sector sampled form.  These cases exercise operands whose contracted modes lead
(CC2, CC3), a single contracted mode (MPS), |G| up to 100 (MM_b), and very
tall products (PEPS_a: M = 320000).
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

SMALL = {
    "cc": dict(i=4, j=3, k=5, l=2, m=3, n=2, o=2, p=3),
    "mm": dict(i=7, j=5, k=6),
    "mps": dict(i=5, j=3, k=6, l=1, m=4),
    "peps": dict(i=5, j=4, k=3, l=2, m=3, n=2),
}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    import paper_2007_08056_amd
    return paper_2007_08056_amd


@pytest.fixture(scope="module")
def SG():
    import synth.gpu
    return synth.gpu


def _small(label):
    fam = "".join(ch for ch in label if ch.isalpha())[:-1]
    return synth.configs.paper_suite_case(label, SMALL[fam])


def _sym(wl, name):
    op = wl.operands[name]
    return O.Sym.make(op.signs, op.charge, op.dims, O.Group(wl.group))


def _tensor(P, SG, wl, name, dtype=torch.float64):
    op = wl.operands[name]
    return P.SymTensor(SG.device_input(wl, name, dtype=dtype, device=DEV), op.signs, op.charge, wl.group)


@pytest.mark.parametrize("label", synth.configs.SUITE_LABELS)
def test_suite_small_vs_oracle(P, SG, label):
    wl = _small(label)
    st = wl.steps[0]
    su, sv = _sym(wl, "U"), _sym(wl, "V")
    Ru, Rv = synth.host_input(wl, "U"), synth.host_input(wl, "V")
    ref, sw = O.contract_blocks(st.einsum, Ru, su, Rv, sv)
    absref, _ = O.contract_blocks(st.einsum, np.abs(Ru), su, np.abs(Rv), sv)
    assert sw.sign_string() == wl.operands["W"].signs or \
        sw.sign_string() == "".join("+" if c == "-" else "-" for c in wl.operands["W"].signs)
    k = H.contracted_extent(st.einsum, su)
    for compute in ("f64", "f32", "bf16x3"):
        dt = torch.float64 if compute == "f64" else torch.float32
        u, v = _tensor(P, SG, wl, "U", dt), _tensor(P, SG, wl, "V", dt)
        info = P.plan(st.einsum, u, v, compute)
        say(f"suite {label} small {compute}: batch {info.group_size} m {info.m} k {info.k} n {info.n}")
        w = P.output_like(st.einsum, u, v, dtype=torch.float64)
        P.contract_into(st.einsum, u, v, w, compute)
        got = H.to_np(w.data)
        if compute == "f64":
            assert H.rel_err(got, ref) <= 1e-12
            assert np.all(np.abs(got - ref) <= H.bound_factor("f64", k) * absref + 1e-300)
            assert np.array_equal(O.expand(got, sw) == 0, O.expand(ref, sw) == 0)
        else:
            # against the binary64 inputs: adds the input rounding
            assert np.all(np.abs(got - ref) <= (H.bound_factor(compute, k) + 2.1 * H.U32) * absref + 1e-300)


def _full_sampled_three_precisions(P, SG, wl, label, count, seed_):
    """A full-size contraction in f64, f32 and split-bf16, on `count` sampled outputs against
    the allowed-sector sampled oracle (binary64 inputs, binary32-rounded inputs, |inputs|)."""
    st = wl.steps[0]
    su, sv = _sym(wl, "U"), _sym(wl, "V")
    sw = O.output_symmetry(st.einsum, su, sv)
    red, full = H.random_w_positions(sw, count, np.random.default_rng(seed_))
    fu, fv = H.value_fn(wl, "U"), H.value_fn(wl, "V")
    say(f"{label} full: oracle on {len(red)} sampled outputs")
    ref = O.sample_contract_allowed(st.einsum, su, sv, fu, fv, full)
    ref32 = O.sample_contract_allowed(st.einsum, su, sv, H.f32_value_fn(fu), H.f32_value_fn(fv), full)
    absref = O.sample_contract_allowed(st.einsum, su, sv, H.value_fn(wl, "U", True), H.value_fn(wl, "V", True),
                                       full)
    k = H.contracted_extent(st.einsum, su)
    idx = torch.as_tensor(np.asarray(red, dtype=np.int64))
    for compute in ("f64", "f32", "bf16x3"):
        dt = torch.float64 if compute == "f64" else torch.float32
        u, v = _tensor(P, SG, wl, "U", dt), _tensor(P, SG, wl, "V", dt)
        info = P.plan(st.einsum, u, v, compute)
        w = P.output_like(st.einsum, u, v, dtype=torch.float64)
        say(f"{label} full {compute}: batch {info.group_size} m {info.m} k {info.k} n {info.n}, "
            f"{info.flops / 1e9:.1f} GFLOP, fused {info.fused}")
        P.contract_into(st.einsum, u, v, w, compute)
        torch.cuda.synchronize()
        del u, v
        got = H.to_np(w.data[tuple(idx.to(w.data.device).T)])
        del w
        torch.cuda.empty_cache()
        bf = H.bound_factor(compute, k)
        if compute == "f64":
            err = H.rel_err(got, ref)
            say(f"  {compute}: normwise relative error on samples {err:.3e}")
            assert err <= 1e-12
            assert np.all(np.abs(got - ref) <= bf * absref)
        else:
            say(f"  {compute}: normwise relative error on samples {H.rel_err(got, ref):.3e} (FP64 oracle)")
            assert np.all(np.abs(got - ref32) <= bf * (1.0 + 2.0 * H.U32) * absref)
            assert np.all(np.abs(got - ref) <= (bf + 2.1 * H.U32) * absref)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("label", synth.configs.SUITE_LABELS)
def test_suite_full_size_sampled(P, SG, label):
    _full_sampled_three_precisions(P, SG, synth.configs.paper_suite_case(label), f"suite {label}", 32, 7)


# ---------------------------------------------------------------------------
# The paper's generic (s, t, v) sweep at G = 4 and its G sweeps (MM, CC1, PEPS):
# small copies against the oracle in three precisions, and a few full-size
# cases on sampled outputs.
# ---------------------------------------------------------------------------
def _check_small(P, SG, wl, label):
    st = wl.steps[0]
    su, sv = _sym(wl, "U"), _sym(wl, "V")
    Ru, Rv = synth.host_input(wl, "U"), synth.host_input(wl, "V")
    ref, sw = O.contract_blocks(st.einsum, Ru, su, Rv, sv)
    absref, _ = O.contract_blocks(st.einsum, np.abs(Ru), su, np.abs(Rv), sv)
    assert sw.sign_string() == wl.operands["W"].signs
    k = H.contracted_extent(st.einsum, su)
    for compute in ("f64", "f32", "bf16x3"):
        dt = torch.float64 if compute == "f64" else torch.float32
        u, v = _tensor(P, SG, wl, "U", dt), _tensor(P, SG, wl, "V", dt)
        info = P.plan(st.einsum, u, v, compute)
        say(f"{label} small {compute}: batch {info.group_size} m {info.m} k {info.k} n {info.n}")
        w = P.output_like(st.einsum, u, v, dtype=torch.float64)
        P.contract_into(st.einsum, u, v, w, compute)
        got = H.to_np(w.data)
        if compute == "f64":
            assert H.rel_err(got, ref) <= 1e-12
            assert np.array_equal(O.expand(got, sw) == 0, O.expand(ref, sw) == 0)
        bound = H.bound_factor(compute, k) + (0 if compute == "f64" else 2.1 * H.U32)
        assert np.all(np.abs(got - ref) <= bound * absref + 1e-300)


@pytest.mark.parametrize("stv", synth.configs.STV_CASES)
def test_stv_sweep_small_vs_oracle(P, SG, stv):
    _check_small(P, SG, synth.configs.stv_case(*stv, n=3), f"stv {stv}")


@pytest.mark.parametrize("family", list(synth.configs.G_SWEEP))
def test_g_sweep_small_vs_oracle(P, SG, family):
    small = {"mm": dict(i=9, j=7, k=8), "cc1": dict(i=2, j=3, k=2, l=3, m=4, n=2),
             "peps": dict(i=4, j=3, k=2, l=2, m=3, n=2)}[family]
    for G in (synth.configs.G_SWEEP[family][0], synth.configs.G_SWEEP[family][-1]):
        _check_small(P, SG, synth.configs.g_sweep_case(family, G, small), f"G sweep {family} G={G}")


def _check_full_sampled(P, SG, wl, label):
    _full_sampled_three_precisions(P, SG, wl, label, 24, 11)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("stv", [(1, 1, 1), (2, 2, 2), (3, 1, 1), (2, 1, 2)])
def test_stv_sweep_full_size_sampled(P, SG, stv):
    _check_full_sampled(P, SG, synth.configs.stv_case(*stv), f"stv {stv}")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("family", list(synth.configs.G_SWEEP))
def test_g_sweep_full_size_sampled(P, SG, family):
    G = synth.configs.G_SWEEP[family][-1]
    _check_full_sampled(P, SG, synth.configs.g_sweep_case(family, G), f"G sweep {family} G={G}")
