"""Host-side checks of the benchmark script: its one-GPU guard and the flop count
that its throughput divides by.

The ladder step w_abij = sum_cd V_abcd T_cdij over Z_G (a coupled-cluster
contraction of the kind Sec. 4 benchmarks) does one multiply-add per element
triple of every block triple whose sectors conserve charge (Sec. 2.2, Eq. symtsr,
signs ++-- on both operands): a + b = c + d for V and c + d = i + j for T.
Counting those block triples by brute force over all sector labels fixes the
flops independently of the planner's aligned shapes (the product step of Alg. 2
costs 2 |G| M K N, Sec. 2.1)."""

import itertools
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _ladder_flops_brute(G, vb, ob):
    n = 0
    for a, b, c, d in itertools.product(range(G), repeat=4):
        if (a + b - c - d) % G:
            continue
        n += sum(1 for i, j in itertools.product(range(G), repeat=2) if (c + d - i - j) % G == 0)
    return 2.0 * n * vb ** 4 * ob ** 2


@pytest.mark.parametrize("name,G,vb,ob", [("ccd_ladder_z8", 8, 24, 6), ("ccd_ladder_z16", 16, 32, 8)])
def test_bench_flops_match_block_count(name, G, vb, ob):
    import bench
    import synth
    got = bench.chain_flops(synth.configs.get(name), "f64")
    assert got == _ladder_flops_brute(G, vb, ob)
    # the aligned product's closed form, 2 |G| M K N with M = K = |G| vb^2, N = |G| ob^2
    assert got == 2.0 * G * (G * vb * vb) ** 2 * (G * ob * ob)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
