"""Throughput of the irrep-alignment contraction on one MI355X.

One step = the whole hot path on one batch of synthetic input already resident
in HBM: align V_abcd and T_cdij, one sector-batched FP64 product, unalign
W_abij -- the coupled-cluster particle-particle ladder w_abij = sum_cd
V_abcd T_cdij with Z_8 symmetry, virtual block 24, occupied block 6.

Prints one JSON line: effective GFLOP/s (algorithmic flops of allowed blocks
only, 2 |G| M K N, divided by the measured step time), the roofline of the
dominant kernel (the sector product; its duration from HIP events the library
records around each launch on the stream it launches on), and the CPU oracle's
rate on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--extra PATH] [--all] [--suite]

Where the layout allows (here it does), one step runs the fused product: A is
read straight from V_abcd's standard form, B from T_cdij's and C written
straight into W_abij's through offset tables, so no aligned form is written
(include/symtensor.h, FUSED PRODUCT); the three separate steps are timed too
and reported in the --extra file.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3, "bf16x3": 2500.0}     # dense MFMA TFLOP/s, MI355X
HBM_PEAK_GBS = 8000.0
WORKLOAD = "ccd_ladder_z8"


# Sources that decide the sector product's machine code and launch choice;
# stored counter readings apply only while their digest is unchanged.
PRODUCT_SOURCES = ("paper_2007_08056_amd/csrc/gemm.hip", "paper_2007_08056_amd/csrc/plan.hpp",
                   "paper_2007_08056_amd/csrc/plan.cpp", "paper_2007_08056_amd/build.py")


def source_digest(*rel):
    h = hashlib.sha256()
    for r in rel:
        with open(os.path.join(ROOT, r), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def gemm_traffic(kernel_key, digest):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if still current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_digest") != digest:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(wl, budget_s=12.0, threads=None):
    """Loop-over-blocks oracle on a sample of V's stored blocks, timed on the host cores
    (all of them, or `threads` BLAS threads)."""
    import contextlib

    import numpy as np
    import oracle as O
    import synth
    from synth import philox
    limit = contextlib.nullcontext()
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        if threads:
            limit = threadpool_limits(limits=threads)
        cores = threads or max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        cores = threads or os.cpu_count() or 1
    with limit:
        return _oracle_sample(wl, budget_s, cores, np, O, synth, philox)


_ORACLE_INPUTS: dict = {}


def _oracle_sample(wl, budget_s, cores, np, O, synth, philox):
    st = wl.steps[0]
    g = O.Group(wl.group)
    ou, ov = wl.operands[st.u], wl.operands[st.v]
    su = O.Sym.make(ou.signs, ou.charge, ou.dims, g)
    sv = O.Sym.make(ov.signs, ov.charge, ov.dims, g)
    G = g.size
    # V blocks are generated once per process and shared by the timed samples
    cache = _ORACLE_INPUTS.setdefault(wl.name, {})
    if "Rv" not in cache:
        cache["Rv"] = synth.host_input(wl, st.v)          # T: 10.6 M elements
        cache["Ru"] = np.zeros(wl.reduced_shape(st.u))
        cache["made"] = set()
    Rv, Ru, made = cache["Rv"], cache["Ru"], cache["made"]
    blk = int(np.prod(ou.dims))
    all_blocks = [(a, b, c) for a in range(G) for b in range(G) for c in range(G)]
    done_blocks, flops_per_block = 0, 2 * blk * int(np.prod(ov.dims[2:])) * G
    elapsed = 0.0
    i = 0
    while i < len(all_blocks) and elapsed < budget_s:
        batch = all_blocks[i:i + 8]
        for b in batch:                                   # generate the sampled V blocks
            if b in made:
                continue
            made.add(b)
            lin = np.ravel_multi_index(b, (G, G, G)) * blk
            Ru[b] = philox.values_at(np.arange(lin, lin + blk), wl.seed, ou.tensor_id, ou.dist,
                                     ou.scale).reshape(ou.dims)
        t0 = time.perf_counter()
        O.contract_blocks(st.einsum, Ru, su, Rv, sv, u_blocks=batch)
        elapsed += time.perf_counter() - t0
        done_blocks += len(batch)
        i += len(batch)
    gflops = done_blocks * flops_per_block / elapsed / 1e9
    return {"value": round(gflops, 3), "unit": "GFLOP/s", "cores": int(cores), "kind": "oracle",
            "sample": f"loop-over-blocks oracle (numpy FP64) over {done_blocks} of {len(all_blocks)} "
                      f"stored blocks of V_abcd against all of T_cdij, {elapsed:.1f} s"}


def cold_and_copy(P, st, u, v, w, ws, reps=5):
    """Median step time with the 256 MB Infinity Cache flushed before every
    repetition (a 1 GiB write), and the device-to-device copy rate of 1 GiB
    (read + write bytes per second), the practical ceiling of a transform."""
    import torch
    flush = torch.empty(2 ** 27, dtype=torch.float64, device="cuda:0")
    times = []
    for _ in range(reps):
        flush.fill_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        P.contract_into(st.einsum, u, v, w, "f64", ws)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    src = torch.ones(2 ** 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del flush, src, dst
    return sorted(times)[len(times) // 2], copy_gbs


def chain_flops(wl, compute, cplx=False):
    """Algorithmic flops of a workload's contraction chain (host-only planning); complex
    operands count 8 real flops per complex multiply-add."""
    from paper_2007_08056_amd import _lib as L
    dt = L.SYMT_C128 if cplx else L.SYMT_F64
    total = 0.0
    for st in wl.steps:
        ou, ov = wl.operands[st.u], wl.operands[st.v]
        info = L.plan(st.einsum, L.make_group(wl.group),
                      L.TensorDesc(ou.signs, ou.charge, ou.dims, dt, None, None, ou.sectors),
                      L.TensorDesc(ov.signs, ov.charge, ov.dims, dt, None, None, ov.sectors), None,
                      L.COMPUTE[compute])
        total += info.flops
    return total


def time_workload(P, SG, wl, compute, steps, warmup, grad=False, cplx=False):
    """ms per step and effective TFLOP/s of a workload's contraction chain (optionally fwd+bwd).

    cplx: complex operands (storage complex128 for f64, complex64 for f32), the
    imaginary parts from a second seeded fill of the same distribution.

    With grad, the backward of every step is two contractions of the forward's
    size (dU and dV), so the step does three times the forward's flops.
    Warm-up runs at least `warmup` steps and at least 50 ms (clocks ramp up
    after host-side idle); the figure is the median of three timed batches of
    at least `steps` steps and 10 ms each.
    """
    import torch
    dt = torch.float64 if compute == "f64" else torch.float32
    t = {}
    for name in wl.inputs:
        op = wl.operands[name]
        d = SG.device_input(wl, name, dtype=dt, device="cuda:0")
        if cplx:
            im = SG.fill_(torch.empty_like(d), wl.seed, op.tensor_id + 1000, op.dist, op.scale)
            d = torch.complex(d, im)
        if grad and name != "R":
            d.requires_grad_(True)
        t[name] = P.SymTensor(d, op.signs, op.charge, wl.group, None, op.sectors)
    flops = chain_flops(wl, compute, cplx) * (3.0 if grad else 1.0)

    def step():
        cur = dict(t)
        for st in wl.steps:
            cur[st.w] = P.einsum(st.einsum, cur[st.u], cur[st.v], compute)
        if grad:
            (cur[wl.output].data * cur["R"].data).sum().backward()

    def run(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            step()
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    n, spent = 0, 0.0
    while n < warmup or spent < 0.05:
        spent += run(1)
        n += 1
    per = spent / n
    batch = max(steps, int(0.01 / max(per, 1e-6)) + 1)
    ms = sorted(run(batch) * 1e3 / batch for _ in range(3))[1]
    return {"ms_per_step": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 2),
            "flops_per_step": flops, "steps_per_batch": batch}


def dense_ms(wl, reps=3):
    """The symmetry-oblivious baseline of the paper's G sweeps: one dense f64 einsum of
    full tensors of the same shapes (every block materialised; values are random, the
    time does not depend on them), through torch's vendor BLAS."""
    import torch
    st = wl.steps[0]
    G = wl.group_size
    full = lambda name: torch.randn([G * d for d in wl.operands[name].dims], dtype=torch.float64,  # noqa: E731
                                    device="cuda:0")
    u, v = full(st.u), full(st.v)
    torch.einsum(st.einsum, u, v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        torch.einsum(st.einsum, u, v)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    del u, v
    torch.cuda.empty_cache()
    return round(ms, 4)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--extra", default="", help="write per-kernel details to this JSON file")
    ap.add_argument("--all", action="store_true",
                    help="also time every workload in every precision (written to --extra)")
    ap.add_argument("--suite", action="store_true",
                    help="also time the paper's Table 2 suite at full size (written to --extra)")
    ap.add_argument("--sweeps", action="store_true",
                    help="also time the paper's (s, t, v) sweep and its G sweeps (written to --extra)")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run one plain elementwise kernel that reads and writes 256 MiB "
                         "(the reference for scaling HBM byte counters)")
    ap.add_argument("--only", default="",
                    help="WORKLOAD/COMPUTE (e.g. ccd_ladder_z8/bf16x3): time that one workload's chain "
                         "(as --all does), print one line and exit; for profiling runs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the contraction is benchmarked on a single MI355X "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2007_08056_amd as P
    import synth
    import synth.gpu as SG

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only:
        name, compute = args.only.split("/")
        r = time_workload(P, SG, synth.configs.get(name), compute, args.steps, args.warmup)
        print(json.dumps({"workload": name, "compute": compute, **r}), flush=True)
        return
    wl = synth.configs.get(WORKLOAD)
    st = wl.steps[0]
    ou, ov, ow = (wl.operands[x] for x in (st.u, st.v, st.w))
    u = P.SymTensor(SG.device_input(wl, st.u, device=dev), ou.signs, ou.charge, wl.group)
    v = P.SymTensor(SG.device_input(wl, st.v, device=dev), ov.signs, ov.charge, wl.group)
    w = P.output_like(st.einsum, u, v)
    info = P.plan(st.einsum, u, v, "f64", w)
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    if args.calibrate:
        x = torch.ones(32 * 2 ** 20, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        del x, y
    for _ in range(args.warmup):
        P.contract_into(st.einsum, u, v, w, "f64", ws)
    torch.cuda.synchronize()
    P.read_timing(0)
    P.set_timing(0, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P.contract_into(st.einsum, u, v, w, "f64", ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    P.set_timing(0, False)
    ms, launches = P.read_timing(0)
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = info.flops / (ms_step * 1e-3) / 1e9

    # the three separate steps on the same inputs: per-transform HBM rates
    wsteps = P.output_like(st.einsum, u, v)
    for _ in range(2):
        P.contract_into(st.einsum, u, v, wsteps, "f64", steps=True)
    torch.cuda.synchronize()
    P.read_timing(0)
    P.set_timing(0, True)
    for _ in range(5):
        P.contract_into(st.einsum, u, v, wsteps, "f64", steps=True)
    torch.cuda.synchronize()
    P.set_timing(0, False)
    ms_s, launches_s = P.read_timing(0)
    same = bool(torch.equal(wsteps.data, w.data))
    del wsteps

    gemm_ms = ms[2] / max(1, launches[2])
    achieved = info.flops / (gemm_ms * 1e-3) / 1e12
    digest = source_digest(*PRODUCT_SOURCES)
    traffic = gemm_traffic("sector_gemm_f64_ccd_ladder_z8", digest)
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["f64"], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK["f64"], 4), "traffic": traffic}

    extra = {
        "fused": bool(info.fused),
        "fused_v": bool(info.fused_v),
        "kernel_ms_per_launch": {name: (ms[i] / launches[i] if launches[i] else None)
                                 for i, name in enumerate(("offset_tables" if info.fused else "align_u",
                                                           "align_v", "sector_gemm", "unalign_w"))},
        "steps_kernel_ms_per_launch": {name: (ms_s[i] / launches_s[i] if launches_s[i] else None)
                                       for i, name in enumerate(("align_u", "align_v", "sector_gemm",
                                                                 "unalign_w"))},
        "steps_result_identical_to_fused": same,
        "shape": {"batch": info.group_size, "m": info.m, "k": info.k, "n": info.n},
        "flops": info.flops,
        "bytes_u": info.elems_u * 8, "bytes_v": info.elems_v * 8, "bytes_w": info.elems_w * 8,
        "gemm_source_digest": digest,
    }
    cold_ms, copy_gbs = cold_and_copy(P, st, u, v, w, ws)
    extra["cold_ms_per_step"] = round(cold_ms, 4)
    extra["cold_gflops"] = round(info.flops / (cold_ms * 1e-3) / 1e9, 2)
    extra["d2d_copy_GBs"] = round(copy_gbs, 1)
    xf = extra["steps_kernel_ms_per_launch"]
    for key, nbytes in (("align_u", 2 * info.elems_u * 8), ("align_v", 2 * info.elems_v * 8),
                        ("unalign_w", 2 * info.elems_w * 8)):
        if xf[key]:
            extra[key + "_GBs"] = nbytes / (xf[key] * 1e-3) / 1e9

    if args.all:
        import synth as S
        table = {}
        for name, computes, grad, cplx in (("plain_z4", ("f64",), False, False),
                                           ("ccd_ladder_z8", ("f32", "bf16x3"), False, False),
                                           ("mps_env_z2z3", ("f64", "f32", "bf16x3"), False, False),
                                           ("ccd_ladder_z16", ("f64", "f32", "bf16x3"), False, False),
                                           ("mps_env_grad", ("f64", "f32"), False, False),
                                           ("mps_env_grad", ("f64", "f32"), True, False),
                                           ("ccd_ladder_z8", ("f64", "f32"), False, True),
                                           ("ccd_ladder_z8_sub", ("f64", "f32", "bf16x3"), False, False),
                                           ("mps_env_z2z3", ("f64", "f32"), False, True)):
            wlx = S.configs.get(name)
            for c in computes:
                n_steps = 3 if name == "ccd_ladder_z16" else 10
                r = time_workload(P, SG, wlx, c, n_steps, 2, grad, cplx)
                key = f"{name}/{c}" + ("/complex" if cplx else "") + ("/fwd+bwd" if grad else "")
                table[key] = r
                print(f"{key}: {r['ms_per_step']:.3f} ms, {r['tflops']:.1f} TFLOP/s", file=sys.stderr, flush=True)
                torch.cuda.empty_cache()
        extra["workloads"] = table

    if args.sweeps:
        import synth as S
        stv = {}
        for case in S.configs.STV_CASES:
            wlx = S.configs.stv_case(*case)
            r = time_workload(P, SG, wlx, "f64", 3, 2)
            r["einsum"], r["block_dim"] = wlx.steps[0].einsum, wlx.operands["U"].dims[0]
            stv["".join(map(str, case))] = r
            print(f"stv {case}: {r['ms_per_step']:.3f} ms, {r['tflops']:.1f} TFLOP/s", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
        extra["stv_sweep"] = stv
        gs = {}
        for fam, Gs in S.configs.G_SWEEP.items():
            for G in Gs:
                wlx = S.configs.g_sweep_case(fam, G)
                r = time_workload(P, SG, wlx, "f64", 5, 2)
                r["dense_ms"] = dense_ms(wlx)
                gs[f"{fam}/G={G}"] = r
                print(f"G sweep {fam} G={G}: {r['ms_per_step']:.3f} ms ({r['tflops']:.1f} TFLOP/s); "
                      f"dense {r['dense_ms']:.3f} ms", file=sys.stderr, flush=True)
                torch.cuda.empty_cache()
        extra["g_sweep"] = gs

    if args.suite:
        import synth as S
        table = {}
        for label in S.configs.SUITE_LABELS:
            wlx = S.configs.paper_suite_case(label)
            for c in ("f64", "f32", "bf16x3"):
                try:
                    r = time_workload(P, SG, wlx, c, 3, 2)
                except P._lib.SymtError as e:      # e.g. split-bf16 with K not a multiple of 8
                    table[f"{label}/{c}"] = {"unsupported": str(e)}
                    continue
                table[f"{label}/{c}"] = r
                print(f"suite {label}/{c}: {r['ms_per_step']:.3f} ms, {r['tflops']:.1f} TFLOP/s",
                      file=sys.stderr, flush=True)
                torch.cuda.empty_cache()
        extra["suite"] = table

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl)
        extra["cpu_baseline_1thread"] = cpu_baseline(wl, budget_s=6.0, threads=1)

    line = {
        "metric": "effective GFLOP/s of symmetric contraction (fwd) vs FP64 plain",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Philox4x32-10, N(0,1) V, 1e-2 N(0,1) T)",
        "config": {"workload": "ccd_ladder_z8: w_abij = sum_cd V_abcd T_cdij, Z_8, virtual block 24, "
                               "occupied block 6, FP64; aligned product 8 x (4608 x 4608 x 288)",
                   "group": "Z_8", "einsum": st.einsum, "flops_per_step": info.flops},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if args.extra:
        with open(args.extra, "w") as f:
            json.dump(extra, f, indent=1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
