"""Throughput of the irrep-alignment contraction on one MI355X.

One step = the whole hot path on one batch of synthetic input already resident
in HBM: the coupled-cluster particle-particle ladder w_abij = sum_cd V_abcd
T_cdij with Z_16 symmetry, virtual block 32, occupied block 8, in FP64 (8.80
TFLOP of allowed-block products per step).  Where the layout allows (here it
does), the step is the fused product: offset tables, then one sector-batched
product that reads V_abcd and T_cdij in their standard reduced forms and writes
W_abij in place (include/symtensor.h, FUSED PRODUCT).

Prints one JSON line: effective GFLOP/s of that forward step (algorithmic flops
of allowed blocks only, 2 |G| M K N, divided by the measured step time), plus
* roofline: the sector product's achieved TFLOP/s (HIP events that the library
  records around its launches on the stream it launches on) against the f64
  MFMA peak, and its HBM traffic from the committed counter summary;
* error: the forward's normwise and componentwise error against the oracle on
  sampled outputs, computed outside the timed region;
* precisions: the same step in f32 and split-bf16 with their errors;
* fwd_bwd: the differentiated tensor-network chain (MPS environment, bond 128,
  L = <E', R>, forward plus the hand-written backward) in f64 and f32;
* cpu_baseline: the CPU oracle (loop over blocks, NumPy FP64) on a bounded
  sample of the same contraction, on all host cores and on one.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--extra PATH] [--all] [--suite]
                       [--sweeps] [--ladder-z8] [--calibrate] [--only WORKLOAD/COMPUTE]
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
WORKLOAD = "ccd_ladder_z16"
METRIC = "effective GFLOP/s of symmetric contraction (fwd, fwd+bwd) vs FP64 plain at stated rel. error"


# Sources that decide the sector product's machine code and launch choice;
# stored counter readings apply only while their digest is unchanged.
PRODUCT_SOURCES = ("paper_2007_08056_amd/csrc/gemm.hip", "paper_2007_08056_amd/csrc/plan.hpp",
                   "paper_2007_08056_amd/csrc/plan.cpp", "paper_2007_08056_amd/csrc/sk_index.hpp",
                   "paper_2007_08056_amd/build.py")


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


def _host_description():
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model


def cpu_baseline(wl, blocks=64, threads=None, runs=3):
    """The loop-over-blocks oracle (Alg. 1 generalised, NumPy FP64) on a bounded sample of the
    workload: `blocks` stored blocks of U (spread evenly over its stored-sector tuples) against
    all of V, one warm-up and `runs` timed repetitions (median), input generation excluded.
    `threads`: BLAS threads (None: all the process may use)."""
    import contextlib

    import numpy as np
    import oracle as O
    import synth
    from synth import host as synth_host
    from threadpoolctl import threadpool_info, threadpool_limits
    limit = threadpool_limits(limits=threads) if threads else contextlib.nullcontext()
    with limit:
        info = threadpool_info()
        blas = [f"{p.get('internal_api')} {p.get('version')}" for p in info if p.get("user_api") == "blas"]
        used = max([p.get("num_threads", 1) for p in info if p.get("user_api") == "blas"] or [1])
        st = wl.steps[0]
        g = O.Group(wl.group)
        ou, ov = wl.operands[st.u], wl.operands[st.v]
        su = O.Sym.make(ou.signs, ou.charge, ou.dims, g)
        sv = O.Sym.make(ov.signs, ov.charge, ov.dims, g)
        shape = wl.reduced_shape(st.u)
        stored = list(O.stored_tuples(su))
        pick = [stored[i] for i in np.linspace(0, len(stored) - 1, blocks).astype(int)]
        Rv = synth.host_input(wl, st.v)
        Ru = np.zeros(shape)                     # untouched pages outside the sampled blocks
        blk = int(np.prod(ou.dims))
        for b in pick:
            lin = int(np.ravel_multi_index(b, shape[:len(b)])) * blk
            Ru[b] = synth_host.fill(ou.dims, wl.seed, ou.tensor_id, ou.dist, ou.scale, first=lin)
        flops = O.flop_count(st.einsum, su, sv) / len(stored) * len(pick)
        times = []
        for rep in range(runs + 1):
            t0 = time.perf_counter()
            O.contract_blocks(st.einsum, Ru, su, Rv, sv, u_blocks=pick)
            if rep:
                times.append(time.perf_counter() - t0)
        med = sorted(times)[len(times) // 2]
    return {"value": round(flops / med / 1e9, 3), "unit": "GFLOP/s", "cores": int(used), "kind": "oracle",
            "sample": f"loop-over-blocks oracle (NumPy FP64) over {len(pick)} of {len(stored)} stored blocks of "
                      f"{st.u} against all of {st.v} ({flops / 1e9:.1f} GFLOP), median of {runs} after one "
                      f"warm-up: {med:.2f} s",
            "host": _host_description(), "blas": ", ".join(blas)}


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
    Warm-up runs at least `warmup` steps and at least 0.5 s (the device's clocks
    ramp up over tens of milliseconds after host-side idle: a bond-128 chain
    step runs about 15% longer in its first 30 ms of work); the figure is the
    median of three timed batches of at least `steps` steps and 50 ms each.
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
        if grad:
            # each step's gradients are its own (as a training step that clears
            # them to None): no add of the previous step's into them
            for x in t.values():
                x.data.grad = None
        for st in wl.steps:
            cur[st.w] = P.einsum(st.einsum, cur[st.u], cur[st.v], compute)
        if grad:
            # L = <E', R> as one dot product (its backward: one scaled copy of R)
            torch.dot(cur[wl.output].data.reshape(-1), cur["R"].data.reshape(-1)).backward()

    def run(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            step()
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    n, spent = 0, 0.0
    while n < warmup or spent < 0.5:
        spent += run(1)
        n += 1
    per = spent / n
    batch = max(steps, int(0.05 / max(per, 1e-6)) + 1)
    ms = sorted(run(batch) * 1e3 / batch for _ in range(3))[1]
    return {"ms_per_step": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 2),
            "flops_per_step": flops, "steps_per_batch": batch}


def timed_steps(step, steps, warmup):
    """ms per step of `steps` calls after `warmup` (wall clock between two device synchronisations)."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def random_reduced_positions(shape, count, seed):
    """`count` random coordinates of a reduced form (plain indexing, no symmetry arithmetic)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, d, count) for d in shape], axis=1).astype(np.int64)


def chain_roofline_ms(wl, compute, grad):
    """Roofline time of a contraction chain (forward, plus the backward's two contractions per
    step with grad): each contraction costs max(flops / MFMA peak, bytes / HBM peak), its bytes
    being one read of U and V and one write of W in the storage type (the fused path's minimum)."""
    from paper_2007_08056_amd import _lib as L
    elem = 8 if compute == "f64" else 4
    g = L.make_group(wl.group)
    total = 0.0

    def cost(sub, a, b):
        info = L.plan(sub, g, L.TensorDesc(a.signs, a.charge, a.dims, L.SYMT_F64, None),
                      L.TensorDesc(b.signs, b.charge, b.dims, L.SYMT_F64, None), None, L.COMPUTE[compute])
        byts = (info.elems_u + info.elems_v + info.elems_w) * elem
        return max(info.flops / (PEAK[compute] * 1e12), byts / (HBM_PEAK_GBS * 1e9))
    for st in wl.steps:
        ou, ov, ow = wl.operands[st.u], wl.operands[st.v], wl.operands[st.w]
        tu, rest = st.einsum.split(",")
        tv, tw = rest.split("->")
        total += cost(st.einsum, ou, ov)
        if grad:
            total += cost(f"{tw},{tv}->{tu}", ow, ov) + cost(f"{tu},{tw}->{tv}", ou, ow)
    return total * 1e3


def cpu_leg(wl, samples, losses):
    """The CPU side of the benchmark: the oracle's own throughput (cpu_baseline, all host cores
    and one), and the oracle's values at the GPU's sampled outputs (the stated errors)."""
    import numpy as np
    import oracle as O
    import synth
    from synth import host as synth_host
    st = wl.steps[0]
    g = O.Group(wl.group)
    sym = {k: O.Sym.make(op.signs, op.charge, op.dims, g) for k, op in wl.operands.items()}
    su, sv, sw = sym[st.u], sym[st.v], sym[st.w]
    out = {}
    red = samples["positions"]
    full = []
    for r in red:
        secs = O.full_sectors(sw, tuple(int(x) for x in r[: sw.order - 1]))
        full.append([S * n + int(i) for S, n, i in zip(secs, sw.dims, r[sw.order - 1:])])
    full = np.asarray(full, dtype=np.int64)

    def vf(name, absolute=False, round32=False):
        op = wl.operands[name]
        shape = wl.reduced_shape(name)

        def fn(secs, inner):
            x = synth_host.values_at(np.ravel_multi_index(tuple(secs) + tuple(inner), shape), wl.seed,
                                     op.tensor_id, op.dist, op.scale)
            if round32:
                x = x.astype(np.float32).astype(np.float64)
            return np.abs(x) if absolute else x
        return fn
    ref = O.sample_contract_allowed(st.einsum, su, sv, vf(st.u), vf(st.v), full)
    absref = O.sample_contract_allowed(st.einsum, su, sv, vf(st.u, True), vf(st.v, True), full)
    ref32 = O.sample_contract_allowed(st.einsum, su, sv, vf(st.u, round32=True), vf(st.v, round32=True), full)
    den = float(np.max(np.abs(ref)))
    for compute, got in samples["values"].items():
        e = {"vs": "FP64 oracle, same sampled outputs", "samples": len(full),
             "normwise": float(np.max(np.abs(got - ref)) / den),
             "componentwise": float(np.max(np.abs(got - ref) / absref))}
        if compute != "f64":
            e["normwise_vs_binary32_inputs"] = float(np.max(np.abs(got - ref32)) / den)
        out[compute] = e
    # the differentiated chain: L of the library against the oracle's L
    gwl = synth.configs.mps_env_grad()
    gsym = {k: O.Sym.make(op.signs, op.charge, op.dims, O.Group(gwl.group)) for k, op in gwl.operands.items()}
    cur = {k: synth.host_input(gwl, k) for k in gwl.inputs}
    for gst in gwl.steps:
        cur[gst.w], _ = O.contract_blocks(gst.einsum, cur[gst.u], gsym[gst.u], cur[gst.v], gsym[gst.v])
    l_ref = float(np.sum(cur[gwl.output] * cur["R"]))
    out["loss"] = {c: abs(v - l_ref) / abs(l_ref) for c, v in losses.items()}
    out["cpu"] = cpu_baseline(wl)
    out["cpu_1thread"] = cpu_baseline(wl, blocks=16, threads=1)
    return out


def ladder_z8_details(P, SG, extra):
    """The Z_8 ladder (f64): fused step, its three separate steps, per-transform HBM rates."""
    import torch
    import synth
    wl = synth.configs.get("ccd_ladder_z8")
    st = wl.steps[0]
    dev = torch.device("cuda:0")
    ou, ov = (wl.operands[x] for x in (st.u, st.v))
    u = P.SymTensor(SG.device_input(wl, st.u, device=dev), ou.signs, ou.charge, wl.group)
    v = P.SymTensor(SG.device_input(wl, st.v, device=dev), ov.signs, ov.charge, wl.group)
    w = P.output_like(st.einsum, u, v)
    info = P.plan(st.einsum, u, v, "f64", w)
    ws = torch.empty(info.workspace_bytes, dtype=torch.uint8, device=dev)
    P.read_timing(0)
    P.set_timing(0, True)
    ms_step = timed_steps(lambda: P.contract_into(st.einsum, u, v, w, "f64", ws), 20, 30)
    P.set_timing(0, False)
    ms, launches = P.read_timing(0)
    wsteps = P.output_like(st.einsum, u, v)
    P.set_timing(0, True)
    timed_steps(lambda: P.contract_into(st.einsum, u, v, wsteps, "f64", steps=True), 5, 2)
    P.set_timing(0, False)
    ms_s, launches_s = P.read_timing(0)
    xf = {name: (ms_s[i] / launches_s[i] if launches_s[i] else None)
          for i, name in enumerate(("align_u", "align_v", "sector_gemm", "unalign_w"))}
    d = {"ms_per_step": round(ms_step, 4), "tflops": round(info.flops / (ms_step * 1e-3) / 1e12, 2),
         "fused": bool(info.fused), "fused_v": bool(info.fused_v),
         "kernel_ms_per_launch": {name: (ms[i] / launches[i] if launches[i] else None)
                                  for i, name in enumerate(("offset_tables", "align_v", "sector_gemm", "unalign_w"))},
         "steps_kernel_ms_per_launch": xf,
         "steps_result_identical_to_fused": bool(torch.equal(wsteps.data, w.data))}
    for key, nbytes in (("align_u", 2 * info.elems_u * 8), ("align_v", 2 * info.elems_v * 8),
                        ("unalign_w", 2 * info.elems_w * 8)):
        if xf[key]:
            d[key + "_GBs"] = nbytes / (xf[key] * 1e-3) / 1e9
    extra["ccd_ladder_z8"] = d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU leg (oracle baseline and sampled errors)")
    ap.add_argument("--extra", default="", help="write per-kernel details to this JSON file")
    ap.add_argument("--all", action="store_true",
                    help="also time every workload in every precision (written to --extra)")
    ap.add_argument("--suite", action="store_true",
                    help="also time the paper's Table 2 suite at full size (written to --extra)")
    ap.add_argument("--sweeps", action="store_true",
                    help="also time the paper's (s, t, v) sweep and its G sweeps (written to --extra)")
    ap.add_argument("--ladder-z8", action="store_true",
                    help="also time the Z_8 ladder's fused and three-step paths (written to --extra)")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run one plain elementwise kernel that reads and writes 256 MiB "
                         "(the reference for scaling HBM byte counters)")
    ap.add_argument("--only", default="",
                    help="WORKLOAD/COMPUTE[/grad] (e.g. ccd_ladder_z8/bf16x3, mps_env_grad/f64/grad): time that "
                         "one workload's chain (forward, or forward and backward), print one line and exit; "
                         "for profiling runs")
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline step only (no precisions, fwd+bwd or CPU leg); for profiling runs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the contraction is benchmarked on a single MI355X "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2007_08056_amd as P
    import synth
    import synth.gpu as SG

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate:
        x = torch.ones(32 * 2 ** 20, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        del x, y
    if args.only:
        name, compute, *mode = args.only.split("/")
        grad = mode == ["grad"]
        r = time_workload(P, SG, synth.configs.get(name), compute, args.steps, args.warmup, grad=grad)
        print(json.dumps({"workload": name, "compute": compute, "fwd+bwd": grad, **r}), flush=True)
        return

    wl = synth.configs.get(WORKLOAD)
    st = wl.steps[0]
    ou, ov = wl.operands[st.u], wl.operands[st.v]
    positions = random_reduced_positions(wl.reduced_shape(st.w), 256, 5)
    pos_t = torch.from_numpy(positions).to(dev)
    values = {}
    extra = {}

    def make(dtype, wdtype=torch.float64):
        u = P.SymTensor(SG.device_input(wl, st.u, dtype=dtype, device=dev), ou.signs, ou.charge, wl.group)
        v = P.SymTensor(SG.device_input(wl, st.v, dtype=dtype, device=dev), ov.signs, ov.charge, wl.group)
        w = P.output_like(st.einsum, u, v, dtype=wdtype)
        return u, v, w

    # ---- headline: Z_16 ladder, FP64, forward
    u, v, w = make(torch.float64)
    info = P.plan(st.einsum, u, v, "f64", w)
    ws = torch.empty(max(1, info.workspace_bytes), dtype=torch.uint8, device=dev)
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
    values["f64"] = w.data[tuple(pos_t.T)].cpu().numpy()
    gemm_ms = ms[2] / max(1, launches[2])
    achieved = info.flops / (gemm_ms * 1e-3) / 1e12
    digest = source_digest(*PRODUCT_SOURCES)
    traffic = gemm_traffic(f"sector_gemm_f64_{WORKLOAD}", digest)
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["f64"], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK["f64"], 4), "traffic": traffic}
    extra["headline"] = {
        "fused": bool(info.fused), "fused_v": bool(info.fused_v),
        "kernel_ms_per_launch": {name: (ms[i] / launches[i] if launches[i] else None)
                                 for i, name in enumerate(("offset_tables", "align_v", "sector_gemm",
                                                           "unalign_w"))},
        "shape": {"batch": info.group_size, "m": info.m, "k": info.k, "n": info.n}, "flops": info.flops,
        "gemm_source_digest": digest}
    del u, v, w, ws
    torch.cuda.empty_cache()

    precisions, fwd_bwd, losses = {}, {}, {}
    if not args.headline_only:
        # ---- the same step in binary32 (binary32 W) and split-bf16 (binary32 operands, binary64 W)
        for compute in ("f32", "bf16x3"):
            u, v, w = make(torch.float32, torch.float32 if compute == "f32" else torch.float64)
            ci = P.plan(st.einsum, u, v, compute, w)
            wsc = torch.empty(max(1, ci.workspace_bytes), dtype=torch.uint8, device=dev)
            P.read_timing(0)
            P.set_timing(0, True)
            m = timed_steps(lambda: P.contract_into(st.einsum, u, v, w, compute, wsc), 5, 2)
            P.set_timing(0, False)
            cms, cl = P.read_timing(0)
            gm = cms[2] / max(1, cl[2])
            values[compute] = w.data[tuple(pos_t.T)].double().cpu().numpy()
            mfma_work = ci.flops * (3.0 if compute == "bf16x3" else 1.0)
            precisions[compute] = {"ms_per_step": round(m, 4), "gflops": round(ci.flops / (m * 1e-3) / 1e9, 1),
                                   "sector_gemm_ms": round(gm, 4),
                                   "mfma_frac": round(mfma_work / (gm * 1e-3) / 1e12 / PEAK[compute], 4),
                                   "fused": bool(ci.fused)}
            del u, v, w, wsc
            torch.cuda.empty_cache()
        # ---- the differentiated MPS environment chain, forward + backward (bond 128)
        gwl = synth.configs.get("mps_env_grad")
        for compute in ("f64", "f32"):
            r = time_workload(P, SG, gwl, compute, 20, 5, grad=True)
            roof = chain_roofline_ms(gwl, compute, True)
            fwd = time_workload(P, SG, gwl, compute, 20, 5)
            fwd_bwd[compute] = {"ms_per_step": r["ms_per_step"], "gflops": round(r["tflops"] * 1e3, 1),
                                "flops_per_step": r["flops_per_step"],
                                "mfma_frac": round(r["tflops"] / PEAK[compute], 4),
                                "roofline_ms": round(roof, 4), "roofline_frac": round(roof / r["ms_per_step"], 4),
                                "fwd_ms_per_step": fwd["ms_per_step"], "fwd_gflops": round(fwd["tflops"] * 1e3, 1)}
            dt = torch.float64 if compute == "f64" else torch.float32
            t = {}
            for name in gwl.inputs:
                op = gwl.operands[name]
                t[name] = P.SymTensor(SG.device_input(gwl, name, dtype=dt, device=dev), op.signs, op.charge,
                                      gwl.group)
            for gst in gwl.steps:
                t[gst.w] = P.einsum(gst.einsum, t[gst.u], t[gst.v], compute)
            losses[compute] = float((t[gwl.output].data.double() * t["R"].data.double()).sum().item())
            del t
            torch.cuda.empty_cache()

    if args.ladder_z8:
        ladder_z8_details(P, SG, extra)
    if args.all:
        table = {}
        for name, computes, grad, cplx in (("plain_z4", ("f64",), False, False),
                                           ("ccd_ladder_z8", ("f64", "f32", "bf16x3"), False, False),
                                           ("mps_env_z2z3", ("f64", "f32", "bf16x3"), False, False),
                                           ("ccd_ladder_z16", ("f64", "f32", "bf16x3"), False, False),
                                           ("mps_env_grad", ("f64", "f32"), False, False),
                                           ("mps_env_grad", ("f64", "f32"), True, False),
                                           ("ccd_ladder_z8", ("f64", "f32"), False, True),
                                           ("ccd_ladder_z8_sub", ("f64", "f32", "bf16x3"), False, False),
                                           ("mps_env_z2z3", ("f64", "f32"), False, True)):
            wlx = synth.configs.get(name)
            for c in computes:
                n_steps = 3 if name == "ccd_ladder_z16" else 10
                r = time_workload(P, SG, wlx, c, n_steps, 2, grad, cplx)
                key = f"{name}/{c}" + ("/complex" if cplx else "") + ("/fwd+bwd" if grad else "")
                table[key] = r
                print(f"{key}: {r['ms_per_step']:.3f} ms, {r['tflops']:.1f} TFLOP/s", file=sys.stderr, flush=True)
                torch.cuda.empty_cache()
        extra["workloads"] = table
    if args.sweeps:
        stv = {}
        for case in synth.configs.STV_CASES:
            wlx = synth.configs.stv_case(*case)
            r = time_workload(P, SG, wlx, "f64", 3, 2)
            r["einsum"], r["block_dim"] = wlx.steps[0].einsum, wlx.operands["U"].dims[0]
            stv["".join(map(str, case))] = r
            print(f"stv {case}: {r['ms_per_step']:.3f} ms, {r['tflops']:.1f} TFLOP/s", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
        extra["stv_sweep"] = stv
        gs = {}
        for fam, Gs in synth.configs.G_SWEEP.items():
            for G in Gs:
                r = time_workload(P, SG, synth.configs.g_sweep_case(fam, G), "f64", 5, 2)
                gs[f"{fam}/G={G}"] = r
                print(f"G sweep {fam} G={G}: {r['ms_per_step']:.3f} ms ({r['tflops']:.1f} TFLOP/s)",
                      file=sys.stderr, flush=True)
                torch.cuda.empty_cache()
        extra["g_sweep"] = gs
    if args.suite:
        table = {}
        for label in synth.configs.SUITE_LABELS:
            wlx = synth.configs.paper_suite_case(label)
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

    cpu, errors = None, None
    if not args.no_cpu and not args.headline_only:
        leg = cpu_leg(wl, {"positions": positions, "values": values}, losses)
        cpu = leg.pop("cpu")
        cpu["single_thread"] = leg.pop("cpu_1thread")
        errors = leg
    for compute in precisions:
        if errors and compute in errors:
            precisions[compute]["error"] = errors[compute]
    for compute in fwd_bwd:
        if errors and compute in errors.get("loss", {}):
            fwd_bwd[compute]["loss_rel_err_vs_oracle"] = errors["loss"][compute]

    line = {
        "metric": METRIC,
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
        "config": {"workload": "ccd_ladder_z16: w_abij = sum_cd V_abcd T_cdij, Z_16, virtual block 32, "
                               "occupied block 8, FP64, forward; aligned product 16 x (16384 x 16384 x 1024)",
                   "group": "Z_16", "einsum": st.einsum, "flops_per_step": info.flops},
        "error": errors["f64"] if errors else None,
        "precisions": precisions,
        "fwd_bwd": {"workload": "mps_env_grad: E'_ABC = E_abc A_asA W_bsSB A_cSC over Z_2 x Z_3, bond 128, "
                                "L = <E', R>; forward and the hand-written backward (dL/dE, dL/dA, dL/dW)",
                    **fwd_bwd} if fwd_bwd else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if args.extra:
        with open(args.extra, "w") as f:
            json.dump(extra, f, indent=1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
