#!/usr/bin/env python3
"""Benchmark of the compiled-CUT-graph hot path on one MI355X.

Workload: the batched coflow on the 2n = 40 Majorana-string graph (N = 92,170
strings, E = 39,539,760 records): 64 coefficient sets (mass-scaling sweep) x
(H + 4 quadratic observables) = 320 operand columns, G2 generator, classic RK4
at ds = 5e-3, float-operand graph passes with compensated accumulation, FP64 RK
state, one hipGraph launch per RK step.  A step = one RK4 step of the whole
batch (4 x {generator, graph pass with the fused stage update}).

Printed (one JSON line): contributions x batch / s over the timed steps; the
dominant kernel's roofline (HIP-event average of the fused graph pass; its
algorithmic HBM bytes per launch over that time, against the 8 TB/s HBM peak,
for every precision); the same flow in the other precisions (FP64 at the full
width too); the whole ragged flow counting active columns only; the stress-scale
2n = 64 graph; the plain FP64 one-column flow for the batched / plain ratio;
and the oracle's CPU rate on a bounded sample (cpu_baseline leg).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue rate without packed FP32 instructions (which this library does not
# emit): 256 CUs x 4 SIMDs, one 64-lane instruction every 4 clocks at 2.4 GHz
VALU_INSTS_PER_S = 256 * 4 * 2.4e9 / 4
FP64_VEC_TFLOPS = 78.6
FP64_MFMA_TFLOPS = 78.6   # dense FP64 matrix peak (the vector FP64 peak is the same figure)


def stream_copy_gbs(torch, dev, nbytes=1 << 30, reps=10):
    """Measured device copy rate (bytes read + written per second) of a 1 GiB
    buffer: the practical HBM ceiling the algorithmic and counter rates are
    also compared with."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pass_bytes(N, E, nsets, nops, prec_bytes):
    """Algorithmic HBM bytes of one fused graph pass, averaged over the 4 RK stages.

    records 8 B each; offsets; generator [N, nsets] and stage operand [N, cols]
    read once; per state element the RK epilogue reads z, reads/writes the
    accumulator (stage 0 write, 1-2 read+write, 3 read + z write: 14 B average)
    and writes the next stage operand; the FP64 Hamiltonian column is written.
    """
    cols = nsets * nops
    return (E * 8 + (N + 1) * 8 + N * nsets * prec_bytes + N * cols * prec_bytes
            + N * cols * (8 + 14) + N * cols * prec_bytes + N * nsets * 8)


def pass_kernels(flags: int) -> str:
    """The kernels of one fused flow pass at 64 sets x 5 operands in a tiling."""
    parts = []
    if flags & 16:
        parts.append("k_qblock<5,prec> (quadratic-target blocks)")
    if flags & 2:
        parts.append("k_tile64<5,prec> (shared-triple tiles of the quartic targets)")
    G = 64 >> ((flags >> 5) & 3)   # the B-chunk: lanes per record of the segment kernel
    parts.append(f"k_pass<{G},5,prec,0,2> (" + ("remaining targets" if flags & 18 else "every target") +
                 (", unchunked" if flags & 4 else ", long ones in chunks") + ")")
    if not flags & 4 or flags & 18:
        parts.append("k_chunk_combine<5,prec,2> (partial rows + RK4 stage epilogue)")
    return "fused graph pass with RK4 stage epilogue: " + " + ".join(parts)


KERNEL_SOURCES = ("kernels.hip",)


def kernel_digest() -> str:
    """sha256 over the sources of the segment-pass kernels, in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2609_14831_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def measured_counters(precision: str, what: str = "traffic", prof_name: str = "fused_pass_m40_counters.md"):
    """A per-launch figure of the fused pass from a committed counter summary,
    if it was taken on the current kernel sources (else None).

    The summary carries lines `<what> <precision> <kernel_digest()> <value>`:
    what = traffic (HBM bytes per launch: FETCH_SIZE x copy factor +
    WRITE_SIZE) or valu (SQ_INSTS_VALU per launch).
    """
    prof = os.path.join(ROOT, "profiles", prof_name)
    if not os.path.exists(prof):
        return None
    digest = kernel_digest()
    for line in open(prof):
        parts = line.strip().strip("`").split()
        if len(parts) == 4 and parts[0] == what and parts[1] == precision and parts[2] == digest:
            return float(parts[3])
    return None


def cpu_baseline(inp, w, nsets, nops, budget_s=15.0):
    """Oracle (plain-C FP64 engine, all host threads) on a sample of targets."""
    import numpy as np
    from oracle import algebra as A
    from oracle import gen as OG
    from oracle import native

    reg = A.MajoranaRegistry(w.size)
    stride = 40
    targets = np.arange(0, reg.N, stride)
    ks, is_, js, cs = [], [], [], []
    for t in targets:
        ii, jj, cc = reg.records_for_target(int(t))
        ks.append(np.full(ii.size, t))
        is_.append(ii)
        js.append(jj)
        cs.append(cc)
    g = A.Graph("majorana", w.size, reg.N, np.concatenate(ks), np.concatenate(is_),
                np.concatenate(js), np.concatenate(cs), reg.diag, reg.pairs, -1.0, masks=reg.masks)
    eng = native.Engine(g, "g2", w.delta)
    eta = OG.G2(w.size, w.delta)(inp.z0[:, 0, :])
    x = inp.z0
    eng.apply(eta, x)  # warm
    reps, t0 = 0, time.perf_counter()
    while True:
        eng.apply(eta, x)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= 200:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": g.E * nsets * nops * reps / el, "unit": "contributions*batch/s",
            "cores": threads, "kind": "oracle",
            "sample": f"one graph action (all {nsets * nops} columns, FP64) over the records of every "
                      f"{stride}th target ({targets.size} targets, {g.E} records), {reps} repetitions, "
                      f"{el:.1f} s; plain-C oracle engine with OpenMP"}


def _time_calls(torch, fn, reps):
    """Mean wall time of `reps` stream-ordered calls of fn (after one warm call)."""
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def derivative_leg(L, torch, g, inp, w, prec, E):
    """cut_graph_jvp on the headline workload: 64 sets x 5 operands, both tangents."""
    import numpy as np
    dev = torch.device("cuda:0")
    N, nops, nsets = inp.z0.shape
    cols = nops * nsets
    h = torch.tensor(np.ascontiguousarray(inp.z0[:, 0, :]), device=dev)
    x = torch.tensor(inp.z0.reshape(N, cols), device=dev)
    gen = torch.Generator(device="cpu").manual_seed(5)
    dh = torch.randn((N, nsets), generator=gen, dtype=torch.float64).to(dev)
    dx = torch.randn((N, cols), generator=gen, dtype=torch.float64).to(dev)
    dy = torch.empty((N, cols), dtype=torch.float64, device=dev)
    y = torch.empty_like(dy)

    def jvp():
        L.cut_graph_jvp(g, L.CUT_GEN_G2, w.delta, prec, nsets, nops, h, dh, x, dx, None, dy)

    def jvp_y():
        L.cut_graph_jvp(g, L.CUT_GEN_G2, w.delta, prec, nsets, nops, h, dh, x, dx, y, dy)

    t1 = _time_calls(torch, jvp, 10)
    t2 = _time_calls(torch, jvp_y, 10)
    return {"call": "cut_graph_jvp (dh and dx), 64 sets x 5 operands", "ms": t1 * 1e3,
            "ms_with_action": t2 * 1e3, "passes": 2, "contributions_per_s": 2 * E * cols / t1,
            "unit": "contributions×batch/s"}


def timed_flow(L, torch, g, inp, w, prec, W, K, E, N, tune=True):
    """The headline flow (same sets, steps W .. W+K, hipGraph) in another
    precision, in the tiling the autotuner picks for it; HIP-event average of
    its fused pass from the same steps in stream order."""
    dev = torch.device("cuda:0")
    N_, nops, nsets = inp.z0.shape
    ns = [int(v) for v in inp.n_steps]
    tuning = L.cut_graph_autotune(g, nsets, nops, prec, 0) if tune else None
    z = torch.tensor(inp.z0, device=dev).contiguous()
    p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH, step_begin=0, step_end=W)
    L.cut_flow_integrate(g, p, nsets, nops, ns, z)
    p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH, step_begin=W,
                      step_end=W + K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L.cut_flow_integrate(g, p, nsets, nops, ns, z)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    zt = torch.tensor(inp.z0, device=dev).contiguous()
    p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0, flags=L.CUT_FLOW_TIME_PASSES, step_begin=0,
                      step_end=W + K)
    L.cut_flow_integrate(g, p, nsets, nops, ns, zt)
    tm = L.cut_flow_last_timing(g)
    pass_ms = tm["pass_ms"] / max(1, tm["pass_launches"])
    pb = pass_bytes(N, E, nsets, nops, 8 if prec == L.CUT_F64 else 4)
    name = {L.CUT_F64: "f64", L.CUT_F32C: "f32c", L.CUT_F32X: "f32x", L.CUT_F32: "f32"}[prec]
    traffic = measured_counters(name, "traffic")
    return {"value": 4 * E * nops * nsets * K / wall, "unit": "contributions×batch/s",
            "ms_per_step": wall * 1e3 / K, "pass_ms": pass_ms, "algorithmic_bytes_per_launch": pb,
            "hbm_GBs": pb / (pass_ms * 1e-3) / 1e9, "hbm_frac": pb / (pass_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "traffic": traffic, "traffic_GBs": traffic / (pass_ms * 1e-3) / 1e9 if traffic else None,
            "tiling": tuning}


def ragged_windows_leg(L, torch, g, inp, w, prec, E, all_active_value, steps=10):
    """Windows of `steps` RK4 steps starting late in the config-3 flow, in
    stream order (the state's values do not change the work, only which sets
    are still active); rate over active columns, against the all-active rate of
    the timed steps."""
    dev = torch.device("cuda:0")
    N_, nops, nsets = inp.z0.shape
    ns = [int(v) for v in inp.n_steps]
    L.cut_graph_autotune(g, nsets, nops, prec, 0)
    res = []
    for t0 in (1000, 2000, 2800, 3200, 3500):
        active = sum(sum(1 for n in ns if n > t) for t in range(t0, t0 + steps))
        z = torch.tensor(inp.z0, device=dev).contiguous()
        p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0, flags=0, step_begin=t0, step_end=t0 + 1)
        L.cut_flow_integrate(g, p, nsets, nops, ns, z)
        p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0, flags=0, step_begin=t0, step_end=t0 + steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.cut_flow_integrate(g, p, nsets, nops, ns, z)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        v = 4 * E * nops * active / wall
        res.append({"first_step": t0, "active_sets": sum(1 for n in ns if n > t0), "ms_per_step": wall * 1e3 / steps,
                    "value": v, "ratio_to_all_active": v / all_active_value})
    return res


def full_flow_leg(L, torch, g, inp, w, prec, E, all_active_value):
    """The whole config-3 flow: every set over its own n_b steps (421 ... 3,660),
    hipGraph replays with the passes launched over the active sets only.  The
    rate counts active columns (E x operands x active sets per pass) and is
    compared with the all-active rate of the timed steps."""
    dev = torch.device("cuda:0")
    N_, nops, nsets = inp.z0.shape
    ns = [int(v) for v in inp.n_steps]
    T = max(ns)
    L.cut_graph_autotune(g, nsets, nops, prec, 0)
    z = torch.tensor(inp.z0, device=dev).contiguous()
    p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH, step_end=2)
    L.cut_flow_integrate(g, p, nsets, nops, ns, z)        # captures the step graphs
    z = torch.tensor(inp.z0, device=dev).contiguous()
    p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L.cut_flow_integrate(g, p, nsets, nops, ns, z)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    active = sum(ns) * nops                               # active column-steps
    value = 4 * E * active / wall
    return {"steps": T, "s": wall, "value": value, "unit": "contributions×batch/s (active columns)",
            "active_fraction_of_lane_steps": sum(ns) / (nsets * T),
            "ratio_to_all_active": value / all_active_value}


def stress_leg(L, torch, tmp, profile=False):
    """Stress scale (the 2n = 64 Majorana graph: 637,392 strings, 457,720,704
    records): 16 sets (H only), G2, RK4 at ds = 5e-3, 200 steps; F32C and FP64,
    each in its autotuned tiling, hipGraph replays; the fused pass's
    algorithmic bytes over its HIP-event average against HBM peak."""
    import numpy as np
    import workloads
    dev = torch.device("cuda:0")
    w = workloads.WORKLOADS[4]
    path = os.path.join(tmp, "m64.cgb")
    desc = L.cut_graph_build(L.CUT_ALG_MAJORANA, w.size, path, 0)
    t0 = time.perf_counter()
    g = L.cut_graph_load(path, 0, 0)
    load_s = time.perf_counter() - t0
    os.remove(path)
    N, E = desc["n_ops"], desc["n_records"]
    inp = workloads.make_inputs(4)
    nsets, nops = w.nsets, w.nops
    ns = [int(v) for v in inp.n_steps]
    T = max(ns)
    res = {"graph": f"majorana m={w.size}: N={N}, E={E} records ({E * 8 / 1e9:.2f} GB at 8 B)",
           "compile_s": desc["build_seconds"], "load_s": load_s, "steps": T,
           "sets": nsets, "operands": nops}
    for name, prec in (("f32c", L.CUT_F32C), ("f64", L.CUT_F64)):
        if profile:
            # counter runs: the tiling the autotuner picks for both precisions in
            # unprofiled runs, fixed (counter collection perturbs the timings)
            L.cut_graph_set_tiling(g, 1024, 512, 0)
            tuning = {"long_records": 1024, "chunk_records": 512, "tiling_flags": 0, "autotuned": False}
        else:
            tuning = L.cut_graph_autotune(g, nsets, nops, prec, 0)
        if profile:
            z = torch.tensor(inp.z0, device=dev).contiguous()
            p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0, flags=L.CUT_FLOW_TIME_PASSES, step_end=3)
            L.cut_flow_integrate(g, p, nsets, nops, ns, z)
            res[name] = {"tiling": tuning}
            continue
        z = torch.tensor(inp.z0, device=dev).contiguous()
        p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH, step_end=2)
        L.cut_flow_integrate(g, p, nsets, nops, ns, z)        # capture
        z = torch.tensor(inp.z0, device=dev).contiguous()
        p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.cut_flow_integrate(g, p, nsets, nops, ns, z)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        zt = torch.tensor(inp.z0, device=dev).contiguous()
        p = L.flow_params(L.CUT_GEN_G2, prec, w.ds, w.delta, 0, flags=L.CUT_FLOW_TIME_PASSES, step_end=5)
        L.cut_flow_integrate(g, p, nsets, nops, ns, zt)
        tm = L.cut_flow_last_timing(g)
        pass_ms = tm["pass_ms"] / max(1, tm["pass_launches"])
        pb = pass_bytes(N, E, nsets, nops, 8 if prec == L.CUT_F64 else 4)
        res[name] = {"s_200_steps": wall, "ms_per_step": wall * 1e3 / T,
                     "value": 4 * E * nsets * nops * T / wall, "unit": "contributions×batch/s",
                     "pass_ms": pass_ms, "algorithmic_bytes_per_launch": pb,
                     "hbm_GBs": pb / (pass_ms * 1e-3) / 1e9,
                     "hbm_frac": pb / (pass_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "record_stream_GBs": E * 8 / (pass_ms * 1e-3) / 1e9, "tiling": tuning}
        del z, zt
    L.cut_graph_free(g)
    return res


def reverse_flow_leg(L, torch, tmp):
    """The differentiated flow of config 5 (2n = 24 graph, 8 sets, H only,
    G2, ds = 5e-3 to s = 10: 2,000 RK4 steps): the forward flow with a
    checkpoint every 16 steps, then the discrete adjoint of the whole flow
    (each checkpoint block recomputed in FP64 with its stage states kept, four
    transposed graph passes per RK stage).  Both in FP64, timed separately."""
    import workloads
    dev = torch.device("cuda:0")
    w = workloads.WORKLOADS[5]
    path = os.path.join(tmp, "m24.cgb")
    desc = L.cut_graph_build(L.CUT_ALG_MAJORANA, w.size, path, 0)
    g = L.cut_graph_load(path, 0, L.CUT_LOAD_ADJOINT)
    os.remove(path)
    N, E = desc["n_ops"], desc["n_records"]
    inp = workloads.make_inputs(5)
    nsets, nops, C = w.nsets, w.nops, w.ckpt_every
    ns = [int(v) for v in inp.n_steps]
    T = max(ns)
    ck = torch.zeros(((T + C - 1) // C, N, nops, nsets), dtype=torch.float64, device=dev)
    L.cut_graph_reserve(g, nsets, nops, C, L.CUT_RESERVE_FLOW | L.CUT_RESERVE_ADJOINT)
    res = {"workload": f"majorana m={w.size} (N={N}, E={E}), {nsets} sets, H only, {T} RK4 steps, "
                       f"checkpoints every {C} steps, FP64"}
    for rep in range(2):   # the first round captures the step graph and warms up
        z = torch.tensor(inp.z0, device=dev).contiguous()
        p = L.flow_params(L.CUT_GEN_G2, L.CUT_F64, w.ds, w.delta, C)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.cut_flow_integrate(g, p, nsets, nops, ns, z, ck)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lam = torch.zeros_like(z)
        lam[torch.tensor(workloads_pairs(w.size), device=dev), 0, :] = 1.0
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        L.cut_flow_adjoint(g, p, nsets, nops, ns, ck, lam)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
    fwd_pass = 4 * T * E * nops * nsets
    res.update({"forward_s": t1 - t0, "adjoint_s": t3 - t2, "adjoint_over_forward": (t3 - t2) / (t1 - t0),
                "forward_contributions_per_s": fwd_pass / (t1 - t0),
                "adjoint_note": "per step: the block's forward recompute (4 passes) + 4 stages x "
                                "(generator, j-grouped and i-grouped passes, generator VJP)"})
    L.cut_graph_free(g)
    return res


def workloads_pairs(m):
    """Registry rows of the pair strings {2a, 2a+1} (2-subsets come first,
    lexicographic): the rows the config-5 loss sums."""
    rows, r = [], 0
    for i in range(m):
        for j in range(i + 1, m):
            if j == i + 1 and i % 2 == 0:
                rows.append(r)
            r += 1
    return rows


def assembly_leg(L, torch, N):
    """Multi-operator assembly (Sec. 3.4): 1024 output combinations of a
    120-operator transformed library over N registry rows, FP64 on the matrix
    cores; torch's FP64 matmul (the vendor BLAS) on the same operands as a
    reference point."""
    dev = torch.device("cuda:0")
    S, K = 120, 1024
    gen = torch.Generator(device="cpu").manual_seed(11)
    X = torch.randn((N, S), generator=gen, dtype=torch.float64).to(dev)
    W = torch.randn((S, K), generator=gen, dtype=torch.float64).to(dev)
    Y = torch.empty((N, K), dtype=torch.float64, device=dev)
    t = _time_calls(torch, lambda: L.cut_assemble(X, W, Y), 20)
    tb = _time_calls(torch, lambda: torch.matmul(X, W, out=Y), 20)
    flops = 2.0 * N * S * K
    return {"shape": f"Y[{N}, {K}] = X[{N}, {S}] W[{S}, {K}], FP64", "ms": t * 1e3,
            "tflops": flops / t / 1e12, "peak_tflops": FP64_MFMA_TFLOPS,
            "frac": flops / t / 1e12 / FP64_MFMA_TFLOPS, "vendor_blas_ms": tb * 1e3,
            "bytes_min": 8 * (N * S + S * K + N * K)}


def pauli_boson_leg(L, torch, tmp):
    """The paper's own algebra at its benchmark size (Sec. 3.2-3.3): five boson
    modes, complete degree-four Pauli-boson registry (4,004 labels), generator
    and retained flow 7,017,036 records, outside space 345,388,180 records.
    FP64 on complex coefficients (real-split rows), Wegner block generator,
    a batch of eight operators (the Hamiltonian and seven Hermitian operators):
    one retained-flow action (generator + retained pass), the same with the
    outside-space action, and a 100-step RK4 flow without and with the
    outside-space diagnostic at every right-hand side."""
    import numpy as np
    import workloads
    dev = torch.device("cuda:0")
    M, p = 5, 4
    path = os.path.join(tmp, "pb5.cgb")
    t0 = time.perf_counter()
    desc = L.cut_graph_build(L.CUT_ALG_PAULI_BOSON, 256 * M + p, path, 0, L.CUT_BUILD_OUTSIDE)
    build_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    g = L.cut_graph_load(path, 0, 0)
    load_s = time.perf_counter() - t0
    os.remove(path)
    N, NG, Nc = desc["n_ops"], desc["n_gen_ops"], desc["n_out_ops"]
    W = (3 * p).bit_length()
    labels = [workloads.pb_label(int(k), M, W) for k in L.cut_graph_labels(g, 0)]
    rng = np.random.default_rng([260914831, 55])
    nops, nsets = 8, 1
    # H with small off-diagonal parts (the projected flow of a complete boson
    # registry is stiff), seven Hermitian operators with O(1) coefficients
    z0 = np.stack([workloads.pb_hermitian(labels, rng, 1.0, 0.02 if o == 0 else 1.0) for o in range(nops)], 1)
    z0 = workloads.real_split(z0)[:, :, None]                                 # [2N, 8, 1]
    x = torch.tensor(z0.reshape(2 * N, nops), device=dev)
    h = x[:, :1].contiguous()
    eta = torch.empty((2 * NG, 1), dtype=torch.float64, device=dev)
    y = torch.empty((2 * N, nops), dtype=torch.float64, device=dev)
    yc = torch.empty((2 * Nc, nops), dtype=torch.float64, device=dev)

    def retained():
        L.cut_generator(g, L.CUT_GEN_WEGNER_GRAPH, 0.0, nsets, h, eta)
        L.cut_graph_apply(g, L.CUT_GRAPH_FLOW, L.CUT_F64, nsets, nops, eta, x, y)

    def diagnostic():
        retained()
        L.cut_graph_apply(g, L.CUT_GRAPH_OUTSIDE, L.CUT_F64, nsets, nops, eta, x, yc)

    t_ret = _time_calls(torch, retained, 20)
    t_diag = _time_calls(torch, diagnostic, 5)
    ds, steps = 1e-3, 100

    def flow(with_diag):
        z = torch.tensor(z0, device=dev).contiguous()
        leak = torch.zeros(nops * nsets, dtype=torch.float64, device=dev) if with_diag else None
        prm = L.flow_params(L.CUT_GEN_WEGNER_GRAPH, L.CUT_F64, ds, 0.0, 0, outside_norm2=leak)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.cut_flow_integrate(g, prm, nsets, nops, [steps], z)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, z

    try:
        flow(False)                       # capture the step graph once
        t_flow, z_plain = flow(False)
        t_flow_d, z_diag = flow(True)
        same = bool(torch.equal(z_plain, z_diag))
    except L.CutError as e:               # reported, not hidden: the leg records the failure
        t_flow = t_flow_d = None
        same = None
        log(f"pauli-boson flow failed: {e}")
    L.cut_graph_free(g)
    return {"graph": f"pauli-boson M={M} p={p}: {N} labels, generator registry {NG}, outside registry {Nc}; "
                     f"E_eta {desc['n_gen_records']} + E_L {desc['n_records']} = "
                     f"{desc['n_gen_records'] + desc['n_records']} production records, "
                     f"E_C {desc['n_out_records']} outside-space records",
            "compile_s": build_s, "load_s": load_s, "bundle_bytes": desc["file_bytes"],
            "batch": "8 operators (H + 7), FP64 complex (real-split vectors, complex-record passes), Wegner block generator",
            "retained_action_ms": t_ret * 1e3, "action_with_outside_ms": t_diag * 1e3,
            "flow_100_steps_s": t_flow, "flow_100_steps_with_outside_s": t_flow_d,
            "trajectory_unchanged_by_diagnostic": same,
            "paper_h100": {"retained_action_ms": 0.632, "action_with_outside_ms": 48.439,
                           "flow_100_steps_s": 0.498, "flow_100_steps_with_outside_s": 22.216}}


def outside_leg(L, torch, tmp):
    """The outside-space action C_q (Eq. graph-actions, third line) on the
    m = 32 Majorana graph: 906,192 outside targets, 471.2M records (the scale of
    the paper's diagnostic-enabled stress graph); one FP64 column (a single
    action) and 8 sets x 3 operands in the compensated float mode."""
    dev = torch.device("cuda:0")
    m = 32
    path = os.path.join(tmp, "m32_outside.cgb")
    t0 = time.perf_counter()
    desc = L.cut_graph_build(L.CUT_ALG_MAJORANA, m, path, 0, L.CUT_BUILD_OUTSIDE)
    build_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    g = L.cut_graph_load(path, 0, 0)
    load_s = time.perf_counter() - t0
    N, Nc, Ec = desc["n_ops"], desc["n_out_ops"], desc["n_out_records"]
    res = {"graph": f"majorana m={m}: N={N}, outside targets {Nc}, E_C={Ec} records, "
                    f"E_L={desc['n_records']} records",
           "compile_s": build_s, "load_s": load_s, "bundle_bytes": desc["file_bytes"]}
    gen = torch.Generator(device="cpu").manual_seed(7)
    for name, prec, nsets, nops in (("f64_one_column", L.CUT_F64, 1, 1), ("f32c_8x3", L.CUT_F32C, 8, 3)):
        dt = torch.float64 if prec == L.CUT_F64 else torch.float32
        eta = torch.randn((N, nsets), generator=gen, dtype=torch.float64).to(dev).to(dt)
        x = torch.randn((N, nsets * nops), generator=gen, dtype=torch.float64).to(dev).to(dt)
        y = torch.empty((Nc, nsets * nops), dtype=torch.float64, device=dev)

        def call():
            L.cut_graph_apply(g, L.CUT_GRAPH_OUTSIDE, prec, nsets, nops, eta, x, y)

        ts = _time_calls(torch, call, 10)
        stream_bytes = 8 * Ec + 8 * (Nc + 1) + 8 * Nc * nsets * nops   # records, offsets, output
        res[name] = {"ms": ts * 1e3, "records_per_s": Ec / ts,
                     "contributions_per_s": Ec * nsets * nops / ts,
                     "stream_GBs": stream_bytes / ts / 1e9}
        del eta, x, y
    L.cut_graph_free(g)
    os.remove(path)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="f32c", choices=["f32c", "f32x", "f64", "f32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-outside", action="store_true", help="skip the outside-space action leg")
    ap.add_argument("--no-stress", action="store_true", help="skip the 2n = 64 stress-scale leg")
    ap.add_argument("--no-full-flow", action="store_true",
                    help="skip the whole ragged flow (3,660 steps, about 30 s)")
    ap.add_argument("--only", choices=["assembly", "outside", "pauli_boson", "stress"],
                    help="run only that leg and print its JSON (for profiling)")
    ap.add_argument("--minimal", action="store_true", help="timed flow only")
    ap.add_argument("--profile", action="store_true",
                    help="counter runs: a 1 GiB device copy (calibration), then the steps in "
                         "stream order (no hipGraph), nothing else")
    ap.add_argument("--plain", action="store_true",
                    help="with --profile: the plain FP64 flow, one operand column (one set, H only)")
    ap.add_argument("--long-records", type=int, default=0,
                    help="fixed tiling (long-target threshold); 0 = autotune")
    ap.add_argument("--chunk-records", type=int, default=512, help="chunk length with --long-records")
    ap.add_argument("--tiling-flags", type=int, default=0, help="CUT_TILE_* flags with --long-records")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding the coefficient sets "
              "across GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2609_14831_amd import _lib as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    w = workloads.WORKLOADS[3]
    if args.only == "assembly":
        import math
        n40 = math.comb(w.size, 2) + math.comb(w.size, 4)     # registry rows of the m = 40 graph
        print(json.dumps({"assembly": assembly_leg(L, torch, n40)}), flush=True)
        return
    if args.only == "pauli_boson":
        print(json.dumps({"pauli_boson": pauli_boson_leg(L, torch, tempfile.mkdtemp(prefix="cutgraph_bench_"))}),
              flush=True)
        return
    if args.only == "stress":
        print(json.dumps({"stress_m64": stress_leg(L, torch, tempfile.mkdtemp(prefix="cutgraph_bench_"),
                                                   profile=args.profile)}), flush=True)
        return
    if args.only == "outside":
        print(json.dumps({"outside_space": outside_leg(L, torch, tempfile.mkdtemp(prefix="cutgraph_bench_"))}),
              flush=True)
        return
    PREC = {"f32c": L.CUT_F32C, "f32x": L.CUT_F32X, "f64": L.CUT_F64, "f32": L.CUT_F32}[args.precision]
    pbytes = 8 if PREC == L.CUT_F64 else 4

    tmp = tempfile.mkdtemp(prefix="cutgraph_bench_")
    path = os.path.join(tmp, "m40.cgb")
    desc = L.cut_graph_build(L.CUT_ALG_MAJORANA, w.size, path, 0)
    log(f"compiled m={w.size}: N={desc['n_ops']} E={desc['n_records']} in {desc['build_seconds']:.2f} s")
    t0 = time.perf_counter()
    g = L.cut_graph_load(path, 0, 0)
    load_s = time.perf_counter() - t0
    if args.long_records > 0:
        L.cut_graph_set_tiling(g, args.long_records, args.chunk_records, args.tiling_flags)
        tuning = {"long_records": args.long_records, "chunk_records": args.chunk_records,
                  "tiling_flags": args.tiling_flags, "autotuned": False}
    else:
        t0 = time.perf_counter()
        tuning = L.cut_graph_autotune(g, w.nsets, w.nops, PREC, 0)
        tuning["autotune_s"] = time.perf_counter() - t0
        tuning["autotuned"] = True
        log(f"autotuned: {tuning}")
    N, E = desc["n_ops"], desc["n_records"]

    inp = workloads.make_inputs(3)
    nsets, nops = w.nsets, w.nops
    ns = [int(v) for v in inp.n_steps]
    z = torch.tensor(inp.z0, device=dev).contiguous()
    W, K = args.warmup, args.steps
    assert W + K <= min(ns), "timed steps must keep every set active"
    if args.profile:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        if args.plain:
            nsets, nops, ns = 1, 1, [ns[0]]
            z = torch.tensor(inp.z0[:, :1, :1], device=dev).contiguous()
        p = L.flow_params(L.CUT_GEN_G2, PREC, w.ds, w.delta, 0, flags=L.CUT_FLOW_TIME_PASSES,
                          step_begin=0, step_end=W + K)
        L.cut_flow_integrate(g, p, nsets, nops, ns, z)
        tm = L.cut_flow_last_timing(g)
        print(json.dumps({"profile": True, "copy_bytes_each_way": 1 << 30, "steps": W + K,
                          "sets": nsets, "operands": nops,
                          "pass_avg_ms": tm["pass_ms"] / max(1, tm["pass_launches"]),
                          "pass_bytes": pass_bytes(N, E, nsets, nops, pbytes)}), flush=True)
        return

    p = L.flow_params(L.CUT_GEN_G2, PREC, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH,
                      step_begin=0, step_end=W)
    L.cut_flow_integrate(g, p, nsets, nops, ns, z)
    torch.cuda.synchronize()
    log(f"warmup {W} steps done")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    p = L.flow_params(L.CUT_GEN_G2, PREC, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH,
                      step_begin=W, step_end=W + K)
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    L.cut_flow_integrate(g, p, nsets, nops, ns, z)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    e1.record(stream)
    torch.cuda.synchronize()
    active_cols = sum(nops * sum(1 for n in ns if n > t) for t in range(W, W + K))
    contributions = 4 * E * active_cols
    value = contributions / wall
    log(f"timed {K} steps: {wall * 1e3 / K:.3f} ms/step, {value:.3e} contributions*batch/s")
    out = {"metric": "graph contributions×batch/s + HBM GB/s; batched FP32 vs plain FP64 flow",
           "value": value, "unit": "contributions×batch/s", "n_gpus": 1, "steps": K, "warmup": W,
           "ms_per_step": wall * 1e3 / K, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if PREC != L.CUT_F64 else "f64",
           "data": "synthetic (seeded mass-scaling sweep, no dataset)",
           "config": {"workload": f"majorana_m40_batched: 2n=40 Majorana strings, N={N}, E={E} records, "
                                  f"{nsets} sets x {nops} operands = {nsets * nops} columns, ragged "
                                  f"s_max in [2,20], ds={w.ds}, G2 generator (delta={w.delta}), RK4, "
                                  f"one hipGraph per step",
                      "precision": {"f32c": "float operands and products, compensated (two-product + "
                                            "two-sum) accumulation, FP64 result and RK state",
                                    "f32x": "float operands, products and sums in FP64, FP64 RK state",
                                    "f64": "FP64 throughout", "f32": "plain float sums"}[args.precision],
                      "graph_compile_s": desc["build_seconds"], "graph_load_s": load_s,
                      "tiling": tuning}}
    if args.minimal:
        print(json.dumps(out), flush=True)
        return

    # kernel timing leg: same steps in stream order, HIP events around each pass
    zt = torch.tensor(inp.z0, device=dev).contiguous()
    p = L.flow_params(L.CUT_GEN_G2, PREC, w.ds, w.delta, 0, flags=L.CUT_FLOW_TIME_PASSES,
                      step_begin=0, step_end=W + K)
    L.cut_flow_integrate(g, p, nsets, nops, ns, zt)
    tm = L.cut_flow_last_timing(g)
    pass_ms = tm["pass_ms"] / max(1, tm["pass_launches"])
    gen_ms = tm["gen_ms"] / max(1, tm["gen_launches"])
    bytes_per = pass_bytes(N, E, nsets, nops, pbytes)
    achieved = bytes_per / (pass_ms * 1e-3) / 1e9
    flops_per = 2.0 * E * nsets * nops
    log(f"fused pass avg {pass_ms:.4f} ms ({tm['pass_launches']} launches), generator {gen_ms:.4f} ms")
    traffic = measured_counters(args.precision, "traffic")
    valu = measured_counters(args.precision, "valu")
    gathered = E * (nsets + nops * nsets) * pbytes   # one eta row + one operand row per record
    terms = E * nsets * nops                          # contributions x columns of one pass
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS,
                       "traffic": traffic,
                       "traffic_unit": "HBM bytes per fused pass (FETCH_SIZE x copy factor + WRITE_SIZE)",
                       "kernel": pass_kernels(tuning["tiling_flags"]),
                       "avg_launch_ms": pass_ms, "algorithmic_bytes_per_launch": bytes_per,
                       "gathered_row_bytes_per_launch": gathered,
                       "gathered_row_rate_GBs": gathered / (pass_ms * 1e-3) / 1e9,
                       "fp64_equiv_tflops": flops_per / (pass_ms * 1e-3) / 1e12,
                       "fp64_vector_peak_tflops": FP64_VEC_TFLOPS}
    if valu:
        # diagnostic: VALU instructions per contribution x column and the share
        # of the SIMDs' issue cycles they fill (counters in profiles/)
        out["roofline"]["valu_diagnostic"] = {
            "insts_per_launch": valu, "per_term": valu * 64 / terms,
            "issue_frac": valu / (pass_ms * 1e-3) / VALU_INSTS_PER_S}
    out["generator_avg_ms"] = gen_ms
    copy_gbs = stream_copy_gbs(torch, dev)
    rl = out["roofline"]
    rl["stream_copy_GBs"] = copy_gbs
    rl["hbm_frac_of_copy"] = achieved / copy_gbs
    if traffic:
        rl["traffic_GBs"] = traffic / (pass_ms * 1e-3) / 1e9
        rl["traffic_frac_of_copy"] = rl["traffic_GBs"] / copy_gbs

    # the other compensated float mode on the same workload (same steps)
    alt = {"f32c": "f32x", "f32x": "f32c"}.get(args.precision)
    if alt:
        PALT = {"f32c": L.CUT_F32C, "f32x": L.CUT_F32X}[alt]
        alt_tuning = L.cut_graph_autotune(g, w.nsets, w.nops, PALT, 0) if args.long_records <= 0 else None
        za = torch.tensor(inp.z0, device=dev).contiguous()
        p = L.flow_params(L.CUT_GEN_G2, PALT, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH,
                          step_begin=0, step_end=W)
        L.cut_flow_integrate(g, p, nsets, nops, ns, za)
        p = L.flow_params(L.CUT_GEN_G2, PALT, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH,
                          step_begin=W, step_end=W + K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.cut_flow_integrate(g, p, nsets, nops, ns, za)
        torch.cuda.synchronize()
        alt_wall = time.perf_counter() - t0
        out["alt_precision"] = {"precision": alt, "value": contributions / alt_wall,
                                "ms_per_step": alt_wall * 1e3 / K, "tiling": alt_tuning}
        log(f"{alt}: {alt_wall * 1e3 / K:.3f} ms/step")
        del za

    # the same flow with FP64 passes at the full width (64 sets x 5 operands)
    out["batched_fp64"] = timed_flow(L, torch, g, inp, w, L.CUT_F64, W, K, E, N, tune=args.long_records <= 0)
    log(f"batched fp64: {out['batched_fp64']}")
    # ragged batch: windows late in the flow, where fewer sets are active,
    # counting active columns only (stream order, every window's passes
    # launched over the active prefix), then the whole flow
    out["ragged_windows"] = ragged_windows_leg(L, torch, g, inp, w, PREC, E, value)
    log(f"ragged windows: {out['ragged_windows']}")
    if not args.no_full_flow:
        out["full_ragged_flow"] = full_flow_leg(L, torch, g, inp, w, PREC, E, value)
        log(f"full ragged flow: {out['full_ragged_flow']}")

    # plain FP64 flow, one operand column per pass (one set, H only), in the
    # tiling tuned for that shape
    out["plain_fp64_flow_tiling"] = L.cut_graph_autotune(g, 1, 1, L.CUT_F64, 0)
    z1 = torch.tensor(inp.z0[:, :1, :1], device=dev).contiguous()
    ns1 = [ns[0]]
    p = L.flow_params(L.CUT_GEN_G2, L.CUT_F64, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH,
                      step_begin=0, step_end=W)
    L.cut_flow_integrate(g, p, 1, 1, ns1, z1)
    p = L.flow_params(L.CUT_GEN_G2, L.CUT_F64, w.ds, w.delta, 0, flags=L.CUT_FLOW_HIPGRAPH,
                      step_begin=W, step_end=W + K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L.cut_flow_integrate(g, p, 1, 1, ns1, z1)
    torch.cuda.synchronize()
    plain = 4 * E * K / (time.perf_counter() - t0)
    z1 = torch.tensor(inp.z0[:, :1, :1], device=dev).contiguous()
    p = L.flow_params(L.CUT_GEN_G2, L.CUT_F64, w.ds, w.delta, 0, flags=L.CUT_FLOW_TIME_PASSES,
                      step_begin=0, step_end=W + K)
    L.cut_flow_integrate(g, p, 1, 1, ns1, z1)
    tm1 = L.cut_flow_last_timing(g)
    plain_ms = tm1["pass_ms"] / max(1, tm1["pass_launches"])
    pb1 = pass_bytes(N, E, 1, 1, 8)
    tr1 = measured_counters("plain", "traffic")
    out["plain_fp64_flow"] = {"value": plain, "unit": "contributions×batch/s",
                              "columns": 1, "ratio_batched_over_plain": value / plain,
                              "pass_ms": plain_ms, "algorithmic_bytes_per_launch": pb1,
                              "hbm_GBs": pb1 / (plain_ms * 1e-3) / 1e9,
                              "hbm_frac": pb1 / (plain_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "traffic": tr1}
    log(f"plain FP64 one-column flow {plain:.3e}/s; batched/plain = {value / plain:.1f}x")
    # directional derivative of one action at the headline shape (Sec. 2.4,
    # Eq. directional-derivative): generator + its JVP + two forward passes
    t = L.cut_graph_autotune(g, w.nsets, w.nops, PREC, 0) if args.long_records <= 0 else None
    if t is not None:
        L.cut_graph_set_tiling(g, t["long_records"], t["chunk_records"], t["tiling_flags"])
    out["derivative"] = derivative_leg(L, torch, g, inp, w, PREC, E)
    log(f"jvp: {out['derivative']}")
    L.cut_graph_free(g)
    os.remove(path)

    out["assembly"] = assembly_leg(L, torch, N)
    log(f"assembly: {out['assembly']}")
    out["reverse_flow"] = reverse_flow_leg(L, torch, tmp)
    log(f"reverse flow: {out['reverse_flow']}")

    if not args.no_stress:
        out["stress_m64"] = stress_leg(L, torch, tmp)
        log(f"stress-scale m=64: {out['stress_m64']}")

    if not args.no_outside:
        out["outside_space"] = outside_leg(L, torch, tmp)
        log(f"outside-space action: {out['outside_space']}")
        out["pauli_boson"] = pauli_boson_leg(L, torch, tmp)
        log(f"pauli-boson five-mode graph: {out['pauli_boson']}")

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inp, w, nsets, nops)
        log(f"cpu baseline {out['cpu_baseline']['value']:.3e}/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
