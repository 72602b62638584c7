#!/usr/bin/env python3
"""Throughput of the AFC hot path on one MI355X.

Workload: the stationary monolithic-convex-limiter (MCL) problem on Q1
128^3 (2,146,689 nodes, 57,066,625 nonzeros): eps = 1e-6, b = (1,1,1)/sqrt(3),
c = 1, f = 1 on [0.25, 0.5]^3, u = 0 on the boundary.  One step is one
fixed-point iteration of the paper's scheme (Sec. 4): MCL bounds, limited
fluxes and the FP64 nonlinear residual, then the linear solve of the
low-order matrix to ||b - A x|| <= 1e-10 ||b|| with GMRES(30)-Jacobi, FP32
Arnoldi (s-step blocks of 15 basis vectors unless --sstep says otherwise)
inside FP64 iterative refinement.  Steps continue from the low-order
solution (computed before timing).  value = nodes x steps / seconds
(DOF-iterations/s).

Also reported: the rate with one basis vector per Arnoldi step, the
plain-FP64 GMRES rate, Krylov iterations per step, the
roofline of the dominant kernel (FP32 SELL-64 SpMV) from HIP-event timings
taken live in this process, batched CN-FCT solves/s (one persistent launch
for 256 instances, against one-at-a-time solves), serving solves/s with
p50/p99 latency, and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sell_spmv32_q1_128_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2110_15676_amd", "csrc", "afc_kernels.hip")


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def spmv32_bytes(N, info):
    """Algorithmic bytes of one FP32 SELL-64 SpMV (`info`: the Krylov layout,
    the pattern without its diagonal): the FP32 value of every slot, the
    per-row column offsets of non-uniform slices, the shared offset patterns,
    two 32-bit slice headers per slice, one read of x, one write of y."""
    return (4 * info["slots"] + info["delta_bytes"] * info["lane_delta_slots"] + 4 * info["pattern_ints"]
            + 4 * (info["slices"] + 1) + 4 * info["slices"] + 4 * N + 4 * N)


def step_model_bytes(N, info, kinfo, krylov, sweeps, steps, sstep=0):
    """Algorithmic HBM bytes of `steps` fixed-point iterations (model: every
    cycle of equal length, Arnoldi index k uniform over the cycle).  `info`:
    the system layout (FP64 residual, MCL passes), `kinfo`: the FP32 Krylov
    layout.  With s-step blocks the projections and the update read the old
    basis once per block of `sstep` vectors."""
    L = krylov / max(sweeps, 1)  # mean FP32 GMRES cycle length
    kbar = (L - 1) / 2.0         # mean Arnoldi index inside a cycle
    if sstep > 0:
        kb = max(0.0, (L - sstep) / 2.0)  # mean block start
        per_it = spmv32_bytes(N, kinfo) + ((kb + 1) / sstep + 1) * 4 * N + ((kb + 1) / sstep + 2) * 4 * N
    else:
        # SpMV, projections (V[0..k] and W) and the update
        per_it = spmv32_bytes(N, kinfo) + (kbar + 2) * 4 * N + (kbar + 3) * 4 * N
    index = info["delta_bytes"] * info["lane_delta_slots"] + 4 * info["pattern_ints"] + 8 * info["slices"] + 4
    residual = 8 * info["slots"] + index + 24 * N
    per_sweep = residual + kbar * 4 * N + 16 * N + 12 * N
    # MCL bounds (slot masks, u, u^max, u^min) and flux pass (A_low, c_ij, c_ji slots + node vectors)
    per_fp = (index + 4 * N + 24 * N) + (index + 24 * info["slots"] + 4 * N + 57 * N)
    return krylov * per_it + sweeps * per_sweep + steps * per_fp


def _oracle_first_iteration(n):
    """The oracle's first fixed-point iteration of the MCL workload on Q1 n^3
    from its low-order solution (one thread).  Returns (nodes, seconds,
    Krylov iterations, seconds of the untimed low-order solve)."""
    from threadpoolctl import threadpool_limits

    from oracle import afc_oracle as O
    from paper_2110_15676_amd import inputs as I

    inst = I.config3(n)

    def progress(it, res):  # one line per GMRES cycle of the oracle
        print("bench: oracle GMRES at %d iterations, residual %.3e" % (it, res), file=sys.stderr, flush=True)

    O.PROGRESS = progress
    with threadpool_limits(1):
        P = O.problem_from_instance(inst, conv=True)
        t = time.perf_counter()
        lo = O.low_order_solution(P, inst.F, lin_rtol=1e-10)
        t_lo = time.perf_counter() - t
        t = time.perf_counter()
        _, st = O.stationary_mcl(P, inst.F, lo.x, tol=0.0, tol_mode="rel", maxit=1, lin_rtol=1e-10)
        el = time.perf_counter() - t
    O.PROGRESS = None
    return inst.N, el, int(sum(st.krylov_iters)), t_lo


def _oracle_cn_instance(k):
    """20 CN-FCT steps of batch instance k with the oracle (one process per
    instance, one thread), at the batch's tolerances."""
    from threadpoolctl import threadpool_limits

    from oracle import afc_oracle as O
    from paper_2110_15676_amd import inputs as I

    with threadpool_limits(1):
        inst = I.config4_instance(I.config4_params(k + 1)[k])
        P = O.problem_from_instance(inst, conv=False)
        u = inst.u0.copy()
        t = time.perf_counter()
        for _ in range(20):
            u, _ = O.cn_fct_step(P, u, inst.F, inst.F, 1e-3, tol=1e-12, tol_mode="abs", maxit=50,
                                 lin="bicgstab", lin_atol=1e-12)
        return inst.N, time.perf_counter() - t


def gpu_first_iteration(afc, torch, I, n, sstep):
    """The GPU on the oracle's sample: the first fixed-point iteration of the
    MCL workload on Q1 n^3 from its low-order solution, with the bench's
    mixed-precision solver and with plain FP64 GMRES (the oracle's
    arithmetic)."""
    inst = I.config3(n)
    out = {"nodes": inst.N}
    for name, prec, ss in (("mixed", afc.AFC_PREC_MIXED, sstep), ("fp64", afc.AFC_PREC_FP64, sstep),
                           ("fp64_one_vector", afc.AFC_PREC_FP64, 0)):
        o = afc.afc_default_options(precision=prec, krylov=afc.AFC_KRYLOV_GMRES, restart=30, fp_tol=0.0,
                                    fp_tol_mode=afc.AFC_TOL_REL, fp_maxit=0, lin_atol=0.0, lin_rtol=1e-10,
                                    lin_maxit=100000, sstep=ss)
        o.stream = torch.cuda.current_stream().cuda_stream
        h = afc.afc_create_instance(inst, o, conv=True)
        try:
            u = torch.zeros(inst.N, dtype=torch.float64, device="cuda:0")
            F = torch.tensor(inst.F, device="cuda:0")
            afc.afc_solve_stationary(h, u, F, init_low_order=True)
            o.fp_maxit = 1
            afc.afc_set_options(h, o)
            u1 = u.clone()
            afc.afc_solve_stationary(h, u1, F)  # warm-up (graphs, coefficient layouts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, s = afc.afc_solve_stationary(h, u, F)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        finally:
            afc.afc_destroy(h)
        out[name] = {"seconds": el, "krylov_iters": s["krylov_iters"], "dof_its_per_s": inst.N / el,
                     "dof_krylov_its_per_s": inst.N * s["krylov_iters"] / el}
    return out


def host_cores():
    """Host cores this process may use (affinity), at most the 16 of a one-GPU
    share."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(n, gpu_sample, batch_sample):
    """The FP64 oracle on bounded samples of the workloads, on the host cores.
    (1) The first fixed-point iteration of the MCL workload on Q1 n^3 from its
    low-order solution, one thread, beside the GPU's time for the same
    iteration (`gpu_sample`).  (2) Every 8th of the 256 batched CN-FCT
    instances, 20 steps each, one process per instance over the host cores."""
    import multiprocessing as mp

    N, el, kr, t_lo = _oracle_first_iteration(n)
    out = {
        "value": N / el,
        "unit": "DOF-iterations/s",
        "cores": 1,
        "host_cores": host_cores(),
        "nproc": os.cpu_count(),
        "kind": "oracle",
        "sample": "first fixed-point iteration of the same MCL problem on Q1 %d^3 (%d nodes) from its low-order "
                  "solution: %d GMRES(30)-Jacobi iterations to 1e-10 ||b||, numpy FP64, one thread; %.1f s "
                  "(low-order start %.1f s, not timed)" % (n, N, kr, el, t_lo),
        "krylov_iters": kr,
        "dof_krylov_its_per_s": N * kr / el,
        "gpu_same_sample": gpu_sample,
    }
    if batch_sample:
        ids = list(range(0, 256, 8))
        workers = host_cores()
        ctx = mp.get_context("spawn")
        t = time.perf_counter()
        with ctx.Pool(workers) as pool:
            res = pool.map(_oracle_cn_instance, ids, chunksize=1)
        wall = time.perf_counter() - t
        out["batch_oracle"] = {
            "solves_per_s": len(ids) / wall, "seconds": wall, "processes": workers,
            "sample": "every 8th of the 256 batched CN-FCT instances (%d instances, %d nodes), 20 steps each, "
                      "one process per instance, numpy FP64" % (len(ids), sum(r[0] for r in res)),
            "cpu_seconds": sum(r[1] for r in res),
        }
    return out


def solve_to_tolerance(afc, torch, inst, make_opts, rel_tol, cap, lin_eta=0.0, dynamic_damping=1, label=""):
    """The stationary problem solved to its own stopping rule, R <= rel_tol R_0
    (R_0: the nonlinear residual at the low-order start), as a user runs it:
    the low-order solve, then one afc_solve_stationary call that iterates
    until the rule holds or `cap` iterations have run.  The residual curve
    comes from the library's residual history of that call.  Returns counts,
    seconds and the curve (R / R_0 every 10 iterations)."""
    N = inst.N
    dev = torch.device("cuda:0")
    h = afc.afc_create_instance(inst, make_opts(fp_maxit=0, lin_eta=lin_eta), conv=True)
    try:
        u = torch.zeros(N, dtype=torch.float64, device=dev)
        F = torch.tensor(inst.F, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, s0 = afc.afc_solve_stationary(h, u, F, init_low_order=True, raise_on_error=False)
        torch.cuda.synchronize()
        t_low = time.perf_counter() - t0
        afc.afc_set_options(h, make_opts(fp_maxit=cap, fp_tol=rel_tol, fp_tol_mode=afc.AFC_TOL_REL,
                                         lin_eta=lin_eta, dynamic_damping=dynamic_damping))
        print("bench: %s solve to R <= %g R0 (cap %d)" % (label, rel_tol, cap), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, s = afc.afc_solve_stationary(h, u, F, raise_on_error=False)
        torch.cuda.synchronize()
        t_fp = time.perf_counter() - t0
        hist = afc.afc_residual_history(h)
        x_min, x_max = float(u.min()), float(u.max())
    finally:
        afc.afc_destroy(h)
    R0 = float(hist[0])
    rel = hist / R0
    fp = s["fp_iters"]
    half = fp // 2
    contraction = None
    if fp >= 2 and rel[half] > 0 and rel[fp] > 0:
        contraction = float((rel[fp] / rel[half]) ** (1.0 / (fp - half)))
    curve = [[k, float("%.4g" % rel[k])] for k in range(0, len(rel), 10)]
    if curve[-1][0] != len(rel) - 1:
        curve.append([len(rel) - 1, float("%.4g" % rel[-1])])
    return {
        "status": st, "reached": st == 0, "fp_iters": fp, "krylov_iters": s["krylov_iters"],
        "krylov_per_fp_iter": s["krylov_iters"] / max(1, fp), "seconds": t_fp,
        "low_order_seconds": t_low, "low_order_krylov_iters": s0["krylov_iters"], "R0": R0,
        "final_rel_residual": float(rel[-1]), "contraction_last_half": contraction,
        "ms_per_iteration": 1e3 * t_fp / max(1, fp), "solution_range": [x_min, x_max],
        "lin_eta": lin_eta, "dynamic_damping": dynamic_damping,
        "residual_curve": curve,
    }


def bench_batch(afc, torch, I, count, steps, every):
    """256 seeded P1 CN-FCT instances x 20 steps in one persistent launch, and
    every `every`-th instance one at a time through afc_step_cn (an unbiased
    sample of the same size mix; the rate is that sample's solves/s)."""
    import numpy as np

    insts = [I.config4_instance(p) for p in I.config4_params(count)]
    o = afc.afc_default_options(krylov=afc.AFC_KRYLOV_BICGSTAB, fp_tol=1e-12, fp_maxit=50, lin_atol=1e-12)
    o.stream = torch.cuda.current_stream().cuda_stream
    b = afc.afc_batch_create(insts, o)
    try:
        offs = afc.afc_batch_offsets(b, count)
        u0 = np.zeros(offs[-1])
        Fp = np.zeros(offs[-1])
        for k, inst in enumerate(insts):
            u0[offs[k]:offs[k + 1]] = inst.u0
            Fp[offs[k]:offs[k + 1]] = inst.F
        F = torch.tensor(Fp, device="cuda:0")
        # schedule from the autotuner (one trial step per candidate, not timed)
        t0 = time.perf_counter()
        sched, trials = afc.afc_batch_autotune(b, torch.tensor(u0, device="cuda:0"), F, [1e-3] * count, 1)
        tune_s = time.perf_counter() - t0
        u = torch.tensor(u0, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, stats = afc.afc_batch_step_cn(b, u, F, [1e-3] * count, steps)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
    finally:
        afc.afc_batch_destroy(b)
    tseq = 0.0
    sample = insts[::every]
    nseq = len(sample)
    for inst in sample:
        h = afc.afc_create_instance(inst, o, conv=False)
        try:
            uk = torch.tensor(inst.u0, device="cuda:0")
            Fk = torch.tensor(inst.F, device="cuda:0")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                afc.afc_step_cn(h, uk, Fk, Fk, 1e-3)
            torch.cuda.synchronize()
            tseq += time.perf_counter() - t0
        finally:
            afc.afc_destroy(h)
    seq_rate = nseq / tseq
    return {
        "workload": "%d seeded P1 CN-FCT instances (n in 8..32, %d nodes), %d steps each, BiCGStab-Jacobi FP64"
                    % (count, int(offs[-1]), steps),
        "solves_per_s": count / tb, "seconds": tb, "status": st,
        "fp_iters": int(sum(x["fp_iters"] for x in stats)), "krylov_iters": int(sum(x["krylov_iters"] for x in stats)),
        "one_at_a_time_solves_per_s": seq_rate,
        "one_at_a_time_sample": "every %d-th instance (%d instances, mean %.0f nodes; all %d: mean %.0f)" % (
            every, nseq, sum(i.N for i in sample) / nseq, count, sum(i.N for i in insts) / count),
        "speedup": (count / tb) / seq_rate,
        "schedule": {"threads": sched[0], "workgroups": sched[1], "autotune_s": round(tune_s, 3),
                     "trial_ms": [round(t, 2) for t in trials]},
    }


def bench_cn(afc, torch, I, n, steps):
    """Nonlinear Zal+CN (fixed point) against linear Zal+CN (one solve per
    step) on the Q1 n^3 rotating-transport problem, BiCGStab-Jacobi FP64."""
    inst = I.config2(n)
    dt = 4.0 * inst.params["dt"]
    o = afc.afc_default_options(krylov=afc.AFC_KRYLOV_BICGSTAB, fp_tol=1e-8, fp_tol_mode=afc.AFC_TOL_REL,
                                fp_maxit=50, lin_atol=0.0, lin_rtol=1e-10)
    o.stream = torch.cuda.current_stream().cuda_stream
    out = {"workload": "Q1 %d^3 (%d nodes), rotating b, eps 1e-8, dt = 4 x CFL-0.2 step, %d CN steps, "
                       "BiCGStab-Jacobi FP64 to 1e-10 ||b||, fixed point to 1e-8 R0" % (n, inst.N, steps)}
    for name, step in (("nonlinear", afc.afc_step_cn), ("linear", afc.afc_step_cn_linear)):
        h = afc.afc_create_instance(inst, o, conv=False)
        try:
            u = torch.tensor(inst.u0, device="cuda:0")
            F = torch.tensor(inst.F, device="cuda:0")
            step(h, u.clone(), F, F, dt)  # warm-up (matrix build, graphs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fp = kr = 0
            for _ in range(steps):
                _, st = step(h, u, F, F, dt)
                fp += st["fp_iters"]
                kr += st["krylov_iters"]
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        finally:
            afc.afc_destroy(h)
        out[name] = {"ms_per_step": 1e3 * el / steps, "dof_steps_per_s": inst.N * steps / el,
                     "fp_iters_per_step": fp / steps, "krylov_per_step": kr / steps}
    return out


def bench_config1(afc, torch, I):
    """The P1 CN-FCT workload (Kuhn 8^3, 729 nodes): all 50 steps of dt 1e-3,
    BiCGStab-Jacobi FP64 to 1e-12, fixed point to sqrt(N) 1e-12 (<= 50)."""
    inst = I.config1()
    prm = inst.params
    o = afc.afc_default_options(krylov=afc.AFC_KRYLOV_BICGSTAB, fp_tol=prm["fp_tol"], fp_maxit=prm["fp_maxit"],
                                lin_atol=prm["lin_atol"], prelimit=prm["prelimit"])
    o.stream = torch.cuda.current_stream().cuda_stream
    h = afc.afc_create_instance(inst, o, conv=False)
    try:
        F = torch.tensor(inst.F, device="cuda:0")
        afc.afc_step_cn(h, torch.tensor(inst.u0, device="cuda:0"), F, F, prm["dt"])  # warm-up
        u = torch.tensor(inst.u0, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fp = kr = 0
        for _ in range(prm["steps"]):
            _, st = afc.afc_step_cn(h, u, F, F, prm["dt"])
            fp += st["fp_iters"]
            kr += st["krylov_iters"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        afc.afc_destroy(h)
    return {"workload": "P1 CN-FCT, Kuhn 8^3 x 6 tets (%d nodes), %d steps of dt %g" % (inst.N, prm["steps"], prm["dt"]),
            "seconds": el, "ms_per_step": 1e3 * el / prm["steps"], "fp_iters_per_step": fp / prm["steps"],
            "krylov_per_step": kr / prm["steps"], "dof_iterations_per_s": inst.N * fp / el,
            "range": [float(u.min()), float(u.max())]}


def bench_time_dependent(afc, torch, I, n, ssp_steps, cn_steps):
    """Explicit SSP-RK3 (Zalesak FCT vs MC limiter) and implicit CN (MC) on the
    Q1 n^3 rotating-transport problem (CFL 0.2 for SSP, 4x that step for CN)."""
    inst = I.config2(n)
    dt = inst.params["dt"]
    out = {"workload": "Q1 %d^3 (%d nodes), rotating b, eps 1e-8, ball indicator u0" % (n, inst.N)}
    o = afc.afc_default_options()
    o.stream = torch.cuda.current_stream().cuda_stream
    for name, step in (("fct_ssprk3", afc.afc_step_ssprk3), ("mc_ssprk3", afc.afc_step_mc_ssprk3)):
        h = afc.afc_create_instance(inst, o, conv=True)
        try:
            u = torch.tensor(inst.u0, device="cuda:0")
            F = torch.tensor(inst.F, device="cuda:0")
            step(h, u.clone(), F, dt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(ssp_steps):
                step(h, u, F, dt)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        finally:
            afc.afc_destroy(h)
        # u0 lies in [0, 1]; the limited explicit schemes keep the iterate there
        out[name] = {"ms_per_step": 1e3 * el / ssp_steps, "dof_stages_per_s": 3 * inst.N * ssp_steps / el,
                     "steps": ssp_steps, "range": [float(u.min()), float(u.max())]}
    oc = afc.afc_default_options(krylov=afc.AFC_KRYLOV_BICGSTAB, fp_tol=1e-8, fp_tol_mode=afc.AFC_TOL_REL,
                                 fp_maxit=50, lin_atol=0.0, lin_rtol=1e-10)
    oc.stream = o.stream
    h = afc.afc_create_instance(inst, oc, conv=True)
    try:
        u = torch.tensor(inst.u0, device="cuda:0")
        F = torch.tensor(inst.F, device="cuda:0")
        afc.afc_step_mc_cn(h, u.clone(), F, F, 4 * dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fp = 0
        for _ in range(cn_steps):
            _, st = afc.afc_step_mc_cn(h, u, F, F, 4 * dt)
            fp += st["fp_iters"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        afc.afc_destroy(h)
    out["mc_cn"] = {"ms_per_step": 1e3 * el / cn_steps, "dof_iterations_per_s": inst.N * fp / el,
                    "fp_iters_per_step": fp / cn_steps, "steps": cn_steps, "range": [float(u.min()), float(u.max())]}
    return out


def serve_opts(afc, kind):
    """Solver options of the serving workload: FP32-inner / FP64-outer GMRES;
    CN to R < sqrt(N) 1e-12 per step, the stationary MCL solve to R <= 1e-8 R0
    with the dynamic damping of Sec. 4 and inexact linear solves."""
    if kind == "cn":
        return afc.afc_default_options(precision=afc.AFC_PREC_MIXED, fp_tol=1e-12, fp_maxit=50, lin_atol=1e-13)
    return afc.afc_default_options(precision=afc.AFC_PREC_MIXED, fp_tol=1e-8, fp_tol_mode=afc.AFC_TOL_REL,
                                   fp_maxit=20000, lin_atol=0.0, lin_rtol=1e-10, lin_maxit=5000, dynamic_damping=1,
                                   lin_eta=1e-2)


def serve_run(afc, reqs, insts, rate, cfg):
    """Submit the requests at their arrival times (scaled to `rate`), wait for
    all; returns latencies, wall time, statuses and the server's round counts."""
    import threading

    import numpy as np

    s = afc.afc_server_create_cfg(cfg)
    ids = [None] * len(reqs)
    scale = 200.0 / rate  # the seeded arrival times are for 200 requests/s
    t0 = time.perf_counter()

    def submitter():
        for k, (r, inst) in enumerate(zip(reqs, insts)):
            d = scale * r["arrival"] - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            kind = afc.AFC_REQ_CN if r["kind"] == "cn" else afc.AFC_REQ_STATIONARY
            ids[k] = afc.afc_server_submit(s, kind, inst, serve_opts(afc, r["kind"]),
                                           u0=inst.u0 if r["kind"] == "cn" else None, dt=1e-3, steps=20,
                                           conv=r["kind"] == "mcl")

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    res = []
    for k, (rid, inst) in enumerate(zip(ids, insts)):
        res.append(afc.afc_server_wait(s, rid, inst.N))
        if (k + 1) % 25 == 0:
            print("bench: serving at %.3g/s: %d/%d done" % (rate, k + 1, len(reqs)), file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    rounds, carried, _ = afc.afc_server_info(s)
    afc.afc_server_destroy(s)
    lat = np.array([r[3][2] for r in res])
    mcl = [r for r, q in zip(res, reqs) if q["kind"] == "mcl"]
    return {
        "requests": len(reqs), "arrival_rate": rate, "solves_per_s": len(reqs) / wall, "seconds": wall,
        "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
        "statuses": {str(k): int(v) for k, v in zip(*np.unique([r[0] for r in res], return_counts=True))},
        "mcl_reached_1e-8": sum(1 for r in mcl if r[0] == 0), "mcl_requests": len(mcl),
        "fused_rounds": rounds, "requests_per_round": carried / max(1, rounds),
    }, [r[1] for r in res]


def one_at_a_time(afc, torch, reqs, insts):
    """The same requests solved one after another on their own handle with the
    same options (setup included, as a served request's is)."""
    t0 = time.perf_counter()
    out = []
    for r, inst in zip(reqs, insts):
        o = serve_opts(afc, r["kind"])
        o.stream = torch.cuda.current_stream().cuda_stream
        h = afc.afc_create_instance(inst, o, conv=r["kind"] == "mcl")
        try:
            F = torch.tensor(inst.F, device="cuda:0")
            if r["kind"] == "cn":
                u = torch.tensor(inst.u0, device="cuda:0")
                for _ in range(20):
                    afc.afc_step_cn(h, u, F, F, 1e-3, raise_on_error=False)
            else:
                u = torch.zeros(inst.N, dtype=torch.float64, device="cuda:0")
                afc.afc_solve_stationary(h, u, F, init_low_order=True, raise_on_error=False)
            out.append(u.cpu().numpy())
        finally:
            afc.afc_destroy(h)
    wall = time.perf_counter() - t0
    return {"solves_per_s": len(reqs) / wall, "seconds": wall, "requests": len(reqs)}, out


def bench_serve(afc, torch, I, count, sample_every):
    """Serving workload (Q1 n log-uniform 16..96, CN-FCT 20 steps or
    stationary MCL to 1e-8 R0): `count` Poisson arrivals at 200/s; the same
    requests at 0.8 x the saturation rate measured there; and every
    `sample_every`-th request, served at 200/s and solved one at a time (the
    same requests both ways)."""
    import numpy as np

    reqs = I.config5_requests(count)
    insts = [I.config5_instance(r) for r in reqs]
    cfg = afc.afc_server_default_config()
    # warm-up: ten requests of the same kind of stream (not reported)
    wreqs = I.config5_requests(10, seed=(0, 5, 9))
    serve_run(afc, wreqs, [I.config5_instance(r) for r in wreqs], 200.0, cfg)
    print("bench: serving %d requests at 200/s" % count, file=sys.stderr, flush=True)
    at200, _ = serve_run(afc, reqs, insts, 200.0, cfg)
    sat = at200["solves_per_s"]
    print("bench: serving %d requests at %.3g/s" % (count, 0.8 * sat), file=sys.stderr, flush=True)
    sustainable, _ = serve_run(afc, reqs, insts, 0.8 * sat, cfg)
    pick = list(range(0, count, sample_every))
    sub_r, sub_i = [reqs[k] for k in pick], [insts[k] for k in pick]
    print("bench: %d requests served and one at a time" % len(pick), file=sys.stderr, flush=True)
    served_sub, u_srv = serve_run(afc, sub_r, sub_i, 200.0, cfg)
    seq, u_seq = one_at_a_time(afc, torch, sub_r, sub_i)
    diff = max(float(np.abs(a - b).max() / max(np.abs(a).max(), 1e-300)) for a, b in zip(u_seq, u_srv))
    nodes = np.array([i.N for i in insts])
    return {
        "workload": "%d requests, Poisson arrivals, CN-FCT (20 steps, dt 1e-3) / stationary MCL (R <= 1e-8 R0, "
                    "dynamic damping, lin_eta 1e-2), Q1 n log-uniform 16..96, FP32-inner/FP64-outer options" % count,
        "config": {"slots": cfg.slots, "fuse_max_nodes": cfg.fuse_max_nodes, "loop_threads": cfg.loop_threads,
                   "quantum_ms": cfg.quantum_ms},
        "fused_lane_requests": int(np.sum(nodes <= cfg.fuse_max_nodes)),
        "mean_nodes": float(nodes.mean()),
        "at_200_per_s": at200,
        "at_0.8x_saturation": sustainable,
        "same_requests": {
            "sample": "every %d-th request (%d requests)" % (sample_every, len(pick)),
            "served_at_200_per_s": served_sub, "one_at_a_time": seq,
            "served_vs_one_at_a_time": served_sub["solves_per_s"] / seq["solves_per_s"],
            "max_rel_diff": diff,
        },
    }


def traffic_probe(n, sstep):
    """Program for the two HBM counter passes (FETCH_SIZE, then WRITE_SIZE):
    three plain 1 GiB device copies (the calibration of each counter), then
    one fixed-point iteration of the workload from its low-order solution with
    one basis vector per Arnoldi step, and one with s-step blocks."""
    import torch

    from paper_2110_15676_amd import afc
    from paper_2110_15676_amd import inputs as I

    src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    print("traffic probe: 3 copies of %d bytes done" % (1 << 30), flush=True)
    inst = I.config3(n)
    F = torch.tensor(inst.F, device="cuda")
    work = {}

    def add(name, kid, h):
        by, cnt = afc.afc_kernel_work(h, kid)
        w = work.setdefault(name, {"bytes": 0.0, "launches_with_work": 0})
        w["bytes"] += by
        w["launches_with_work"] += cnt

    for ss in (0, sstep):
        # profiled from the start, so that the library's work counters cover
        # every launch the counter passes see
        o = afc.afc_default_options(precision=afc.AFC_PREC_MIXED, krylov=afc.AFC_KRYLOV_GMRES, restart=30,
                                    fp_tol=0.0, fp_tol_mode=afc.AFC_TOL_REL, fp_maxit=0, lin_atol=0.0,
                                    lin_rtol=1e-10, lin_maxit=100000, profile=1, sstep=ss)
        o.stream = torch.cuda.current_stream().cuda_stream
        h = afc.afc_create_instance(inst, o, conv=True)
        u = torch.zeros(inst.N, dtype=torch.float64, device="cuda")
        afc.afc_solve_stationary(h, u, F, init_low_order=True)
        o.fp_maxit = 1
        afc.afc_set_options(h, o)
        _, st = afc.afc_solve_stationary(h, u, F)
        torch.cuda.synchronize()
        pre = "k_sstep" if ss else "k_gmres"
        add("k_sell_spmv32", afc.AFC_KERNEL_SPMV32, h)
        # blocks of more than eight vectors: the projections run on the matrix cores
        add(pre + ("_dots_mfma" if ss > 8 else "_dots"), afc.AFC_KERNEL_DOTS, h)
        add(pre + ("_update_mfma" if ss > 8 else "_update"), afc.AFC_KERNEL_UPDATE, h)
        add("k_sell_residual", afc.AFC_KERNEL_RESIDUAL, h)
        afc.afc_destroy(h)
        del u
        print("traffic probe: s=%d, 1 fixed-point iteration, %d Krylov iterations" % (ss, st["krylov_iters"]),
              flush=True)
    print("traffic probe work: " + json.dumps(work), flush=True)


def traffic_summarize(fetch_csv, write_csv, probe_log, n):
    """Turn the two counter CSVs of `traffic_probe` into HBM bytes per launch.
    Each counter is scaled by what it reads for the 1 GiB copies; launches that
    moved under 1 MiB (no-op launches after a cycle converged) are left out.
    Writes the SpMV figure, keyed by the kernel source hash, for the bench."""
    import csv

    from paper_2110_15676_amd import inputs as I

    def load(path, counter):
        out = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    fe, wr = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    work = None
    with open(probe_log) as f:
        for line in f:
            if line.startswith("traffic probe work: "):
                work = json.loads(line[len("traffic probe work: "):])
    if work is None:
        raise SystemExit("traffic: no 'traffic probe work' line in %s" % probe_log)

    def series(d, name):
        # demangled names: "void afc::(anonymous namespace)::k_sell_spmv32<short>(int, ...)"
        return [v for k, vals in d.items() if re.search(r"(^|::)%s[<(]" % name, k) or k == name for v in vals]

    gib_kib = float(1 << 20)
    cf = [v for v in series(fe, "__amd_rocclr_copyBuffer") if v > 0.25 * gib_kib]
    cw = [v for v in series(wr, "__amd_rocclr_copyBuffer") if v > 0.5 * gib_kib]
    if len(cf) < 3 or len(cw) < 3:
        raise SystemExit("traffic: the three 1 GiB calibration copies are missing from the counter files")
    sf, sw = gib_kib / (sum(cf[:3]) / 3), gib_kib / (sum(cw[:3]) / 3)
    table = {}
    for name in ("k_sell_spmv32", "k_gmres_dots", "k_gmres_update", "k_gmres_reduce", "k_sstep_dots",
                 "k_sstep_dots_mfma", "k_sstep_update", "k_sstep_update_mfma", "k_sstep_sums", "k_sell_residual",
                 "k_mcl_bounds_sell", "k_mcl_apply_sell"):
        f = [v for v in series(fe, name) if v > 1024]
        w = [v for v in series(wr, name) if v > 1024]
        if f:
            table[name] = {"launches": len(f), "fetch_bytes": 1024 * sf * sum(f) / len(f),
                           "write_bytes": 1024 * sw * sum(w) / len(w) if w else 0.0}
    for name, t in table.items():
        if name in work and work[name]["launches_with_work"] == t["launches"]:
            t["algorithmic_bytes"] = work[name]["bytes"] / t["launches"]
    inst = I.config3(n)
    sp = table["k_sell_spmv32"]
    if "algorithmic_bytes" not in sp:
        raise SystemExit("traffic: counted %d SpMV launches with work, the library %d"
                         % (sp["launches"], work["k_sell_spmv32"]["launches_with_work"]))
    rec = {"kernel": "k_sell_spmv32<short>",
           "workload": "stationary MCL Q1 %d^3 (%d nodes, %d nnz)" % (n, inst.N, inst.nnz),
           "nnz": inst.nnz, "bytes_per_launch": round(sp["fetch_bytes"] + sp["write_bytes"]),
           "algorithmic_bytes_per_launch": round(sp["algorithmic_bytes"]),
           "fetch_bytes": round(sp["fetch_bytes"]), "write_bytes": round(sp["write_bytes"]),
           "launches_averaged": sp["launches"], "fetch_scale": sf, "write_scale": sw,
           "kernel_source_sha": kernel_source_hash()}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print("copy calibration: FETCH_SIZE %.1f KiB, WRITE_SIZE %.1f KiB per 1 GiB copy -> scales %.4f, %.4f"
          % (sum(cf[:3]) / 3, sum(cw[:3]) / 3, sf, sw))
    print("| kernel | launches | fetch MB | write MB | algorithmic MB |")
    print("|---|---|---|---|---|")
    for name, t in table.items():
        alg = "%.1f" % (t["algorithmic_bytes"] / 1e6) if "algorithmic_bytes" in t else "-"
        print("| %s | %d | %.1f | %.1f | %s |" % (name, t["launches"], t["fetch_bytes"] / 1e6,
                                                  t["write_bytes"] / 1e6, alg))


def accuracy_examples(n_rot, n_circ):
    """The paper's analytic accuracy examples on this package's meshes, run
    through the GPU library: rotating shapes (one full rotation, five schemes)
    and circular convection (stationary MC and MU limiters).  Errors use the
    lumped-mass nodal quadrature: L1 = sum_i m_i |e_i|, L2 = sqrt(sum_i m_i e_i^2)."""
    import numpy as np
    import torch

    from paper_2110_15676_amd import afc
    from paper_2110_15676_amd import inputs as I

    stream = torch.cuda.current_stream().cuda_stream

    def mk_opts(**kw):
        o = afc.afc_default_options(**kw)
        o.stream = stream
        return o

    def lumped(inst):
        m = np.zeros(inst.N)
        np.add.at(m, inst.row_index(), inst.M)
        return m

    out = {}
    inst = I.rotating_shapes(n_rot)
    m = lumped(inst)
    dt, steps = inst.params["dt"], inst.params["steps"]
    # nonlinear loops as in the paper: stop at R < 1e-20 or after 50 iterations
    fp = dict(fp_tol=1e-20 / math.sqrt(inst.N), fp_tol_mode=afc.AFC_TOL_ABS_SQRTN, fp_maxit=50,
              krylov=afc.AFC_KRYLOV_BICGSTAB, lin_atol=0.0, lin_rtol=1e-12)
    schemes = (("MC+SSP", afc.afc_step_mc_ssprk3, dict(ssp_stages=2), False),
               ("MC+CN", afc.afc_step_mc_cn, fp, True),
               ("Zal+CN linear", afc.afc_step_cn_linear, fp, True),
               ("Zal+CN nonlinear", afc.afc_step_cn, fp, True),
               ("Zal+SSP", afc.afc_step_ssprk3, dict(ssp_stages=2), False))
    rot = {"mesh": "Q1 %d^3 (%d nodes), dt = %.4g, %d steps (T = 2 pi)" % (n_rot, inst.N, dt, steps)}
    for name, step, kw, implicit in schemes:
        print("accuracy: rotating shapes, %s" % name, file=sys.stderr, flush=True)
        h = afc.afc_create_instance(inst, mk_opts(**kw), conv=True)
        try:
            u = torch.tensor(inst.u0, device="cuda:0")
            F = torch.tensor(inst.F, device="cuda:0")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                if implicit:
                    step(h, u, F, F, dt, raise_on_error=False)
                else:
                    step(h, u, F, dt, raise_on_error=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        finally:
            afc.afc_destroy(h)
        x = u.cpu().numpy()
        e = x - inst.u0
        rot[name] = {"L2_error": float(np.sqrt(np.sum(m * e * e))), "min": float(x.min()), "max": float(x.max()),
                     "seconds": round(el, 3)}
    out["rotating_shapes"] = rot
    circ = {}
    for n in n_circ:
        inst = I.circular_convection(n)
        m = lumped(inst)
        ex = I.circular_convection_exact(inst.coords)
        row = {"mesh": "P1 %d^3 x 6 tetrahedra (%d nodes)" % (n, inst.N)}
        for name, lim in (("MC", afc.AFC_LIMITER_MCL), ("MU", afc.AFC_LIMITER_MU)):
            print("accuracy: circular convection n=%d, %s" % (n, name), file=sys.stderr, flush=True)
            o = mk_opts(limiter=lim, fp_tol=1e-8, fp_tol_mode=afc.AFC_TOL_REL, fp_maxit=3000, lin_atol=0.0,
                        lin_rtol=1e-12)
            h = afc.afc_create_instance(inst, o, conv=True)
            try:
                u = torch.zeros(inst.N, dtype=torch.float64, device="cuda:0")
                t0 = time.perf_counter()
                st, stats = afc.afc_solve_stationary(h, u, torch.tensor(inst.F, device="cuda:0"), init_low_order=True,
                                                     raise_on_error=False)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
            finally:
                afc.afc_destroy(h)
            x = u.cpu().numpy()
            e = x - ex
            row[name] = {"L1_error": float(np.sum(m * np.abs(e))), "L2_error": float(np.sqrt(np.sum(m * e * e))),
                         "min": float(x.min()), "max": float(x.max()), "fp_iters": stats["fp_iters"],
                         "status": st, "seconds": round(el, 3)}
        circ[str(n)] = row
    out["circular_convection"] = circ
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128, help="cells per direction (128 is the workload)")
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--mu-steps", type=int, default=5)
    ap.add_argument("--sstep", type=int, default=15,
                    help="GMRES basis block size s (0: one vector per step; 2..16: s-step blocks)")
    ap.add_argument("--classical-steps", type=int, default=5,
                    help="steps timed again with one basis vector per Arnoldi step (secondary)")
    ap.add_argument("--cpu-n", type=int, default=64,
                    help="mesh of the oracle's first-iteration sample (cells per direction)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch-oracle", action="store_true", help="leave out the batched-CN oracle sample")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="only time the oracle's first iteration on --cpu-n (and the GPU on the same sample)")
    ap.add_argument("--solve-cap", type=int, default=8000,
                    help="fixed-point cap of the solves run to the stopping rule R <= 1e-8 R0")
    ap.add_argument("--no-solve", action="store_true", help="leave out the solves run to the stopping rule")
    ap.add_argument("--no-strict-solve", action="store_true",
                    help="run the stopping-rule solve with inexact linear solves only")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cn", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-sample", type=int, default=4,
                    help="every k-th served request is also solved one at a time")
    ap.add_argument("--serve-only", action="store_true", help="only run the serving workload")
    ap.add_argument("--accuracy", action="store_true",
                    help="only run the paper's analytic accuracy examples (rotating shapes, circular convection)")
    ap.add_argument("--accuracy-n", type=int, default=64, help="cells per direction of the rotating-shapes mesh")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run the program profiled by the FETCH_SIZE / WRITE_SIZE counter passes")
    ap.add_argument("--traffic-summarize", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "PROBE_LOG"),
                    help="turn the counter CSVs of --traffic-probe into the per-launch traffic file (no GPU)")
    args = ap.parse_args()
    if args.traffic_summarize:
        traffic_summarize(*args.traffic_summarize, args.n)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.traffic_probe:
        traffic_probe(args.n, args.sstep)
        return
    if args.accuracy:
        print(json.dumps(accuracy_examples(args.accuracy_n, (16, 32, 64))))
        return

    import numpy as np
    import torch

    from paper_2110_15676_amd import afc
    from paper_2110_15676_amd import inputs as I

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.serve_only:
        print(json.dumps(bench_serve(afc, torch, I, args.serve_requests, args.serve_sample)))
        return
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(args.cpu_n, gpu_first_iteration(afc, torch, I, args.cpu_n, args.sstep), False)))
        return
    print("bench: building Q1 %d^3 MCL instance" % args.n, file=sys.stderr, flush=True)
    inst = I.config3(args.n)
    N, nnz = inst.N, inst.nnz
    stream = torch.cuda.current_stream().cuda_stream

    def opts(**kw):
        kw.setdefault("sstep", args.sstep)
        o = afc.afc_default_options(precision=afc.AFC_PREC_MIXED, krylov=afc.AFC_KRYLOV_GMRES, restart=30,
                                    fp_tol=0.0, fp_tol_mode=afc.AFC_TOL_REL, lin_atol=0.0, lin_rtol=1e-10,
                                    lin_maxit=100000, **kw)
        o.stream = stream
        return o

    h = afc.afc_create_instance(inst, opts(fp_maxit=0), conv=True)
    info = afc.afc_get_sell_info(h)
    kinfo = afc.afc_get_krylov_sell_info(h)
    u = torch.zeros(N, dtype=torch.float64, device=dev)
    F = torch.tensor(inst.F, device=dev)
    afc.afc_solve_stationary(h, u, F, init_low_order=True)  # low-order start, not timed
    print("bench: warmup %d" % args.warmup, file=sys.stderr, flush=True)
    if args.warmup > 0:
        afc.afc_set_options(h, opts(fp_maxit=args.warmup))
        afc.afc_solve_stationary(h, u, F)

    # --- timed region: exactly `steps` fixed-point iterations ---------------
    afc.afc_set_options(h, opts(fp_maxit=args.steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, s = afc.afc_solve_stationary(h, u, F)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert s["fp_iters"] == args.steps, s
    value = N * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    model_bytes = step_model_bytes(N, info, kinfo, s["krylov_iters"], s["refine_sweeps"], args.steps, args.sstep)
    print("bench: %.1f ms/step, %d Krylov its" % (ms_per_step, s["krylov_iters"]), file=sys.stderr, flush=True)
    # extremes of the iterate after the timed steps (reported, not asserted:
    # with c = 1 the discrete maximum principle of the eps = 0, c = 0 steady
    # state does not apply)
    u_range = {"min": float(u.min()), "max": float(u.max())}

    # --- the same steps again with per-kernel HIP events (roofline) ----------
    afc.afc_set_options(h, opts(fp_maxit=args.steps, profile=1))
    for kid in range(afc.AFC_KERNEL_COUNT):
        afc.afc_kernel_time(h, kid, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st2, s2 = afc.afc_solve_stationary(h, u, F)
    torch.cuda.synchronize()
    elapsed_prof = time.perf_counter() - t0
    classes = (("spmv32", afc.AFC_KERNEL_SPMV32), ("dots", afc.AFC_KERNEL_DOTS), ("update", afc.AFC_KERNEL_UPDATE),
               ("residual", afc.AFC_KERNEL_RESIDUAL), ("mcl", afc.AFC_KERNEL_MCL), ("finish", afc.AFC_KERNEL_FINISH))
    kernels = {}
    for name, kid in classes:
        ms, launches = afc.afc_kernel_time(h, kid)
        by, work = afc.afc_kernel_work(h, kid)
        kernels[name] = {"ms_per_step": round(ms / args.steps, 3), "launches": launches, "with_work": work,
                         "gbs": round(by / (1e-3 * ms) / 1e9, 1) if by > 0 and ms > 0 else None}
    # dominant kernel: the FP32 SELL SpMV of the inner GMRES.  Launches issued
    # after a cycle converged return at once: their (small) time stays in the
    # total, the average is taken over launches with work.
    spmv_ms, spmv_launches = afc.afc_kernel_time(h, afc.AFC_KERNEL_SPMV32)
    spmv_bytes_total, spmv_work = afc.afc_kernel_work(h, afc.AFC_KERNEL_SPMV32)
    spmv_avg_s = 1e-3 * spmv_ms / max(1, spmv_work)
    spmv_b = spmv_bytes_total / max(1, spmv_work)
    achieved = spmv_b / spmv_avg_s / 1e9
    traffic = None
    traffic_alg = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_source_sha") == kernel_source_hash() and tr.get("nnz") == nnz:
            traffic = tr.get("bytes_per_launch")
            traffic_alg = tr.get("algorithmic_bytes_per_launch")
    roofline = {
        "kernel": "k_sell_spmv32 (FP32 SELL-64 SpMV, GMRES inner)",
        "sell": kinfo,
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "traffic_probe_algorithmic": traffic_alg,
        "bytes_per_launch": round(spmv_b), "avg_launch_us": round(spmv_avg_s * 1e6, 2),
        "launches": spmv_launches, "launches_with_work": spmv_work,
        "kernels": kernels,
        "profiled_ms_per_step": round(1e3 * elapsed_prof / args.steps, 3),
    }

    # --- the same GMRES with one basis vector per Arnoldi step (secondary) ---
    classical = None
    if args.classical_steps > 0 and args.sstep > 0:
        afc.afc_set_options(h, opts(fp_maxit=args.classical_steps, sstep=0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, s5 = afc.afc_solve_stationary(h, u, F)
        torch.cuda.synchronize()
        e5 = time.perf_counter() - t0
        classical = {"value": N * s5["fp_iters"] / e5, "ms_per_step": 1e3 * e5 / max(1, s5["fp_iters"]),
                     "krylov_per_step": s5["krylov_iters"] / max(1, s5["fp_iters"]), "steps": s5["fp_iters"]}
    # --- plain FP64 GMRES for comparison (secondary) ------------------------
    fp64 = None
    if args.fp64_steps > 0:
        # FP64 GMRES in the bench's s-step blocks, and with one basis vector
        # per step, the same steps from the same state
        u_start = u.clone()
        runs = {}
        for name, ss in (("sstep", args.sstep), ("one_vector", 0)):
            uu = u_start.clone()
            o = opts(fp_maxit=args.fp64_steps, sstep=ss)
            o.precision = afc.AFC_PREC_FP64
            afc.afc_set_options(h, o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, s3 = afc.afc_solve_stationary(h, uu, F)
            torch.cuda.synchronize()
            e3 = time.perf_counter() - t0
            runs[name] = (uu, s3, e3)
        u = runs["sstep"][0]
        # the same steps with the mixed-precision solve: relative L2 distance of the iterates
        u_mixed = u_start.clone()
        afc.afc_set_options(h, opts(fp_maxit=args.fp64_steps))
        afc.afc_solve_stationary(h, u_mixed, F)
        diff = float(torch.linalg.vector_norm(u_mixed - u) / torch.linalg.vector_norm(u))
        u1 = runs["one_vector"][0]
        diff1 = float(torch.linalg.vector_norm(u1 - u) / torch.linalg.vector_norm(u))

        def rate(r):
            _, st, el = r
            return {"value": N * st["fp_iters"] / el, "ms_per_step": 1e3 * el / max(1, st["fp_iters"]),
                    "krylov_per_step": st["krylov_iters"] / max(1, st["fp_iters"]), "steps": st["fp_iters"]}

        fp64 = dict(rate(runs["sstep"]), gmres_sstep=args.sstep, mixed_vs_fp64_rel_l2=diff,
                    one_vector_per_step=dict(rate(runs["one_vector"]), sstep_vs_one_vector_rel_l2=diff1))
    # --- the MU limiter (Sec. 3.2) on the same problem (secondary) ----------
    mu = None
    if args.mu_steps > 0:
        o = opts(fp_maxit=0, limiter=afc.AFC_LIMITER_MU)
        afc.afc_set_options(h, o)
        umu = torch.zeros(N, dtype=torch.float64, device=dev)
        afc.afc_solve_stationary(h, umu, F, init_low_order=True)
        afc.afc_set_options(h, opts(fp_maxit=args.mu_steps, limiter=afc.AFC_LIMITER_MU))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, s4 = afc.afc_solve_stationary(h, umu, F)
        torch.cuda.synchronize()
        e4 = time.perf_counter() - t0
        mu = {"value": N * s4["fp_iters"] / e4, "ms_per_step": 1e3 * e4 / max(1, s4["fp_iters"]),
              "krylov_per_step": s4["krylov_iters"] / max(1, s4["fp_iters"]), "steps": s4["fp_iters"],
              "nonlinear_residual": {"first": s4["res0"], "last": s4["res"]}}
    afc.afc_destroy(h)

    batch = None
    if not args.no_batch:
        print("bench: batched CN-FCT", file=sys.stderr, flush=True)
        batch = bench_batch(afc, torch, I, 256, 20, 4)
    cn = None
    if not args.no_cn:
        print("bench: CN (nonlinear vs linear Zal+CN)", file=sys.stderr, flush=True)
        cn = bench_cn(afc, torch, I, 64, 10)
        cn["time_dependent"] = bench_time_dependent(afc, torch, I, 64, 200, 5)
        cn["config1_p1_cn"] = bench_config1(afc, torch, I)
    serve = None
    if not args.no_serve:
        print("bench: serving", file=sys.stderr, flush=True)
        serve = bench_serve(afc, torch, I, args.serve_requests, args.serve_sample)

    solve = None
    if not args.no_solve:
        def solve_opts(**kw):
            o = opts(**{k: v for k, v in kw.items() if k in ("fp_maxit", "sstep")})
            for k, v in kw.items():
                setattr(o, k, v)
            return o

        solve = {"rule": "R <= 1e-8 R0 from the low-order solution, dynamic damping (Sec. 4), cap %d"
                         % args.solve_cap}
        solve["inexact"] = solve_to_tolerance(afc, torch, inst, solve_opts, 1e-8, args.solve_cap, lin_eta=1e-2,
                                              label="inexact (lin_eta 1e-2)")
        if not args.no_strict_solve:
            solve["strict"] = solve_to_tolerance(afc, torch, inst, solve_opts, 1e-8, args.solve_cap,
                                                 label="strict (1e-10 ||b||)")

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.cpu_n, gpu_first_iteration(afc, torch, I, args.cpu_n, args.sstep),
                           not args.no_batch_oracle)

    line = {
        "metric": "AFC DOF-iterations/s at 128^3 Q1 (stationary MCL fixed-point iterations)",
        "value": value,
        "unit": "DOF-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 limiter/outer + f32 Krylov inner",
        "data": "synthetic",
        "config": {
            "workload": "stationary MCL, Q1 %d^3 (%d nodes, %d nnz), eps=1e-6, b=(1,1,1)/sqrt3, c=1, "
                        "f=1 on [0.25,0.5]^3, u=0 on the boundary; fixed-point iterations from the low-order "
                        "solution, GMRES(30)-Jacobi FP32 inner (%s) + FP64 refinement to 1e-10 ||b||"
                        % (args.n, N, nnz, "s-step blocks of %d" % args.sstep if args.sstep else "one vector per step"),
            "nodes": N, "nnz": nnz, "gmres_sstep": args.sstep, "parallelism": "1 GPU",
        },
        "krylov_per_step": s["krylov_iters"] / args.steps,
        "refine_sweeps_per_step": s["refine_sweeps"] / args.steps,
        "dof_krylov_its_per_s": N * s["krylov_iters"] / elapsed,
        "hbm_gbs_model": model_bytes / elapsed / 1e9,
        "nonlinear_residual": {"first": s["res0"], "last": s["res"]},
        "solution_range": u_range,
        "fp64": fp64,
        "classical_arnoldi": classical,
        "mu_limiter": mu,
        "batch": batch,
        "cn": cn,
        "serving": serve,
        "solve_to_tolerance": solve,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
