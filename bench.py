#!/usr/bin/env python3
"""Throughput of Strang runs on one MI355X: lattice-point Strang steps/s.

Workload: d = 6 rank-1 lattice with N = 1048573 points (prime, so each DFT
runs as a chirp-z convolution of length 2^21), z from a seeded reconstructing
CBC search on the hyperbolic cross R = 10 completed to N keys with minimal-l2
representatives, gamma = 0.05, v = prod_j (1 + cos(2 pi x_j)/2) - 1, seeded
Gaussian packet, dt = 1e-3, 1000 time steps per run.  One benchmark "step" is
one full strang_run (all 1000 time steps) with the state resident in HBM.

The JSON line also carries the roofline of the dominant kernel (HIP-event
timing of the library's own launches during the timed region), the complex128
throughput, the FP64 oracle timed on the host, accuracy indicators, and three
companion workloads: 256 unrelated problems advanced by strang_run_batched in
complex64 against the same problems run one by one in complex128; the d = 10
rank-2 lattice 4096 x 256; and a forward run with checkpoints plus its adjoint
(d = 4, N = 65521, 32 states); and the norm / energy conservation setting of
Sec. 3.3 on a 2^20-point lattice; the time-step convergence protocol of
Sec. 3.2 on a lattice of the paper's Table 1 (d = 3, n = 2^22); and the
fourth-order composition and a time-dependent potential (Sec. 5) on the
benchmark lattice; the Table 1 lattice d = 6, n = 2^25, whose transform
takes rows of 8192 points; the benchmark lattice with 8 states, whose
working set exceeds the 256 MB Infinity Cache; and the initial discretization
error of Sec. 3.4 on Table 1 lattices.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lattice-point Strang steps/s per GPU (C128, C64), fwd+adjoint; % HBM peak"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pass_bytes(plan_info, N, m, S):
    """Algorithmic HBM bytes of every column-pass and row-pass launch of one
    run of the benchmark workload (prime N, so the kinetic part of each step
    is one zero-padded cyclic convolution of length L): each pass reads and
    writes the state once and reads the tables its step needs -- v (FP64,
    8 B per point) in the first and last passes, the merged potential step
    exp(-i dt v / gamma) per point in the middle ones (16 B: a hi/lo pair of
    complex floats for complex64, one complex double for complex128), and the
    convolution spectrum (complex double, 16 B per bin) in the row pass."""
    L = plan_info["fft_len"]
    pot = 16 * N
    col = [N * S + 8 * N + L * S]                 # first: u, v in; transform out
    col += [2 * L * S + pot] * (m - 1)            # merged potential steps P^2
    col += [L * S + 8 * N + N * S]                # last: transform in, v in, u out
    row = [2 * L * S + 16 * L] * m                # state in/out + convolution spectrum
    return col, row


def pmc_traffic(kind="column"):
    """Measured HBM bytes per steady-state launch of one pass kind (complex64),
    from the committed counter summary (FETCH_SIZE / WRITE_SIZE scaled by a
    plain copy's readings); None when absent."""
    path = os.path.join(ROOT, "profiles", "k_colf_k_rowf_c64_d6_N1048573_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if f"{kind}_c64_hbm_bytes_per_launch:" in line:
            return float(line.split(":")[1])
    return None


def time_runs(lt, torch, plan, v, u, work, inst, K, W):
    """Region A: K plain runs (the throughput).  Region B: K more runs with
    every kernel launch bracketed by HIP events on the library's stream (the
    per-kernel durations for the roofline); the event records add gaps between
    launches, so region B's wall time is not used for the throughput."""
    for _ in range(W):
        lt.strang_run(plan, v, u, inst.gamma, inst.dt, inst.steps, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        lt.strang_run(plan, v, u, inst.gamma, inst.dt, inst.steps, work=work)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"timed region: {K} runs in {t1 - t0:.3f}s")
    lt.lt_timing_enable(True)
    tb = time.perf_counter()
    for i in range(K):
        lt.strang_run(plan, v, u, inst.gamma, inst.dt, inst.steps, work=work)
    torch.cuda.synchronize()
    tb = time.perf_counter() - tb
    kinds = {"column": lt.lt_timing_summary(lt.LT_KIND_COLUMN),
             "row": lt.lt_timing_summary(lt.LT_KIND_ROW)}
    lt.lt_timing_enable(False)
    log(f"event-instrumented region: {K} runs in {tb:.3f}s")
    return t1 - t0, kinds, tb


def kernel_summary(lt, fn, K):
    """Per-kernel-class event times of K calls of fn (instrumented region)."""
    import torch
    torch.cuda.synchronize()
    lt.lt_timing_enable(True)
    for _ in range(K):
        fn()
    torch.cuda.synchronize()
    out = {}
    for name, kind in (("column", lt.LT_KIND_COLUMN), ("row", lt.LT_KIND_ROW),
                       ("resident", lt.LT_KIND_RESIDENT)):
        n, ms = lt.lt_timing_summary(kind)
        if n:
            out[name] = {"launches": n // K, "ms_per_call": ms / K, "avg_us": ms / n * 1e3}
    lt.lt_timing_enable(False)
    return out


def wall(fn, K, W):
    import torch
    for _ in range(W):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(K):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / K


def bench_batched(lt, torch, K, W):
    """256 unrelated problems (d 2..10, N 2^12..2^18, 200 steps each):
    strang_run_batched in complex64 vs. the single-state complex128 path
    (strang_run per problem, one after another)."""
    import numpy as np

    import workloads as W_
    t = time.perf_counter()
    insts = W_.mixed_batch()
    plans = [lt.lattice_plan(c.Z, c.n, c.I) for c in insts]
    log(f"batched: inputs and {len(plans)} plans in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda:0")
    vs = [torch.tensor(c.v, dtype=torch.float64, device=dev) for c in insts]
    gam = [c.gamma for c in insts]
    dts = [c.dt for c in insts]
    st = [c.steps for c in insts]
    pt_steps = sum(c.N * c.steps for c in insts)
    res = {}
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        prec = lt.LT_C64 if name == "c64" else lt.LT_C128
        us = [torch.tensor(c.u0, dtype=dtype, device=dev) for c in insts]
        work = torch.empty(lt.strang_batched_workspace_size(plans, prec), dtype=torch.uint8, device=dev)
        run = lambda: lt.strang_run_batched(plans, vs, us, gam, dts, st, work=work)  # noqa: E731
        sec = wall(run, K, W)
        res[f"batched_{name}"] = {"value": pt_steps / sec, "ms_per_call": sec * 1e3,
                                  "kernels": kernel_summary(lt, run, 1)}
        log(f"batched {name}: {pt_steps / sec:.3e} pt-steps/s, {sec * 1e3:.1f} ms per batch")
        del us, work
    # the plain single-state complex128 path over the same problems
    us = [torch.tensor(c.u0, dtype=torch.complex128, device=dev) for c in insts]
    wmax = max(lt.strang_workspace_size(p, lt.LT_C128, 1, True) for p in plans)
    work = torch.empty(wmax, dtype=torch.uint8, device=dev)

    def singles():
        for p, v, u, c in zip(plans, vs, us, insts):
            lt.strang_run(p, v, u, c.gamma, c.dt, c.steps, work=work)
    sec = wall(singles, 1, 1)
    res["single_c128"] = {"value": pt_steps / sec, "ms_per_call": sec * 1e3}
    log(f"single-state c128: {pt_steps / sec:.3e} pt-steps/s, {sec * 1e3:.1f} ms")
    # accuracy of the batched complex64 result against stored FP64 oracle samples
    gold_path = os.path.join(ROOT, "tests", "golden", "mixed_batch_oracle_samples.npz")
    acc = None
    if os.path.exists(gold_path):
        gold = np.load(gold_path)
        us = [torch.tensor(c.u0, dtype=torch.complex64, device=dev) for c in insts]
        lt.strang_run_batched(plans, vs, us, gam, dts, st)
        errs = []
        for i in gold["instances"]:
            got = us[int(i)].cpu().numpy().astype(np.complex128)[gold[f"idx_{i}"]]
            ref = gold[f"u_{i}"]
            errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
        acc = {"c64_max_sampled_rel_l2_vs_oracle": max(errs), "problems_sampled": len(errs)}
    Ns = [c.N for c in insts]
    return {
        "workload": f"{len(insts)} unrelated rank-1 problems, d in 2..10, N in [{min(Ns)}, {max(Ns)}] "
                    f"(primes and 7-smooth composites, sum N = {sum(Ns)}), best-of-8 Korobov lattices, "
                    "minimal-l2 index sets, 16-term cosine potentials, gamma in [0.02, 0.2], dt = 5e-3, "
                    f"{insts[0].steps} steps each",
        "unit": "lattice-point-steps/s",
        "value_c64": res["batched_c64"]["value"],
        "speedup_c64_batched_vs_single_state_c128": res["batched_c64"]["value"] / res["single_c128"]["value"],
        **res, "accuracy": acc,
    }


def bench_rank2(lt, torch, K, W):
    """d = 10 rank-2 lattice n = (4096, 256), 500 steps."""
    import workloads as W_
    c = W_.rank2_d10_n4096x256()
    plan = lt.lattice_plan(c.Z, c.n, c.I)
    dev = torch.device("cuda:0")
    v = torch.tensor(c.v, dtype=torch.float64, device=dev)
    out = {"workload": "rank-2 lattice d=10 n=(4096, 256), hyperbolic cross {-1,0,1}^10 + minimal-l2 "
                       f"completion, gamma=0.05, dt=2e-3, {c.steps} steps per run",
           "unit": "lattice-point-steps/s"}
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        prec = lt.LT_C64 if name == "c64" else lt.LT_C128
        kernels = lt.lattice_plan_autotune(plan, prec, reps=10)
        u = torch.tensor(c.u0, dtype=dtype, device=dev)
        work = torch.empty(lt.strang_workspace_size(plan, prec, 1, True), dtype=torch.uint8, device=dev)
        run = lambda: lt.strang_run(plan, v, u, c.gamma, c.dt, c.steps, work=work)  # noqa: E731
        sec = wall(run, K, W)
        out[name] = {"value": c.N * c.steps / sec, "ms_per_run": sec * 1e3, "kernel_variants": list(kernels),
                     "kernels": kernel_summary(lt, run, 1)}
        log(f"rank-2 {name}: {c.N * c.steps / sec:.3e} pt-steps/s, {sec * 1e3:.1f} ms per run")
    return out


def bench_adjoint(lt, torch, K, W):
    """Forward run with checkpoints every 50 steps plus strang_adjoint: d = 4,
    N = 65521, 32 states sharing v, 500 steps."""
    import workloads as W_
    c = W_.adjoint_d4_n65521()
    plan = lt.lattice_plan(c.Z, c.n, c.I)
    dev = torch.device("cuda:0")
    v = torch.tensor(c.v, dtype=torch.float64, device=dev)
    B, N, m, every = c.u0.shape[0], c.N, c.steps, c.meta["ckpt_every"]
    out = {"workload": f"rank-1 d=4 N={N} (prime), {B} states sharing a 64-term cosine potential, "
                       f"gamma=0.05, dt=2e-3, {m} steps, checkpoints every {every}",
           "unit": "lattice-point-steps/s (forward + adjoint)"}
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        prec = lt.LT_C64 if name == "c64" else lt.LT_C128
        lt.lattice_plan_autotune(plan, prec, reps=10)
        u0 = torch.tensor(c.u0, dtype=dtype, device=dev)
        u = torch.empty_like(u0)
        ck = torch.empty(lt.num_checkpoints(m, every) * B * N, dtype=dtype, device=dev)
        tgt = torch.zeros_like(u0)
        fw = torch.empty(lt.strang_workspace_size(plan, prec, B, True), dtype=torch.uint8, device=dev)
        aw = torch.empty(lt.strang_adjoint_workspace_size(plan, prec, B, True), dtype=torch.uint8, device=dev)

        def fwd():
            u.copy_(u0)
            lt.strang_run(plan, v, u, c.gamma, c.dt, m, ckpt=ck, ckpt_every=every, work=fw)
        fwd()
        gT = (2.0 / N) * (u - tgt)

        def adj():
            lt.strang_adjoint(plan, v, u, gT, c.gamma, c.dt, m, ck, every, work=aw)
        tf = wall(fwd, K, W)
        ta = wall(adj, K, W)
        out[name] = {"value": B * N * m / (tf + ta), "forward_ms": tf * 1e3, "adjoint_ms": ta * 1e3,
                     "variants": {"one_state": lt.lattice_plan_get_kernels_batch(plan, prec, 1),
                                  f"{B}_states": lt.lattice_plan_get_kernels_batch(plan, prec, B)},
                     "adjoint_kernels": kernel_summary(lt, adj, 1)}
        log(f"adjoint {name}: fwd {tf * 1e3:.1f} ms, adj {ta * 1e3:.1f} ms, "
            f"{B * N * m / (tf + ta):.3e} pt-steps/s")
    return out


def bench_conservation(lt, torch, K, W):
    """The conservation setting of Sec. 3.3 (gamma = 0.5, d = 5, g1, harmonic
    v2) on a 2^20-point lattice: 1000 steps with checkpoints every 10, norm and
    energy of every checkpoint by lattice_diagnostics, delta = (max-min)/mean."""
    import numpy as np

    import workloads as W_
    N, d, gamma, dt, steps, every = 1 << 20, 5, 0.5, 1e-3, 1000, 10
    z = W_.korobov_good(N, d, np.random.default_rng(33))
    Z, n = z.reshape(1, -1), np.array([N])
    num = W_.point_numerators(Z, n)
    plan = lt.lattice_plan(Z, n)
    dev = torch.device("cuda:0")
    v = torch.tensor(W_.v_harmonic_paper(num, N), device=dev)
    u0 = W_.paper_g1(num, N, gamma)
    out = {"workload": f"Sec. 3.3 setting: rank-1 d={d} N=2^20 (best-of-8 Korobov), gamma={gamma}, g1, "
                       f"harmonic v2, dt={dt}, {steps} steps, norm and energy every {every} steps"}
    nck = lt.num_checkpoints(steps, every)
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        u = torch.tensor(u0, dtype=dtype, device=dev)
        ck = torch.empty(nck * N, dtype=dtype, device=dev)
        # one untimed run first (the plan's tables and first-use setup)
        lt.strang_run(plan, v, u, gamma, dt, steps, ckpt=ck, ckpt_every=every)
        lt.lattice_diagnostics(plan, v, ck.view(nck, N), gamma)
        u.copy_(torch.tensor(u0, dtype=dtype, device=dev))
        torch.cuda.synchronize()
        t = time.perf_counter()
        lt.strang_run(plan, v, u, gamma, dt, steps, ckpt=ck, ckpt_every=every)
        torch.cuda.synchronize()
        t_run = time.perf_counter() - t
        diag = lt.lattice_diagnostics(plan, v, ck.view(nck, N), gamma)
        torch.cuda.synchronize()
        t = time.perf_counter() - t
        h = diag.cpu().numpy()
        out[name] = {"norm_delta": float((h[:, 0].max() - h[:, 0].min()) / h[:, 0].mean()),
                     "energy_delta": float((h[:, 1].max() - h[:, 1].min()) / h[:, 1].mean()),
                     "energy_0": float(h[0, 1]), "ms_run_plus_diagnostics": t * 1e3,
                     "ms_run": t_run * 1e3, "ms_diagnostics": (t - t_run) * 1e3}
        log(f"conservation {name}: norm delta {out[name]['norm_delta']:.2e}, "
            f"energy delta {out[name]['energy_delta']:.2e}, {t * 1e3:.1f} ms")
        del u, ck
    return out


def bench_convergence(lt, torch, K, W):
    """Time-step convergence on a lattice of the paper's Table 1 (d = 3,
    n = 2^22, z = (1, 1737355, 261247)) with g1, gamma = 0.5, T = 1, for the
    smooth v1 and the harmonic v2: reference dt = 1/10000, errors for dt = 1/m
    (complex128)."""
    import numpy as np

    import workloads as W_
    Z, n = W_.paper_lattice(3, 1 << 22)
    N = int(n[0])
    num = W_.point_numerators(Z, n)
    gamma = 0.5
    plan = lt.lattice_plan(Z, n)
    dev = torch.device("cuda:0")
    u0 = torch.tensor(W_.paper_g1(num, N, gamma), dtype=torch.complex128, device=dev)
    out = {"workload": "paper Table 1 lattice d=3 n=2^22 z=(1,1737355,261247), minimal-l2 index set, g1, "
                       "gamma=0.5, T=1, reference dt=1e-4, complex128"}
    for name, vfun in (("v1", W_.v_smooth_paper), ("v2", W_.v_harmonic_paper)):
        v = torch.tensor(vfun(num, N), device=dev)

        def solve(m):
            u = u0.clone()
            lt.strang_run(plan, v, u, gamma, 1.0 / m, m)
            return u

        torch.cuda.synchronize()
        t = time.perf_counter()
        ref = solve(10000)
        torch.cuda.synchronize()
        t = time.perf_counter() - t
        ms = [10, 20, 40, 80, 160, 320, 640]
        errs = [float(torch.sqrt(torch.mean(torch.abs(solve(m) - ref) ** 2)).item()) for m in ms]
        orders = [float(np.log2(errs[i] / errs[i + 1])) for i in range(len(ms) - 1)]
        fit = float(np.polyfit(np.log(1.0 / np.asarray(ms, dtype=float)), np.log(errs), 1)[0])
        log(f"convergence {name}: errors {['%.2e' % e for e in errs]}, orders {['%.2f' % o for o in orders]}, "
            f"fitted {fit:.2f}")
        out[name] = {"m": ms, "l2_error": errs, "observed_order": orders, "fitted_order": fit,
                     "reference_run": {"value": N * 10000 / t, "unit": "lattice-point-steps/s", "seconds": t}}
        del ref
    return out


def bench_wide(lt, torch, K, W):
    """The paper's Table 1 lattice d = 6, n = 2^25 (the transform split into
    columns of 4096 and rows of 8192 points) with g1, the smooth v1,
    gamma = 0.5, dt = 1e-3, 100 steps per run."""
    import workloads as W_
    Z, n = W_.paper_lattice(6, 1 << 25)
    N, m, gamma, dt = int(n[0]), 100, 0.5, 1e-3
    t = time.perf_counter()
    plan = lt.lattice_plan(Z, n)
    tplan = time.perf_counter() - t
    info = plan.info
    num = W_.point_numerators(Z, n)
    dev = torch.device("cuda:0")
    v = torch.tensor(W_.v_smooth_paper(num, N), device=dev)
    u0 = W_.paper_g1(num, N, gamma)
    out = {"workload": f"paper Table 1 lattice d=6 n=2^25 z={list(map(int, Z[0]))}, minimal-l2 index set, g1, v1, "
                       f"gamma={gamma}, dt={dt}, {m} steps per run; transform {info['L1']} x {info['L2']}",
           "unit": "lattice-point-steps/s", "plan_seconds": tplan}
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        prec = lt.LT_C64 if name == "c64" else lt.LT_C128
        kernels = lt.lattice_plan_autotune(plan, prec, reps=3)
        u = torch.tensor(u0, dtype=dtype, device=dev)
        work = torch.empty(lt.strang_workspace_size(plan, prec, 1, True), dtype=torch.uint8, device=dev)
        run = lambda: lt.strang_run(plan, v, u, gamma, dt, m, work=work)  # noqa: E731
        sec = wall(run, K, W)
        out[name] = {"value": N * m / sec, "ms_per_run": sec * 1e3, "kernel_variants": list(kernels),
                     "kernels": kernel_summary(lt, run, 1)}
        log(f"wide {name}: {N * m / sec:.3e} pt-steps/s, {sec * 1e3:.1f} ms per {m}-step run")
        del u, work
        torch.cuda.empty_cache()
    return out


def bench_hbm(lt, torch, K, W):
    """The benchmark lattice with a batch of states sharing v (16 in complex64,
    8 in complex128: about 500 and 450 MB of states, transform buffers and
    tables, beyond the 256 MB Infinity Cache), 100 steps: the same
    steady-state passes as the headline run, with a working set that has to
    stream from HBM."""
    import numpy as np

    import workloads as W_
    inst = W_.cross_d6_n1048573(steps=1)
    plan = lt.lattice_plan(inst.Z, inst.n, inst.I)
    info = plan.info
    dev = torch.device("cuda:0")
    N, m = inst.N, 100
    v = torch.tensor(inst.v, dtype=torch.float64, device=dev)
    out = {"workload": f"benchmark lattice d=6 N={N}, batches of 16 (complex64) and 8 (complex128) states "
                       f"sharing v, {m} steps per run",
           "unit": "lattice-point-steps/s"}
    for name, dtype, S, B in (("c64", torch.complex64, 8, 16), ("c128", torch.complex128, 16, 8)):
        prec = lt.LT_C64 if name == "c64" else lt.LT_C128
        lt.lattice_plan_autotune(plan, prec, reps=5)
        u = torch.tensor(np.tile(inst.u0, (B, 1)), dtype=dtype, device=dev)
        work = torch.empty(lt.strang_workspace_size(plan, prec, B, True), dtype=torch.uint8, device=dev)
        run = lambda: lt.strang_run(plan, v, u, inst.gamma, inst.dt, m, work=work)  # noqa: E731
        sec = wall(run, K, W)
        ks = kernel_summary(lt, run, 1)
        col_b, row_b = pass_bytes(info, N, m, S)
        L = info["fft_len"]
        col_steady = B * (2 * L * S) + 16 * N   # the shared table is read once per launch
        row_steady = B * (2 * L * S) + 16 * L
        resident = B * (N * S + L * S) + 16 * N + 16 * L
        out[name] = {"value": B * N * m / sec, "states": B, "ms_per_run": sec * 1e3,
                     "working_set_MB": resident / 1e6,
                     "column_us": ks["column"]["avg_us"], "row_us": ks["row"]["avg_us"],
                     "column_GBs": col_steady / (ks["column"]["avg_us"] * 1e-6) / 1e9,
                     "row_GBs": row_steady / (ks["row"]["avg_us"] * 1e-6) / 1e9}
        log(f"hbm {name}: {B * N * m / sec:.3e} pt-steps/s, working set {resident / 1e6:.0f} MB, column "
            f"{out[name]['column_GBs']:.0f} GB/s, row {out[name]['row_GBs']:.0f} GB/s")
        del u, work
        torch.cuda.empty_cache()
    return out


def bench_initial(lt, torch, K, W):
    """The initial discretization error of Sec. 3.4 for the paper's g1 with
    gamma = 1 on Table 1 lattices (d = 2, n = 2^18 and 2^20; d = 3, n = 2^22):
    e_total^2 = ||g||^2 - sum_A |ghat|^2 + sum_A |ghat - ghat_a|^2, the key sums
    from lattice_projection_error (complex128), the exact coefficients of g1
    from 1-D Gauss-Legendre integrals."""
    import numpy as np

    import workloads as W_
    gamma = 1.0
    out = {"workload": "paper g1 with gamma = 1 on Table 1 lattices; complex128 lattice DFT and key sums",
           "unit": "e_total (L2 error of the initial projection)"}
    for d, n in ((2, 1 << 18), (2, 1 << 20), (3, 1 << 22)):
        Z, nn = W_.paper_lattice(d, n)
        plan = lt.lattice_plan(Z, nn)
        _, _, h = lt.lattice_plan_keys(plan)
        kmax = int(np.abs(h).max()) + 1
        tables, norm2 = W_.paper_g1_coefficients(d, gamma, kmax, nodes=max(4096, 4 * kmax))
        ghat = torch.tensor(W_.coefficients_at(h.astype(np.int64), tables), device="cuda:0")
        num = W_.point_numerators(Z, nn)
        u = torch.tensor(W_.paper_g1(num, n, gamma, normalize=False), device="cuda:0")
        work = torch.empty(lt.lattice_projection_error_workspace_size(plan, lt.LT_C128, 1), dtype=torch.uint8,
                           device="cuda:0")
        call = lambda: lt.lattice_projection_error(plan, u, ghat, work=work)  # noqa: E731
        sec = wall(call, K, W)
        s0, s1 = call().cpu().numpy()[0]
        e2 = norm2 - s0 + s1
        out[f"d{d}_n{n}"] = {"e_total": float(np.sqrt(max(e2, 0.0))), "norm2": norm2, "outside_A": norm2 - s0,
                             "aliasing_on_A": float(s1), "ms_per_call": sec * 1e3}
        log(f"initial d={d} n=2^{n.bit_length() - 1}: e_total {np.sqrt(max(e2, 0.0)):.3e} "
            f"(outside A {norm2 - s0:.2e}, on A {s1:.2e}), {sec * 1e3:.2f} ms per call")
        del u, ghat, work
    return out


def bench_splitting(lt, torch, K, W):
    """Higher-order splitting and time-dependent potentials (the two method
    variants of Sec. 5) on the benchmark lattice (d = 6, N = 1048573):
    splitting_run with the fourth-order triple jump, 300 composed steps of
    dt = 1e-3 (900 Strang substeps), with v fixed and with the amplitude-
    modulated v(x, t) = (1 + 0.5 sin(20 t)) v(x); and the accuracy of order 2
    against order 4 at equal cost (900 substeps over T = 0.9) against an
    order-4 reference with dt / 10 (complex128)."""
    import numpy as np

    import workloads as W_
    inst = W_.cross_d6_n1048573(steps=1)
    plan = lt.lattice_plan(inst.Z, inst.n, inst.I)
    dev = torch.device("cuda:0")
    N, m, dt = inst.N, 300, 1e-3
    v = torch.tensor(inst.v, dtype=torch.float64, device=dev)
    out = {"workload": f"benchmark lattice d=6 N={N}, gamma={inst.gamma}, order 4 (triple jump), {m} steps "
                       f"of dt={dt} (3 substeps each); time-dependent: v(x,t) = (1 + 0.5 sin 20t) v(x)",
           "unit": "lattice-point-steps/s (composed fourth-order steps)"}
    f = lambda t: 0.5 * np.sin(20.0 * np.asarray(t))  # noqa: E731
    for name, dtype in (("c64", torch.complex64), ("c128", torch.complex128)):
        prec = lt.LT_C64 if name == "c64" else lt.LT_C128
        lt.lattice_plan_autotune(plan, prec, reps=10)
        u = torch.tensor(inst.u0, dtype=dtype, device=dev)
        work = torch.empty(lt.splitting_workspace_size(plan, prec, 1, True, 4), dtype=torch.uint8, device=dev)
        fk = f(lt.splitting_times(4, m, 0.0, dt))
        fixed = lambda: lt.splitting_run(plan, v, u, inst.gamma, dt, m, order=4, work=work)  # noqa: E731
        tdv = lambda: lt.splitting_run(plan, v, u, inst.gamma, dt, m, order=4, v1=v, f=fk,  # noqa: E731
                                       work=work)
        tf, tt = wall(fixed, K, W), wall(tdv, K, W)
        out[name] = {"value": N * m / tf, "ms_per_run": tf * 1e3,
                     "time_dependent": {"value": N * m / tt, "ms_per_run": tt * 1e3},
                     "kernels": kernel_summary(lt, fixed, 1),
                     "time_dependent_kernels": kernel_summary(lt, tdv, 1)}
        log(f"splitting {name}: order 4 {N * m / tf:.3e} pt-steps/s ({tf * 1e3:.1f} ms), "
            f"time-dependent {N * m / tt:.3e} ({tt * 1e3:.1f} ms)")
        del u, work
    # accuracy at equal cost: 900 substeps over T = 0.9 as order 2 (900 steps) or
    # order 4 (300 steps); reference: order 4 with 3000 steps
    u0 = torch.tensor(inst.u0, dtype=torch.complex128, device=dev)

    def solve(order, steps):
        u = u0.clone()
        lt.splitting_run(plan, v, u, inst.gamma, 0.9 / steps, steps, order=order)
        return u
    ref = solve(4, 3000)
    e2 = float(torch.linalg.vector_norm(solve(2, 900) - ref) / torch.linalg.vector_norm(ref))
    e4 = float(torch.linalg.vector_norm(solve(4, 300) - ref) / torch.linalg.vector_norm(ref))
    out["equal_cost_accuracy"] = {"substeps": 900, "T": 0.9, "order2_rel_l2": e2, "order4_rel_l2": e4}
    log(f"splitting equal cost (900 substeps, T=0.9): order 2 rel err {e2:.2e}, order 4 {e4:.2e}")
    return out


def cpu_baseline(inst, seconds):
    import numpy as np

    import oracle as O
    t = time.perf_counter()
    _, s, _ = O.index_set(inst.Z, inst.n, inst.I)
    log(f"oracle index set {time.perf_counter() - t:.1f}s")
    u = inst.u0.copy()
    steps, spent = 0, 0.0
    while spent < seconds:
        t = time.perf_counter()
        u = O.strang_run(inst.n, s, inst.v, u, inst.gamma, inst.dt, 1)
        spent += time.perf_counter() - t
        steps += 1
    return {"value": inst.N * steps / spent, "unit": "lattice-point-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} Strang steps of the benchmark workload (N={inst.N}, d=6) in the FP64 "
                      f"C oracle (radix-2 chirp-z FFTs), single thread, {spent:.1f}s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--time-steps", type=int, default=1000, help="Strang steps per run")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c128", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the companion workloads")
    ap.add_argument("--only", choices=["batched", "rank2", "adjoint", "conservation", "convergence", "splitting",
                                       "wide", "hbm", "initial"],
                    help="run one companion workload alone (profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device to device (counter calibration for the traffic figure)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(32 * 1024 * 1024, dtype=torch.complex64, device="cuda:0")
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": a.numel() * 8,
                          "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(a single lattice state does not shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1808_06357_amd as lt
    import workloads as W

    extras = {"batched": bench_batched, "rank2": bench_rank2, "adjoint": bench_adjoint,
              "conservation": bench_conservation, "convergence": bench_convergence,
              "splitting": bench_splitting, "wide": bench_wide, "hbm": bench_hbm,
              "initial": bench_initial}
    if args.only:
        print(json.dumps({args.only: extras[args.only](lt, torch, args.steps, args.warmup)}), flush=True)
        return

    t = time.perf_counter()
    inst = W.cross_d6_n1048573(steps=args.time_steps)
    log(f"inputs {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    plan = lt.lattice_plan(inst.Z, inst.n, inst.I)
    info = plan.info
    log(f"plan {time.perf_counter() - t:.1f}s: L={info['fft_len']} L1={info['L1']} L2={info['L2']}")
    N, m = inst.N, inst.steps
    dev = torch.device("cuda:0")
    v = torch.tensor(inst.v, dtype=torch.float64, device=dev)

    results = {}
    for name, dtype, S in (("c64", torch.complex64, 8), ("c128", torch.complex128, 16)):
        if name == "c128" and args.no_c128:
            continue
        u = torch.tensor(inst.u0, dtype=dtype, device=dev)
        prec = lt.LT_C64 if name == "c64" else lt.LT_C128
        kernels = lt.lattice_plan_autotune(plan, prec, reps=20)
        log(f"{name}: autotuned kernel variants (column, row) = {kernels}")
        work = torch.empty(lt.strang_workspace_size(plan, prec, 1, True), dtype=torch.uint8, device=dev)
        # one run from u0 for the accuracy indicators
        lt.strang_run(plan, v, u, inst.gamma, inst.dt, m, work=work)
        torch.cuda.synchronize()
        uT = u.cpu().numpy().astype(np.complex128)
        elapsed, kinds, instrumented = time_runs(lt, torch, plan, v, u, work, inst, args.steps, args.warmup)
        col_b, row_b = pass_bytes(info, N, m, S)
        per_kind = {}
        for kname, bytes_list in (("column", col_b), ("row", row_b)):
            launches, ms = kinds[kname]
            avg_ms = ms / max(launches, 1)
            avg_bytes = sum(bytes_list) / len(bytes_list)
            per_kind[kname] = {"launches": launches, "total_ms": ms, "avg_us": avg_ms * 1e3,
                               "bytes_per_launch": avg_bytes,
                               "achieved_GBs": avg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None}
        results[name] = {"elapsed": elapsed, "kinds": per_kind, "uT": uT, "kernels": kernels,
                         "instrumented_ms_per_run": instrumented / args.steps * 1e3,
                         "value": N * m * args.steps / elapsed, "ms_per_step": elapsed / args.steps * 1e3}
        log(f"{name}: {results[name]['value']:.3e} pt-steps/s, {results[name]['ms_per_step']:.2f} ms/run; "
            + ", ".join(f"{k}: {v_['avg_us']:.1f} us/launch {v_['achieved_GBs'] or 0:.0f} GB/s"
                        for k, v_ in per_kind.items()))
        if name == "c64":
            # the same run captured once into a HIP graph and replayed (a
            # companion figure: a capture failure is recorded, not fatal)
            try:
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    lt.strang_run(plan, v, u, inst.gamma, inst.dt, m, work=work)
                g_sec = wall(g.replay, args.steps, args.warmup)
                results[name]["graph"] = {"eager_ms_per_run": elapsed / args.steps * 1e3,
                                          "graph_ms_per_run": g_sec * 1e3, "passes_per_run": 2 * m + 1}
                log(f"{name}: graph replay {g_sec * 1e3:.2f} ms/run against eager "
                    f"{elapsed / args.steps * 1e3:.2f}")
                del g
            except RuntimeError as e:
                torch.cuda.synchronize()
                results[name]["graph"] = {"error": str(e)[:200]}
                log(f"{name}: graph capture failed: {e}")
        del work, u
        torch.cuda.empty_cache()

    head = results["c64"]
    dom_name = max(head["kinds"], key=lambda k: head["kinds"][k]["total_ms"])
    dom = head["kinds"][dom_name]
    acc = {"norm2_after_run_c64": float(np.mean(np.abs(head["uT"]) ** 2))}
    if "c128" in results:
        ref = results["c128"]["uT"]
        acc["c64_vs_c128_rel_l2_after_run"] = float(np.linalg.norm(head["uT"] - ref) / np.linalg.norm(ref))
        acc["norm2_after_run_c128"] = float(np.mean(np.abs(ref) ** 2))

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "lattice-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "rank-1 lattice d=6 N=1048573 (prime; chirp-z length "
                               f"{info['fft_len']}={info['L1']}x{info['L2']}), hyperbolic cross R=10 "
                               "+ minimal-l2 completion, gamma=0.05, dt=1e-3, "
                               f"{m} Strang steps per run, complex64 with FP64 phases",
                   "N": N, "d": 6, "time_steps_per_run": m, "fft_len": info["fft_len"]},
        "roofline": {"bound": "hbm", "kernel": f"k_{'row' if dom_name == 'row' else 'col'} (c64)",
                     "achieved": dom["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom["achieved_GBs"] / HBM_PEAK_GBS if dom["achieved_GBs"] else None,
                     "traffic": pmc_traffic() if dom_name == "column" else None,
                     "traffic_note": "HBM bytes per steady-state column launch from rocprofv3 FETCH_SIZE x2 + "
                                     "WRITE_SIZE x1 (factors from a 256 MiB copy)",
                     "avg_launch_us": dom["avg_us"],
                     "bytes_per_launch": dom["bytes_per_launch"],
                     "instrumented_ms_per_run": head["instrumented_ms_per_run"]},
        "bytes_per_point_step": {
            name_: {"algorithmic_floor": 4 * S_,
                    "pass_model": (sum(pass_bytes(info, N, m, S_)[0]) + sum(pass_bytes(info, N, m, S_)[1])) / (N * m),
                    "counter": (pmc_traffic("column") * (m + 1) + pmc_traffic("row") * m) / (N * m)
                    if (name_ == "c64" and pmc_traffic("column") and pmc_traffic("row")) else None,
                    "note": "floor: state read and written once plus the two diagonal tables at S bytes each; "
                            "pass model: every launch of the two-pass convolution schedule; counter: the "
                            "steady-state column and row passes' measured HBM bytes (rocprofv3 FETCH_SIZE / "
                            "WRITE_SIZE, copy-calibrated), complex64"}
            for name_, S_ in (("c64", 8), ("c128", 16)) if name_ in results},
        "kernels_c64": head["kinds"],
        "kernel_variants": {k: list(r_["kernels"]) for k, r_ in results.items()},
        "graph_c64": head.get("graph"),
        "accuracy": acc,
    }
    if "c128" in results:
        c = results["c128"]
        out["c128"] = {"value": c["value"], "ms_per_step": c["ms_per_step"], "kernels": c["kinds"]}
    if not args.no_extra:
        for name, fn in extras.items():
            out[name] = fn(lt, torch, args.steps, args.warmup)
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
