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
throughput, the FP64 oracle timed on the host, and accuracy indicators.
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
    """Algorithmic bytes of every column-pass and row-pass launch of one run
    (two-pass chirp-z schedule): state read + write once per pass, plus the
    tables the pass reads."""
    L = plan_info["fft_len"]
    col = [N * S + 8 * N + L * S]                 # first: u, v in; transform out
    col += [(2 * L + N) * S] * (2 * m - 1)        # merged P^2 and kinetic passes
    col += [L * S + N * S + 8 * N]                # last: transform in, v, u out
    row = [3 * L * S] * (2 * m)                   # state in/out + kernel spectrum
    return col, row


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
              "(a single lattice state does not shard; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1808_06357_amd as lt
    import workloads as W

    t = time.perf_counter()
    inst = W.config1(steps=args.time_steps)
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
                     "traffic": None, "avg_launch_us": dom["avg_us"],
                     "bytes_per_launch": dom["bytes_per_launch"],
                     "instrumented_ms_per_run": head["instrumented_ms_per_run"]},
        "kernels_c64": head["kinds"],
        "kernel_variants": {k: list(r_["kernels"]) for k, r_ in results.items()},
        "accuracy": acc,
    }
    if "c128" in results:
        c = results["c128"]
        out["c128"] = {"value": c["value"], "ms_per_step": c["ms_per_step"], "kernels": c["kinds"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
