"""Seeded sweep of lattice shapes across every layout the planner picks, each
run through strang_run (C-ABI) and compared with the FP64 oracle on the same
inputs, in both precisions: tiny lattices, primes and composites on both
sides of the one-workgroup limit (resident vs two passes, direct vs chirp-z),
powers of two up to 2^20, rank-2 tensors (resident, two-pass, non-power-of-two,
and the transposed layout of tensors with long columns); batches of 1 to 3
states, shared and per-state potentials, both signs of dt."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import TOL, gpu_run, rel

pytestmark = pytest.mark.gpu

RANK1 = [(2, 2), (3, 3), (7, 2), (64, 3), (97, 4), (4093, 3), (4096, 3), (4097, 3), (4100, 2), (4116, 3),
         (6561, 2), (65536, 4), (131071, 3), (262144, 5), (1 << 20, 3), (1000003, 4)]
RANK2 = [(8, 4, 2), (256, 16, 3), (1536, 96, 3), (1024, 1024, 3), (2048, 64, 4), (4096, 512, 3), (2048, 1024, 3)]


def _inputs(g, num, N, d, batch, shared):
    if shared:
        v = W.cosine_series(d, 8, g).at(num, N)
    else:
        v = np.stack([W.cosine_series(d, 8, g).at(num, N) for _ in range(batch)])
    u0 = np.stack([W.seeded_packet(num, N, g) for _ in range(batch)])
    return v, (u0[0] if batch == 1 else u0)


def _run_case(lt, Z, n, I, seed):
    g = np.random.default_rng(seed)
    N = int(np.prod(n))
    d = Z.shape[1]
    batch = int(g.integers(1, 4))
    shared = bool(g.integers(0, 2))
    steps = int(g.integers(3, 8))
    gamma = float(g.uniform(0.02, 0.2))
    dt = float(g.choice([-1.0, 1.0]) * g.uniform(1e-3, 5e-3))
    num = W.point_numerators(Z, n)
    v, u0 = _inputs(g, num, N, d, batch, shared)
    plan = lt.lattice_plan(Z, n, I)
    info = plan.info
    print(f"sweep n={list(n)} d={d} batch={batch} shared={shared} steps={steps} dt={dt:+.2e} "
          f"passes={info['passes']} L={info['fft_len']} {info['L1']}x{info['L2']} "
          f"chirp-z={info['bluestein']} swapped={info['swapped']}", flush=True)
    _, s, _ = O.index_set(Z, n, I)
    ref = O.strang_run(n, s, v, u0, gamma, dt, steps)
    for prec in ("c128", "c64"):
        e = rel(gpu_run(lt, plan, v, u0, gamma, dt, steps, prec), ref)
        print(f"  {prec} rel_l2={e:.2e}", flush=True)
        assert e < TOL[prec], (prec, e)


@pytest.mark.parametrize("N,d", RANK1)
def test_sweep_rank1(lt, N, d):
    g = np.random.default_rng(1000 + N)
    z = np.ones(d, dtype=np.int64) if N < 4 else W.korobov_good(N, d, g)
    _run_case(lt, z.reshape(1, -1), np.array([N]), None, 2000 + N)


@pytest.mark.parametrize("n1,n2,d", RANK2)
def test_sweep_rank2(lt, n1, n2, d):
    H = W.hyperbolic_cross(d, 1)
    Z = W.cbc_rank2(H, n1, n2, np.random.default_rng(n1 + 7 * n2))
    _run_case(lt, Z, np.array([n1, n2]), H, 3000 + n1 + n2)
