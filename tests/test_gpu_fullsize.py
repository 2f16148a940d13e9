"""Full-size parity for the benchmark workload (d = 6, N = 1048573, 1000
steps) in the launch configuration bench.py times: the GPU state is compared
with the FP64 oracle at stored sample points (tests/golden/, written by
make_cross_d6_n1048573_golden.py, which calls only the oracle) and checked against
properties that hold at any size (norm, reversibility)."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "cross_d6_n1048573_oracle_samples.npz")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def case(lt):
    import torch
    gold = np.load(GOLD)
    inst = W.cross_d6_n1048573(steps=1000)
    assert np.array_equal(inst.Z[0], gold["z"]), "seeded CBC search changed"
    plan = lt.lattice_plan(inst.Z, inst.n, inst.I)
    v = torch.tensor(inst.v, dtype=torch.float64, device="cuda")
    return inst, plan, v, gold


@pytest.mark.parametrize("prec,tol", [("c128", 1e-11), ("c64", 1e-4)])
def test_cross_d6_n1048573_against_oracle_samples(lt, case, prec, tol):
    import torch
    inst, plan, v, gold = case
    dtype = torch.complex128 if prec == "c128" else torch.complex64
    p = lt.LT_C128 if prec == "c128" else lt.LT_C64
    lt.lattice_plan_autotune(plan, p, reps=3)
    u = torch.tensor(inst.u0, dtype=dtype, device="cuda")
    idx = gold["idx"]
    lt.strang_run(plan, v, u, inst.gamma, inst.dt, 100)
    u100 = u.cpu().numpy().astype(np.complex128)
    lt.strang_run(plan, v, u, inst.gamma, inst.dt, 900)
    u1000 = u.cpu().numpy().astype(np.complex128)
    e100 = rel(u100[idx], gold["u100"])
    e1000 = rel(u1000[idx], gold["u1000"])
    n1000 = np.mean(np.abs(u1000) ** 2)
    print(f"{prec}: sampled rel L2 at step 100 {e100:.2e}, step 1000 {e1000:.2e}, "
          f"norm^2 {n1000:.15f} (oracle {float(gold['norm2_1000']):.15f})", flush=True)
    assert e100 < tol and e1000 < tol
    # |(||a||^2 - ||b||^2)| <= ||a - b|| (||a|| + ||b||): the L2 tolerance bounds the norm gap
    assert abs(n1000 - float(gold["norm2_1000"])) < 2.0 * tol


def test_cross_d6_n1048573_reversible_c128(lt, case):
    """1000 steps forward, then 1000 with -dt: back to u0 (symmetric scheme)."""
    import torch
    inst, plan, v, _ = case
    u = torch.tensor(inst.u0, dtype=torch.complex128, device="cuda")
    lt.strang_run(plan, v, u, inst.gamma, inst.dt, 1000)
    lt.strang_run(plan, v, u, inst.gamma, -inst.dt, 1000)
    assert rel(u.cpu().numpy(), inst.u0) < 1e-11


GOLD3 = os.path.join(os.path.dirname(__file__), "golden", "rank2_d10_n4096x256_oracle_samples.npz")


@pytest.fixture(scope="module")
def case3(lt):
    import torch
    gold = np.load(GOLD3)
    inst = W.rank2_d10_n4096x256()
    assert np.array_equal(inst.Z, gold["Z"]), "seeded rank-2 CBC search changed"
    plan = lt.lattice_plan(inst.Z, inst.n, inst.I)
    v = torch.tensor(inst.v, dtype=torch.float64, device="cuda")
    return inst, plan, v, gold


@pytest.mark.parametrize("prec,tol", [("c128", 1e-11), ("c64", 1e-4)])
def test_rank2_d10_n4096x256_rank2_against_oracle_samples(lt, case3, prec, tol):
    """Rank-2 lattice n = (4096, 256), d = 10, 500 steps, autotuned kernels."""
    import torch
    inst, plan, v, gold = case3
    dtype = torch.complex128 if prec == "c128" else torch.complex64
    p = lt.LT_C128 if prec == "c128" else lt.LT_C64
    lt.lattice_plan_autotune(plan, p, reps=3)
    u = torch.tensor(inst.u0, dtype=dtype, device="cuda")
    idx = gold["idx"]
    lt.strang_run(plan, v, u, inst.gamma, inst.dt, 100)
    u100 = u.cpu().numpy().astype(np.complex128)
    lt.strang_run(plan, v, u, inst.gamma, inst.dt, 400)
    u500 = u.cpu().numpy().astype(np.complex128)
    e100, e500 = rel(u100[idx], gold["u100"]), rel(u500[idx], gold["u500"])
    n500 = np.mean(np.abs(u500) ** 2)
    print(f"rank-2 {prec}: sampled rel L2 step 100 {e100:.2e}, step 500 {e500:.2e}, norm^2 {n500:.15f}",
          flush=True)
    assert e100 < tol and e500 < tol
    assert abs(n500 - float(gold["norm2_500"])) < 2.0 * tol


def test_rank2_d10_n4096x256_reversible_c128(lt, case3):
    import torch
    inst, plan, v, _ = case3
    u = torch.tensor(inst.u0, dtype=torch.complex128, device="cuda")
    lt.strang_run(plan, v, u, inst.gamma, inst.dt, 500)
    lt.strang_run(plan, v, u, inst.gamma, -inst.dt, 500)
    assert rel(u.cpu().numpy(), inst.u0) < 1e-11
