"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle on the
same seeded inputs.  Tolerances (relative L2 over all points): complex128
1e-11, complex64 1e-4."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-11, "c64": 1e-4}


def _torch():
    import torch
    return torch


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def dtype_np(prec):
    return np.complex128 if prec == "c128" else np.complex64


def _dtype(prec):
    torch = _torch()
    return torch.complex128 if prec == "c128" else torch.complex64


def gpu_run(lt, plan, v, u0, gamma, dt, steps, prec, **kw):
    torch = _torch()
    u = torch.tensor(np.asarray(u0), dtype=_dtype(prec), device="cuda")
    vv = torch.tensor(np.asarray(v), dtype=torch.float64, device="cuda")
    lt.strang_run(plan, vv, u, gamma, dt, steps, **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.complex128)


def korobov_case(N, d, seed, steps, gamma=0.05, dt=2e-3, batch=1, shared=True):
    g = np.random.default_rng(seed)
    z = W.korobov(N, d, g)
    Z, n = z.reshape(1, -1), np.array([N])
    num = W.point_numerators(Z, n)
    if shared:
        v = W.cosine_series(d, 16, g).at(num, N)
    else:
        v = np.stack([W.cosine_series(d, 16, g).at(num, N) for _ in range(batch)])
    u0 = np.stack([W.seeded_packet(num, N, g) for _ in range(batch)])
    if batch == 1:
        u0 = u0[0]
    return Z, n, v, u0, gamma, dt, steps


def check_case(lt, Z, n, v, u0, gamma, dt, steps, precs=("c128", "c64"), I=None, tol_scale=1.0):
    print(f"case N={int(np.prod(n))} r={len(n)} steps={steps} shape={np.shape(u0)}", flush=True)
    plan = lt.lattice_plan(Z, n, I)
    _, s, _ = O.index_set(Z, n, I)
    ref = O.strang_run(n, s, v, u0, gamma, dt, steps)
    for prec in precs:
        got = gpu_run(lt, plan, v, u0, gamma, dt, steps, prec)
        e = rel(got, ref)
        print(f"  {prec} plan={plan.info['passes']}-pass bluestein={plan.info['bluestein']} "
              f"L={plan.info['fft_len']} rel_l2={e:.3e}", flush=True)
        assert e < TOL[prec] * tol_scale, (prec, e)
    return plan


def test_box_d2_n1031_resident(lt):
    c = W.box_d2_n1031()
    check_case(lt, c.Z, c.n, c.v, c.u0, c.gamma, c.dt, c.steps, I=c.I)


def test_smooth_two_pass_composite(lt):
    check_case(lt, *korobov_case(15360, 3, 1, 30))


def test_power_of_two_two_pass(lt):
    check_case(lt, *korobov_case(1 << 16, 4, 2, 20))


def test_bluestein_two_pass(lt):
    check_case(lt, *korobov_case(65521, 4, 3, 20))


def test_bluestein_resident_small_prime(lt):
    check_case(lt, *korobov_case(1999, 3, 4, 25))


def test_tiny_lattices(lt):
    check_case(lt, np.array([[1, 34]]), np.array([55]), *korobov_case(55, 2, 5, 7)[2:])
    Z, n = np.array([[1]]), np.array([2])
    check_case(lt, Z, n, np.array([0.3, -0.2]), np.array([1.0, 0.5j]), 0.2, 0.1, 3)


def test_rank2_resident_and_two_pass(lt):
    for n1, n2, d in [(64, 16, 4), (1024, 64, 5)]:
        H = W.hyperbolic_cross(d, 1)
        Z = W.cbc_rank2(H, n1, n2, np.random.default_rng(n1))
        n = np.array([n1, n2])
        num = W.point_numerators(Z, n)
        N = n1 * n2
        g = np.random.default_rng(7)
        v = W.cosine_series(d, 8, g).at(num, N)
        u0 = W.seeded_packet(num, N, g)
        plan = check_case(lt, Z, n, v, u0, 0.05, 2e-3, 15, I=H)
        assert plan.info["passes"] == (1 if N <= 4096 else 2)


@pytest.mark.parametrize("n1,n2,d", [(4096, 256, 6), (2048, 64, 5)])
def test_rank2_swapped_layout(lt, n1, n2, d):
    """Rank-2 tensors with long columns (n1 >= 2048, n2 <= n1 / 4) run
    transposed: every kernel variant, shared and per-state potentials, a run
    with checkpoints (stored in lattice order) and an autotuned run, against
    the oracle."""
    torch = _torch()
    H = W.hyperbolic_cross(d, 1)
    Z = W.cbc_rank2(H, n1, n2, np.random.default_rng(n1 + n2))
    n = np.array([n1, n2])
    num = W.point_numerators(Z, n)
    N = n1 * n2
    g = np.random.default_rng(17)
    vs = np.stack([W.cosine_series(d, 8, g).at(num, N) for _ in range(2)])
    u0 = np.stack([W.seeded_packet(num, N, g) for _ in range(2)])
    gamma, dt, steps = 0.05, 2e-3, 6
    plan = lt.lattice_plan(Z, n, H)
    assert plan.info["swapped"] == 1
    _, s, _ = O.index_set(Z, n, H)
    refs = {"shared": O.strang_run(n, s, vs[0], u0, gamma, dt, steps),
            "per-state": O.strang_run(n, s, vs, u0, gamma, dt, steps)}
    for cv in (0, 1, 2, 3, 4, 5):
        for rv in (0, 1, 3, 4, 5):
            for prec in ("c128", "c64"):
                p = lt.LT_C128 if prec == "c128" else lt.LT_C64
                lt.lattice_plan_set_kernels(plan, p, cv, rv)
                for kind, v in (("shared", vs[0]), ("per-state", vs)):
                    e = rel(gpu_run(lt, plan, v, u0, gamma, dt, steps, prec), refs[kind])
                    print(f"  rank-2 {n1}x{n2} col={cv} row={rv} {prec} {kind} rel_l2={e:.2e}", flush=True)
                    assert e < TOL[prec], (cv, rv, prec, kind, e)
    # checkpoints: written in lattice order by the transposed run's checkpoint passes
    every = 4
    for prec in ("c128", "c64"):
        dtype = _dtype(prec)
        u = torch.tensor(u0, dtype=dtype, device="cuda")
        ck = torch.empty(lt.num_checkpoints(steps, every) * 2 * N, dtype=dtype, device="cuda")
        lt.strang_run(plan, torch.tensor(vs, device="cuda"), u, gamma, dt, steps, ckpt=ck, ckpt_every=every)
        torch.cuda.synchronize()
        e = rel(u.cpu().numpy().astype(np.complex128), refs["per-state"])
        print(f"  rank-2 {n1}x{n2} with checkpoints {prec} rel_l2={e:.2e}", flush=True)
        assert e < TOL[prec], (prec, e)
        cks = ck.view(-1, 2, N).cpu().numpy().astype(np.complex128)
        assert np.array_equal(cks[0], np.asarray(u0).astype(dtype_np(prec)).astype(np.complex128))
        assert rel(cks[1], O.strang_run(n, s, vs, u0, gamma, dt, every)) < TOL[prec]
        # every kernel variant writes the same checkpoint (general and register-staged passes)
        for cv in (0, 1):
            lt.lattice_plan_set_kernels(plan, lt.LT_C128 if prec == "c128" else lt.LT_C64, cv, 1)
            u = torch.tensor(u0, dtype=dtype, device="cuda")
            ck.zero_()
            lt.strang_run(plan, torch.tensor(vs, device="cuda"), u, gamma, dt, steps, ckpt=ck, ckpt_every=every)
            c1 = ck.view(-1, 2, N)[1].cpu().numpy().astype(np.complex128)
            assert rel(c1, O.strang_run(n, s, vs, u0, gamma, dt, every)) < TOL[prec], (prec, cv)
    for prec, p in (("c64", lt.LT_C64), ("c128", lt.LT_C128)):
        lt.lattice_plan_autotune(plan, p, reps=3)
        e = rel(gpu_run(lt, plan, vs[0], u0, gamma, dt, steps, prec), refs["shared"])
        print(f"  rank-2 {n1}x{n2} autotuned {lt.lattice_plan_get_kernels_batch(plan, p, 2)} {prec} "
              f"rel_l2={e:.2e}", flush=True)
        assert e < TOL[prec], (prec, e)


def test_batch_shared_and_per_state_potential(lt):
    check_case(lt, *korobov_case(4096 * 3, 3, 8, 12, batch=3, shared=True))
    check_case(lt, *korobov_case(65521, 3, 9, 6, batch=2, shared=False))
    check_case(lt, *korobov_case(1031, 2, 10, 9, batch=4, shared=False))


def test_zero_and_one_step(lt):
    torch = _torch()
    Z, n, v, u0, gamma, dt, _ = korobov_case(65521, 3, 11, 1)
    plan = lt.lattice_plan(Z, n)
    got = gpu_run(lt, plan, v, u0, gamma, dt, 0, "c128")
    assert np.array_equal(got, u0)
    _, s, _ = O.index_set(Z, n)
    assert rel(gpu_run(lt, plan, v, u0, gamma, dt, 1, "c128"), O.strang_run(n, s, v, u0, gamma, dt, 1)) < 1e-12
    del torch


def test_reversibility_negative_dt(lt):
    """S(-dt) S(dt) = I (symmetric scheme), on the GPU in complex128."""
    torch = _torch()
    for N in (1031, 65521, 1 << 16):
        Z, n, v, u0, gamma, dt, _ = korobov_case(N, 3, 12, 40)
        plan = lt.lattice_plan(Z, n)
        u = torch.tensor(u0, dtype=torch.complex128, device="cuda")
        vv = torch.tensor(v, device="cuda")
        lt.strang_run(plan, vv, u, gamma, dt, 40)
        lt.strang_run(plan, vv, u, gamma, -dt, 40)
        assert rel(u.cpu().numpy(), u0) < 1e-12


def test_checkpoints_match_shorter_runs(lt):
    torch = _torch()
    for N in (1031, 65521):
        Z, n, v, u0, gamma, dt, _ = korobov_case(N, 3, 13, 1, batch=2, shared=False)
        plan = lt.lattice_plan(Z, n)
        steps, every = 23, 5
        u = torch.tensor(u0, dtype=torch.complex128, device="cuda")
        vv = torch.tensor(v, device="cuda")
        ck = torch.empty(lt.num_checkpoints(steps, every) * 2 * N, dtype=torch.complex128, device="cuda")
        lt.strang_run(plan, vv, u, gamma, dt, steps, ckpt=ck, ckpt_every=every)
        ck = ck.view(-1, 2, N).cpu().numpy()
        _, s, _ = O.index_set(Z, n)
        for c in range(ck.shape[0]):
            ref = O.strang_run(n, s, v, u0, gamma, dt, c * every)
            assert rel(ck[c], ref) < 1e-11, (N, c)


@pytest.mark.parametrize("N,d", [(65521, 4), (1 << 16, 3), (4096 * 64, 3), (8209, 3), (1 << 13, 3),
                                 (1 << 19, 3), (262147, 3)])
def test_every_kernel_variant(lt, N, d):
    """All column/row kernel variants give the oracle's result (the autotuner
    may pick any of them)."""
    Z, n, v, u0, gamma, dt, steps = korobov_case(N, d, 21, 9)
    plan = lt.lattice_plan(Z, n)
    _, s, _ = O.index_set(Z, n)
    ref = O.strang_run(n, s, v, u0, gamma, dt, steps)
    pairs = [(cv, rv) for cv in (0, 1, 2, 3) for rv in (0, 1, 2, 3)] + [(4, 0), (4, 1), (0, 4), (1, 4), (4, 4),
                                                                         (5, 0), (5, 1), (1, 5), (5, 5)]
    for cv, rv in pairs:
        for prec in ("c128", "c64"):
            p = lt.LT_C128 if prec == "c128" else lt.LT_C64
            lt.lattice_plan_set_kernels(plan, p, cv, rv)
            e = rel(gpu_run(lt, plan, v, u0, gamma, dt, steps, prec), ref)
            print(f"  N={N} col={cv} row={rv} {prec} rel_l2={e:.2e}", flush=True)
            assert e < TOL[prec], (cv, rv, prec, e)
    for prec in (lt.LT_C64, lt.LT_C128):
        chosen = lt.lattice_plan_autotune(plan, prec, reps=3)
        assert chosen[0] in range(6) and chosen[1] in range(6)
        assert lt.lattice_plan_get_kernels_batch(plan, prec, 1) == tuple(chosen)
        cm, rm = lt.lattice_plan_get_kernels_batch(plan, prec, 64)
        assert cm in range(6) and rm in range(6)
    # a batch large enough for the many-state choice the autotuner made
    L = plan.info["fft_len"]
    batch = max(2, -(-(1 << 20) // L))
    Z, n, v, u0, gamma, dt, steps = korobov_case(N, d, 22, 5, batch=batch)
    ref = O.strang_run(n, s, v, u0, gamma, dt, steps)
    for prec in ("c128", "c64"):
        p = lt.LT_C128 if prec == "c128" else lt.LT_C64
        e = rel(gpu_run(lt, plan, v, u0, gamma, dt, steps, prec), ref)
        print(f"  N={N} batch={batch} variants={lt.lattice_plan_get_kernels_batch(plan, p, batch)} "
              f"{prec} rel_l2={e:.2e}", flush=True)
        assert e < TOL[prec], (batch, prec, e)


@pytest.mark.parametrize("N,d", [(65521, 4), (8191, 3), (262139, 3)])
def test_chirpz_step_forms(lt, N, d):
    """Prime N: runs of fewer than 4 steps apply the chirp-z DFT pair in every
    step; longer runs apply F^-1 K F as one zero-padded cyclic convolution.
    Both against the oracle, including a run of exactly 4 steps."""
    for steps in (3, 4, 9):
        check_case(lt, *korobov_case(N, d, 30 + steps, steps))
