"""Per-step sums fused into the passes (strang_run_sums, Sec. 3.3): the norm
(1/N) sum |u_j|^2 and the potential term (1/(gamma N)) sum v |u_j|^2 of the
energy at every step boundary j = 0..m, against the FP64 oracle's history,
on every schedule (one workgroup, two passes on smooth lengths, the chirp-z
convolution form and the chirp-z pair form of prime N, a transposed rank-2
tensor), shared and per-state v; the state itself equals strang_run's."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-11, "c64": 2e-5}


def rank1_case(N, d, seed, batch, shared, steps):
    g = np.random.default_rng(seed)
    z = W.korobov(N, d, g)
    Z, n = z.reshape(1, -1), np.array([N])
    num = W.point_numerators(Z, n)
    if shared:
        v = W.cosine_series(d, 16, g).at(num, N)
    else:
        v = np.stack([W.cosine_series(d, 16, g).at(num, N) for _ in range(batch)])
    u0 = np.stack([W.seeded_packet(num, N, g) for _ in range(batch)])
    return Z, n, None, v, u0


def rank2_case(n1, n2, d, seed, batch):
    H = W.hyperbolic_cross(d, 1)
    Z = W.cbc_rank2(H, n1, n2, np.random.default_rng(seed))
    n = np.array([n1, n2])
    num = W.point_numerators(Z, n)
    g = np.random.default_rng(seed + 1)
    v = W.cosine_series(d, 16, g).at(num, n1 * n2)
    u0 = np.stack([W.seeded_packet(num, n1 * n2, g) for _ in range(batch)])
    return Z, n, H, v, u0


CASES = [
    # (name, builder, gamma, dt, steps)
    ("resident_N1031", lambda: rank1_case(1031, 2, 1, 2, False, 0), 0.1, 1e-2, 17),
    ("smooth_N16384", lambda: rank1_case(1 << 14, 5, 2, 1, True, 0), 0.5, 1e-2, 23),
    ("chirpz_conv_N65521", lambda: rank1_case(65521, 4, 3, 2, True, 0), 0.05, 2e-3, 12),
    ("chirpz_pair_N65521", lambda: rank1_case(65521, 4, 4, 1, True, 0), 0.05, 2e-3, 3),
    ("composite_N61440", lambda: rank1_case(61440, 3, 5, 2, False, 0), 0.05, 2e-3, 9),
    ("rank2_swapped_2048x64", lambda: rank2_case(2048, 64, 4, 71, 2), 0.05, 2e-3, 11),
]


@pytest.mark.parametrize("name,build,gamma,dt,steps", CASES, ids=[c[0] for c in CASES])
def test_step_sums_against_oracle_history(lt, name, build, gamma, dt, steps):
    import torch
    Z, n, H, v, u0 = build()
    plan = lt.lattice_plan(Z, n, H)
    _, s, _ = O.index_set(Z, n, H)
    ref_u, hist = O.strang_run(n, s, v, u0, gamma, dt, steps, history=True)
    ref = np.stack([hist[:, :, 0], hist[:, :, 2]], axis=-1)
    for prec, dtype in (("c128", torch.complex128), ("c64", torch.complex64)):
        vv = torch.tensor(v, dtype=torch.float64, device="cuda")
        u = torch.tensor(u0, dtype=dtype, device="cuda")
        sums = lt.strang_run_sums(plan, vv, u, gamma, dt, steps)
        u_plain = torch.tensor(u0, dtype=dtype, device="cuda")
        lt.strang_run(plan, vv, u_plain, gamma, dt, steps)
        got = sums.cpu().numpy()
        # the potential term can pass through zero: its error is taken
        # relative to the bound max|v| ||u||^2 / gamma
        scale = np.stack([ref[..., 0], ref[..., 0] * np.max(np.abs(v)) / gamma], axis=-1)
        e = float(np.max(np.abs(got - ref) / scale))
        eu = float(np.linalg.norm(u.cpu().numpy() - ref_u) / np.linalg.norm(ref_u))
        print(f"  {name} {prec} (info {plan.info['passes']} passes, chirp-z {plan.info['bluestein']}): "
              f"max rel error of the step sums {e:.2e}, state {eu:.2e}", flush=True)
        assert got.shape == (u0.shape[0], steps + 1, 2)
        assert e < TOL[prec], (name, prec, e)
        # the fused sums leave the state as strang_run computes it
        assert torch.equal(u, u_plain), name


def test_step_sums_workspace_and_graph_replay(lt):
    """With a caller workspace the call only enqueues kernels: captured into a
    HIP graph, every replay advances the state by m steps and rewrites the
    sums exactly as an eager call on the same input does."""
    import torch
    Z, n, H, v, u0 = rank1_case(65521, 4, 9, 1, True, 0)
    gamma, dt, steps = 0.05, 2e-3, 8
    plan = lt.lattice_plan(Z, n, H)
    vv = torch.tensor(v, device="cuda")
    u = torch.tensor(u0, dtype=torch.complex64, device="cuda")
    nb = lt.strang_run_sums_workspace_size(plan, lt.LT_C64, 1, True, steps)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    sums = torch.empty((1, steps + 1, 2), dtype=torch.float64, device="cuda")
    lt.strang_run_sums(plan, vv, u.clone(), gamma, dt, steps, sums=sums, work=work)  # builds the tables
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    ug = u.clone()
    with torch.cuda.graph(g):
        lt.strang_run_sums(plan, vv, ug, gamma, dt, steps, sums=sums, work=work)
    torch.cuda.synchronize()
    ug.copy_(u)
    ue = u.clone()
    for rep in range(3):
        start = ug.clone()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ue.copy_(start)
        se = lt.strang_run_sums(plan, vv, ue, gamma, dt, steps)
        torch.cuda.synchronize()
        print(f"  replay {rep}: state equal {torch.equal(ug, ue)}, sums equal {torch.equal(sums, se)}", flush=True)
        assert torch.equal(ug, ue), rep
        assert torch.equal(sums, se), rep
    del g


def test_step_sums_zero_steps_and_errors(lt):
    import torch
    Z, n, H, v, u0 = rank1_case(1031, 2, 1, 2, True, 0)
    plan = lt.lattice_plan(Z, n, H)
    _, s, _ = O.index_set(Z, n, H)
    _, hist = O.strang_run(n, s, v, u0, 0.1, 1e-2, 0, history=True)
    vv = torch.tensor(v, device="cuda")
    u = torch.tensor(u0, dtype=torch.complex128, device="cuda")
    got = lt.strang_run_sums(plan, vv, u, 0.1, 1e-2, 0).cpu().numpy()
    assert np.max(np.abs(got[:, 0, 0] - hist[:, 0, 0])) < 1e-13
    assert np.max(np.abs(got[:, 0, 1] - hist[:, 0, 2])) < 1e-12 * np.max(np.abs(v)) / 0.1
    with pytest.raises(Exception):
        lt.strang_run_sums(plan, vv, u, -0.1, 1e-2, 3)


@pytest.mark.parametrize("cv", [1, 5])
def test_step_sums_on_each_column_geometry(lt, cv):
    """The step sums on a forced column geometry: variant 1 (16 elements per
    thread, first radix 16 on the 256-point columns of the prime N = 32749's
    2^16-point convolution, so v is loaded in chunks) and variant 5 (8
    elements), both precisions, per-state v, against the oracle's history;
    the state equals strang_run's on the same geometry."""
    import torch
    Z, n, H, v, u0 = rank1_case(32749, 4, 3, 2, False, 0)
    gamma, dt, steps = 0.05, 2e-3, 12
    plan = lt.lattice_plan(Z, n, H)
    assert plan.info["L1"] == 256 and plan.info["passes"] == 2
    _, s, _ = O.index_set(Z, n, H)
    ref_u, hist = O.strang_run(n, s, v, u0, gamma, dt, steps, history=True)
    ref = np.stack([hist[:, :, 0], hist[:, :, 2]], axis=-1)
    for prec, dtype in (("c128", torch.complex128), ("c64", torch.complex64)):
        lt.lattice_plan_set_kernels(plan, lt.LT_C128 if prec == "c128" else lt.LT_C64, cv, 1)
        vv = torch.tensor(v, dtype=torch.float64, device="cuda")
        u = torch.tensor(u0, dtype=dtype, device="cuda")
        sums = lt.strang_run_sums(plan, vv, u, gamma, dt, steps)
        u_plain = torch.tensor(u0, dtype=dtype, device="cuda")
        lt.strang_run(plan, vv, u_plain, gamma, dt, steps)
        got = sums.cpu().numpy()
        scale = np.stack([ref[..., 0], ref[..., 0] * np.max(np.abs(v)) / gamma], axis=-1)
        e = float(np.max(np.abs(got - ref) / scale))
        print(f"  variant {cv} {prec}: max rel error of the step sums {e:.2e}", flush=True)
        assert e < TOL[prec], (cv, prec, e)
        assert torch.equal(u, u_plain), (cv, prec)
