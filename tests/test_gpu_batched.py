"""strang_run_batched: unrelated problems (own lattice, potential, state,
gamma, dt and step count) advanced in shared launches, against the FP64
oracle per problem and against single-problem runs, through the C-ABI."""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-11, "c64": 1e-4}
GOLD = os.path.join(os.path.dirname(__file__), "golden", "mixed_batch_oracle_samples.npz")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def korobov_problem(N, d, seed, steps, gamma, dt):
    g = np.random.default_rng(seed)
    z = W.korobov(N, d, g)
    Z, n = z.reshape(1, -1), np.array([N])
    num = W.point_numerators(Z, n)
    return dict(Z=Z, n=n, I=None, v=W.cosine_series(d, 16, g).at(num, N), u0=W.seeded_packet(num, N, g),
                gamma=gamma, dt=dt, steps=steps)


def rank2_problem(n1, n2, d, seed, steps, gamma, dt):
    H = W.hyperbolic_cross(d, 1)
    Z = W.cbc_rank2(H, n1, n2, np.random.default_rng(n1))
    n = np.array([n1, n2])
    num = W.point_numerators(Z, n)
    g = np.random.default_rng(seed)
    return dict(Z=Z, n=n, I=H, v=W.cosine_series(d, 8, g).at(num, n1 * n2),
                u0=W.seeded_packet(num, n1 * n2, g), gamma=gamma, dt=dt, steps=steps)


def mixed_problems():
    """One-workgroup problems (smooth 2048, chirp-z 1031, rank-2 64 x 16) and
    two-pass ones (smooth 15360, 2^16, chirp-z 8191 and 65521, rank-2
    1024 x 64), with uneven step counts, a zero-step and a one-step problem."""
    return [
        korobov_problem(2048, 3, 1, 13, 0.07, 2e-3),
        korobov_problem(15360, 4, 2, 9, 0.05, 3e-3),
        korobov_problem(1031, 2, 3, 17, 0.1, 1e-2),
        korobov_problem(8191, 5, 4, 6, 0.03, 4e-3),
        korobov_problem(65521, 3, 5, 11, 0.12, 2e-3),
        korobov_problem(1 << 16, 4, 6, 0, 0.05, 2e-3),
        rank2_problem(64, 16, 4, 7, 8, 0.05, 2e-3),
        korobov_problem(4099, 3, 8, 1, 0.2, 5e-3),
        rank2_problem(1024, 64, 5, 9, 5, 0.08, 2e-3),
    ]


def run_batched(lt, plans, probs, prec):
    import torch
    dtype = torch.complex128 if prec == "c128" else torch.complex64
    us = [torch.tensor(p["u0"], dtype=dtype, device="cuda") for p in probs]
    vs = [torch.tensor(p["v"], dtype=torch.float64, device="cuda") for p in probs]
    lt.strang_run_batched(plans, vs, us, [p["gamma"] for p in probs], [p["dt"] for p in probs],
                          [p["steps"] for p in probs])
    torch.cuda.synchronize()
    return [u.cpu().numpy().astype(np.complex128) for u in us]


@pytest.fixture(scope="module")
def mixed(lt):
    probs = mixed_problems()
    plans = [lt.lattice_plan(p["Z"], p["n"], p["I"]) for p in probs]
    refs = []
    for p in probs:
        _, s, _ = O.index_set(p["Z"], p["n"], p["I"])
        refs.append(O.strang_run(p["n"], s, p["v"], p["u0"], p["gamma"], p["dt"], p["steps"]))
    kinds = [(pl.info["passes"], pl.info["bluestein"]) for pl in plans]
    assert (1, 0) in kinds and (1, 1) in kinds and (2, 0) in kinds and (2, 1) in kinds
    return probs, plans, refs


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_mixed_batch_against_oracle(lt, mixed, prec):
    probs, plans, refs = mixed
    got = run_batched(lt, plans, probs, prec)
    for i, (g, r, p) in enumerate(zip(got, refs, probs)):
        e = rel(g, r)
        print(f"  {prec} problem {i}: N={len(r)} steps={p['steps']} passes={plans[i].info['passes']} "
              f"bluestein={plans[i].info['bluestein']} rel_l2={e:.2e}", flush=True)
        if p["steps"] == 0:
            assert np.array_equal(g, np.asarray(p["u0"]).astype(np.complex64 if prec == "c64" else np.complex128))
        assert e < TOL[prec], (i, e)


def test_batch_equals_single_runs(lt, mixed):
    """Each problem of the batch gives what strang_run gives on its own with the
    same kernels (register-staged passes of the 256-thread geometry where the
    length has one, the general passes otherwise)."""
    import torch
    probs, plans, _ = mixed
    got = run_batched(lt, plans, probs, "c128")
    for i, (pl, p) in enumerate(zip(plans, probs)):
        lt.lattice_plan_set_kernels(pl, lt.LT_C128, 1, 1)
        u = torch.tensor(p["u0"], dtype=torch.complex128, device="cuda")
        v = torch.tensor(p["v"], dtype=torch.float64, device="cuda")
        lt.strang_run(pl, v, u, p["gamma"], p["dt"], p["steps"])
        assert rel(got[i], u.cpu().numpy()) < 1e-14, i


def test_single_problem_and_empty_batch(lt, mixed):
    probs, plans, refs = mixed
    assert lt.strang_run_batched([], [], [], [], [], []) == []
    for i in (0, 4):
        got = run_batched(lt, [plans[i]], [probs[i]], "c128")[0]
        assert rel(got, refs[i]) < TOL["c128"]


def test_batched_argument_errors(lt, mixed):
    import torch
    probs, plans, _ = mixed
    u = torch.zeros(plans[0].N, dtype=torch.complex128, device="cuda")
    v = torch.zeros(plans[0].N, dtype=torch.float64, device="cuda")
    with pytest.raises(Exception):
        lt.strang_run_batched([plans[0]], [v], [u], [-1.0], [1e-3], [3])   # gamma <= 0
    with pytest.raises(Exception):
        lt.strang_run_batched([plans[0]], [v], [u], [0.1], [1e-3], [-1])   # negative steps
    with pytest.raises(Exception):
        lt.strang_run_batched([plans[0]], [v], [u[:-1]], [0.1], [1e-3], [3])  # wrong length


@pytest.fixture(scope="module")
def mixed_batch(lt):
    gold = np.load(GOLD)
    insts = W.mixed_batch()
    plans = [lt.lattice_plan(c.Z, c.n, c.I) for c in insts]
    return insts, plans, gold


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_mixed_batch_full_batch(lt, mixed_batch, prec):
    """All 256 problems, 200 steps, in the launch configuration the benchmark
    times: every problem's state against the oracle's at its stored sample
    points (72 per problem) and its full-vector norm against the oracle's."""
    insts, plans, gold = mixed_batch
    probs = [dict(u0=c.u0, v=c.v, gamma=c.gamma, dt=c.dt, steps=c.steps) for c in insts]
    got = run_batched(lt, plans, probs, prec)
    assert len(gold["instances"]) == len(insts)
    worst, worst_i = 0.0, -1
    for i in gold["instances"]:
        e = rel(got[i][gold[f"idx_{i}"]], gold[f"u_{i}"])
        if e > worst:
            worst, worst_i = e, int(i)
        assert e < TOL[prec], (int(i), insts[i].d, insts[i].N, e)
        assert abs(np.mean(np.abs(got[i]) ** 2) - float(gold[f"norm2_{i}"])) < 2 * TOL[prec]
    print(f"  {prec}: worst sampled rel_l2 over {len(insts)} problems {worst:.2e} (problem {worst_i}, "
          f"d={insts[worst_i].d} N={insts[worst_i].N})", flush=True)


def test_mixed_batch_reversible_c128(lt, mixed_batch):
    """200 steps with dt, then 200 with -dt, batched: every problem returns to u0."""
    import torch
    insts, plans, _ = mixed_batch
    us = [torch.tensor(c.u0, dtype=torch.complex128, device="cuda") for c in insts]
    vs = [torch.tensor(c.v, dtype=torch.float64, device="cuda") for c in insts]
    g = [c.gamma for c in insts]
    st = [c.steps for c in insts]
    lt.strang_run_batched(plans, vs, us, g, [c.dt for c in insts], st)
    lt.strang_run_batched(plans, vs, us, g, [-c.dt for c in insts], st)
    for u, c in zip(us, insts):
        assert rel(u.cpu().numpy(), c.u0) < 1e-11


# ---------------------------------------------------------------- batch objects
def make_states(probs, dtype):
    import torch
    us = [torch.tensor(p["u0"], dtype=dtype, device="cuda") for p in probs]
    vs = [torch.tensor(p["v"], dtype=torch.float64, device="cuda") for p in probs]
    return us, vs


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_batch_object_equals_run_batched(lt, mixed, prec):
    """strang_batch_create + strang_batch_run runs the launches of
    strang_run_batched: the same states, bit for bit, run after run."""
    import torch
    probs, plans, refs = mixed
    dtype = torch.complex128 if prec == "c128" else torch.complex64
    us, vs = make_states(probs, dtype)
    g, dts, st = [p["gamma"] for p in probs], [p["dt"] for p in probs], [p["steps"] for p in probs]
    bo = lt.strang_batch_create(plans, vs, us, g, dts, st)
    ur, vr = make_states(probs, dtype)
    for run in range(2):
        lt.strang_batch_run(bo)
        lt.strang_run_batched(plans, vr, ur, g, dts, st)
        torch.cuda.synchronize()
        for i in range(len(probs)):
            assert torch.equal(us[i], ur[i]), (run, i)
    e = max(rel(us[i].cpu().numpy().astype(np.complex128), O.strang_run(
        probs[i]["n"], O.index_set(probs[i]["Z"], probs[i]["n"], probs[i]["I"])[1], probs[i]["v"], refs[i],
        probs[i]["gamma"], probs[i]["dt"], probs[i]["steps"])) for i in range(len(probs)))
    print(f"  {prec}: two advances vs the oracle's 2m steps: max rel_l2 {e:.2e}", flush=True)
    assert e < 2 * TOL[prec]


def test_batch_object_graph_replay(lt, mixed):
    """strang_batch_run only enqueues launches: captured into a HIP graph, each
    replay advances every state once more, equal to eager advances of a second
    batch object, with eager work and synchronisations between the replays."""
    import torch
    probs, plans, _ = mixed
    g, dts, st = [p["gamma"] for p in probs], [p["dt"] for p in probs], [p["steps"] for p in probs]
    for dtype in (torch.complex64, torch.complex128):
        ug, vg = make_states(probs, dtype)
        ue, ve = make_states(probs, dtype)
        bg = lt.strang_batch_create(plans, vg, ug, g, dts, st)
        be = lt.strang_batch_create(plans, ve, ue, g, dts, st)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            lt.strang_batch_run(bg)
        torch.cuda.synchronize()
        for rep in range(3):
            graph.replay()
            torch.cuda.synchronize()
            lt.strang_batch_run(be)
            torch.cuda.synchronize()
            same = all(torch.equal(a, b) for a, b in zip(ug, ue))
            print(f"  {dtype} replay {rep}: equal to eager {same}", flush=True)
            assert same, rep
        del graph


def test_batch_object_autotune_and_errors(lt, mixed):
    import torch
    probs, plans, refs = mixed
    us, vs = make_states(probs, torch.complex128)
    g, dts, st = [p["gamma"] for p in probs], [p["dt"] for p in probs], [p["steps"] for p in probs]
    bo = lt.strang_batch_create(plans, vs, us, g, dts, st)
    lt.strang_batch_autotune(bo, reps=2)
    ks = lt.strang_batch_kernels(bo)
    print(f"  classes (key, variant): {ks}", flush=True)
    assert ks and all(v in (1, 2, 5) for _, v in ks)
    lt.strang_batch_run(bo)
    torch.cuda.synchronize()
    for i, (u, r) in enumerate(zip(us, refs)):  # the tuner leaves the states alone
        assert rel(u.cpu().numpy(), r) < TOL["c128"], i
    with pytest.raises(Exception):
        lt.strang_batch_create(plans[:1], vs[:1], us[:1], [-1.0], [1e-3], [3])
    empty = lt.strang_batch_create([], [], [], [], [], [])
    lt.strang_batch_run(empty)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_mixed_batch_full_batch_object_autotuned(lt, mixed_batch, prec):
    """All 256 problems through an autotuned batch object (the benchmark's
    launch configuration): every problem against the oracle's samples."""
    import torch
    insts, plans, gold = mixed_batch
    dtype = torch.complex128 if prec == "c128" else torch.complex64
    us = [torch.tensor(c.u0, dtype=dtype, device="cuda") for c in insts]
    vs = [torch.tensor(c.v, dtype=torch.float64, device="cuda") for c in insts]
    bo = lt.strang_batch_create(plans, vs, us, [c.gamma for c in insts], [c.dt for c in insts],
                                [c.steps for c in insts])
    lt.strang_batch_autotune(bo, reps=2)
    for u, c in zip(us, insts):  # the tuner leaves the states alone
        u.copy_(torch.tensor(c.u0, dtype=dtype, device="cuda"))
    lt.strang_batch_run(bo)
    torch.cuda.synchronize()
    worst = 0.0
    for i in gold["instances"]:
        got = us[i].cpu().numpy().astype(np.complex128)
        e = rel(got[gold[f"idx_{i}"]], gold[f"u_{i}"])
        worst = max(worst, e)
        assert e < TOL[prec], (int(i), e)
    print(f"  {prec}: classes {lt.strang_batch_kernels(bo)}, worst sampled rel_l2 {worst:.2e}", flush=True)
