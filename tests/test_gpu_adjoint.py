"""GPU adjoint (strang_adjoint, reverse-time recomputation with checkpoint
resets) against the oracle's recompute-forward VJP, plus the autograd
Function and a dot-product test."""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def problem(N, d, seed, batch, shared, terms=16):
    g = np.random.default_rng(seed)
    z = W.korobov(N, d, g)
    Z, n = z.reshape(1, -1), np.array([N])
    num = W.point_numerators(Z, n)
    if shared:
        v = W.cosine_series(d, terms, g).at(num, N)
    else:
        v = np.stack([W.cosine_series(d, terms, g).at(num, N) for _ in range(batch)])
    u0 = np.stack([W.seeded_packet(num, N, g) for _ in range(batch)])
    tgt = np.stack([W.seeded_packet(num, N, g) for _ in range(batch)])
    return Z, n, v, u0, tgt


def gpu_grad(lt, plan, v, u0, tgt, gamma, dt, steps, every, dtype):
    import torch
    N = plan.N
    u = torch.tensor(u0, dtype=dtype, device="cuda")
    vv = torch.tensor(v, dtype=torch.float64, device="cuda")
    batch = u0.shape[0]
    ck = torch.empty(lt.num_checkpoints(steps, every) * batch * N, dtype=dtype, device="cuda")
    lt.strang_run(plan, vv, u, gamma, dt, steps, ckpt=ck, ckpt_every=every)
    gT = (2.0 / N) * (u - torch.tensor(tgt, dtype=dtype, device="cuda"))
    g0, gv = lt.strang_adjoint(plan, vv, u, gT.contiguous(), gamma, dt, steps, ck, every)
    torch.cuda.synchronize()
    return g0.cpu().numpy().astype(np.complex128), gv.cpu().numpy()


@pytest.mark.parametrize("N,d,shared", [(1031, 2, True), (12288, 3, False), (65521, 4, True),
                                        (4096, 3, True), (97, 2, False)])
def test_adjoint_matches_oracle(lt, N, d, shared):
    import torch
    batch, gamma, dt, steps, every = 2, 0.05, 2e-3, 37, 10
    Z, n, v, u0, tgt = problem(N, d, N, batch, shared)
    plan = lt.lattice_plan(Z, n)
    _, s, _ = O.index_set(Z, n)
    uT = O.strang_run(n, s, v, u0, gamma, dt, steps)
    g0_ref, gv_ref = O.strang_vjp(n, s, v, u0, 2.0 * (uT - tgt) / N, gamma, dt, steps)
    for dtype, tol in ((torch.complex128, 1e-11), (torch.complex64, 1e-4)):
        g0, gv = gpu_grad(lt, plan, v, u0, tgt, gamma, dt, steps, every, dtype)
        e0, ev = rel(g0, g0_ref), rel(gv, gv_ref)
        print(f"N={N} {dtype} dJ/du0 rel={e0:.2e} dJ/dv rel={ev:.2e}", flush=True)
        assert e0 < tol and ev < tol


@pytest.mark.parametrize("shared", [True, False])
def test_adjoint_on_transposed_rank2(lt, shared):
    """A rank-2 tensor with long columns runs its forward transposed and
    stores its checkpoints in lattice order; the adjoint sweep runs
    transposed too (u(T), the cotangent and v transposed in, the checkpoint
    resets read transposed, dJ/du0 and dJ/dv transposed out): the gradients
    against the oracle's VJP, with a shared and a per-state potential."""
    import torch
    n1, n2, d, batch, gamma, dt, steps, every = 2048, 64, 4, 2, 0.05, 2e-3, 13, 5
    H = W.hyperbolic_cross(d, 1)
    Z = W.cbc_rank2(H, n1, n2, np.random.default_rng(71))
    n = np.array([n1, n2])
    N = n1 * n2
    num = W.point_numerators(Z, n)
    g = np.random.default_rng(72)
    if shared:
        v = W.cosine_series(d, 16, g).at(num, N)
    else:
        v = np.stack([W.cosine_series(d, 16, g).at(num, N) for _ in range(batch)])
    u0 = np.stack([W.seeded_packet(num, N, g) for _ in range(batch)])
    tgt = np.stack([W.seeded_packet(num, N, g) for _ in range(batch)])
    plan = lt.lattice_plan(Z, n, H)
    assert plan.info["swapped"] == 1
    _, s, _ = O.index_set(Z, n, H)
    uT = O.strang_run(n, s, v, u0, gamma, dt, steps)
    g0_ref, gv_ref = O.strang_vjp(n, s, v, u0, 2.0 * (uT - tgt) / N, gamma, dt, steps)
    for dtype, tol in ((torch.complex128, 1e-11), (torch.complex64, 1e-4)):
        g0, gv = gpu_grad(lt, plan, v, u0, tgt, gamma, dt, steps, every, dtype)
        e0, ev = rel(g0, g0_ref), rel(gv, gv_ref)
        print(f"rank-2 {n1}x{n2} shared={shared} {dtype} dJ/du0 rel={e0:.2e} dJ/dv rel={ev:.2e}", flush=True)
        assert gv.shape == np.shape(gv_ref)
        assert e0 < tol and ev < tol


def test_autograd_function(lt):
    import torch
    N, d, batch, gamma, dt, steps = 65521, 4, 3, 0.05, 2e-3, 24
    Z, n, v, u0, tgt = problem(N, d, 5, batch, True)
    plan = lt.lattice_plan(Z, n)
    vv = torch.tensor(v, dtype=torch.float64, device="cuda", requires_grad=True)
    u = torch.tensor(u0, dtype=torch.complex128, device="cuda", requires_grad=True)
    t = torch.tensor(tgt, dtype=torch.complex128, device="cuda")
    uT = lt.lattice_strang(plan, vv, u, gamma, dt, steps, ckpt_every=8)
    J = (uT - t).abs().pow(2).sum() / N
    J.backward()
    _, s, _ = O.index_set(Z, n)
    uT_ref = O.strang_run(n, s, v, u0, gamma, dt, steps)
    g0_ref, gv_ref = O.strang_vjp(n, s, v, u0, 2.0 * (uT_ref - tgt) / N, gamma, dt, steps)
    assert rel(uT.detach().cpu().numpy(), uT_ref) < 1e-11
    assert rel(u.grad.cpu().numpy(), g0_ref) < 1e-11
    assert rel(vv.grad.cpu().numpy(), gv_ref) < 1e-11


def test_dot_product_identity(lt):
    """<S^m x, y> = <x, (S^m)^H y> with the GPU forward and GPU adjoint."""
    import torch
    N, d, steps, every = 65521, 3, 20, 7
    Z, n, v, x, y = problem(N, d, 6, 1, True)
    plan = lt.lattice_plan(Z, n)
    vv = torch.tensor(v, device="cuda")
    u = torch.tensor(x, dtype=torch.complex128, device="cuda")
    ck = torch.empty(lt.num_checkpoints(steps, every) * N, dtype=torch.complex128, device="cuda")
    lt.strang_run(plan, vv, u, 0.05, 2e-3, steps, ckpt=ck, ckpt_every=every)
    yy = torch.tensor(y, dtype=torch.complex128, device="cuda")
    g0, _ = lt.strang_adjoint(plan, vv, u, yy, 0.05, 2e-3, steps, ck, every)
    lhs = np.vdot(y, u.cpu().numpy())
    rhs = np.vdot(g0.cpu().numpy(), x)
    assert abs(lhs - rhs) < 1e-11 * np.linalg.norm(x) * np.linalg.norm(y)


# ---------------------------------------------------------------- full-size differentiation workload
GOLD4 = os.path.join(os.path.dirname(__file__), "golden", "adjoint_d4_n65521_oracle_grad.npz")


@pytest.fixture(scope="module")
def case4(lt):
    import torch
    gold = np.load(GOLD4)
    c = W.adjoint_d4_n65521()
    plan = lt.lattice_plan(c.Z, c.n, c.I)
    # the kernels the benchmark times: autotuned (the 32-state runs take the
    # many-state choice)
    for p in (lt.LT_C64, lt.LT_C128):
        lt.lattice_plan_autotune(plan, p, reps=3)
        print(f"adjoint_d4_n65521 kernels {p}: one state {lt.lattice_plan_get_kernels_batch(plan, p, 1)}, "
              f"32 states {lt.lattice_plan_get_kernels_batch(plan, p, 32)}", flush=True)
    basis = torch.tensor(c.meta["series"].basis(c.meta["num"], c.N), dtype=torch.float64, device="cuda")
    return c, plan, basis, gold


def target_run(lt, c, plan, dtype):
    """The target of the loss: u0 run under the hidden potential (on this path,
    in the precision under test)."""
    import torch
    t = torch.tensor(c.u0, dtype=dtype, device="cuda")
    vh = torch.tensor(c.meta["v_hidden"], dtype=torch.float64, device="cuda")
    lt.strang_run(plan, vh, t, c.gamma, c.dt, c.steps)
    return t


def loss_and_grads(lt, c, plan, v, target, dtype, grads=True):
    """J = sum_b (1/N) sum_k |u_b(T)_k - target_b,k|^2 over every point and,
    through strang_adjoint, (dJ/dv, dJ/du0)."""
    import torch
    N, m, every = c.N, c.steps, c.meta["ckpt_every"]
    u = torch.tensor(c.u0, dtype=dtype, device="cuda")
    B = u.shape[0]
    ck = torch.empty(lt.num_checkpoints(m, every) * B * N, dtype=dtype, device="cuda") if grads else None
    lt.strang_run(plan, v, u, c.gamma, c.dt, m, ckpt=ck, ckpt_every=every if grads else 0)
    diff = u.to(torch.complex128) - target.to(torch.complex128)
    J = float(torch.sum(torch.abs(diff) ** 2).item()) / N
    if not grads:
        return J, u
    gT = ((2.0 / N) * diff).to(dtype)
    g0, gv = lt.strang_adjoint(plan, v, u, gT, c.gamma, c.dt, m, ck, every)
    return J, u, g0, gv


@pytest.mark.parametrize("prec,tol", [("c128", 1e-11), ("c64", 1e-4)])
def test_adjoint_d4_n65521_gradients_against_oracle(lt, case4, prec, tol):
    """d = 4, N = 65521, 32 states, 500 steps, checkpoints every 50, the loss
    over the whole lattice: J, the target run, u(T), dJ/da (64 coefficients),
    dJ/dv and dJ/du0 against the FP64 oracle's adjoint (stored samples)."""
    import torch
    c, plan, basis, gold = case4
    dtype = torch.complex128 if prec == "c128" else torch.complex64
    v = torch.tensor(c.v, dtype=torch.float64, device="cuda")
    target = target_run(lt, c, plan, dtype)
    J, u, g0, gv = loss_and_grads(lt, c, plan, v, target, dtype)
    dJda = (basis @ gv).cpu().numpy()
    iu, iv = gold["idx_u"], gold["idx_v"]
    errs = {"J": abs(J - float(gold["J"])) / abs(float(gold["J"])),
            "target": rel(target.cpu().numpy()[:, iu], gold["target"]),
            "uT": rel(u.cpu().numpy()[:, iu], gold["uT"]),
            "dJ/da": rel(dJda, gold["dJ_da"]),
            "dJ/dv": rel(gv.cpu().numpy()[iv], gold["dJ_dv"]),
            "dJ/du0": rel(g0.cpu().numpy()[:, iu], gold["dJ_du0"])}
    print(f"adjoint_d4_n65521 {prec}: " + ", ".join(f"{k} {e:.2e}" for k, e in errs.items())
          + f"; max kappa of dJ/da {float(np.max(gold['kappa'])):.1f}", flush=True)
    for k, e in errs.items():
        assert e < tol, (k, e)


def test_adjoint_d4_n65521_central_differences_c128(lt, case4):
    """dJ/da from the adjoint against central differences, h = 1e-6, every one
    of the 64 coefficients, on the complex128 path."""
    import torch
    c, plan, basis, gold = case4
    a = torch.tensor(c.meta["series"].a, dtype=torch.float64, device="cuda")
    target = target_run(lt, c, plan, torch.complex128)
    _, _, _, gv = loss_and_grads(lt, c, plan, (a @ basis).contiguous(), target, torch.complex128)
    adj = (basis @ gv).cpu().numpy()
    h = 1e-6
    fd = np.empty(a.numel())
    for t in range(a.numel()):
        e = torch.zeros_like(a)
        e[t] = h
        jp, _ = loss_and_grads(lt, c, plan, ((a + e) @ basis).contiguous(), target, torch.complex128, False)
        jm, _ = loss_and_grads(lt, c, plan, ((a - e) @ basis).contiguous(), target, torch.complex128, False)
        fd[t] = (jp - jm) / (2 * h)
    e = rel(fd, adj)
    print(f"adjoint_d4_n65521 central differences vs adjoint: rel {e:.2e} (|dJ/da| = {np.linalg.norm(adj):.3e})", flush=True)
    assert e < 1e-6
