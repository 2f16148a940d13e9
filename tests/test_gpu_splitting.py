"""GPU parity of the composed (higher-order) splitting entry point against
the oracle's composition of Strang steps: the fourth-order triple jump and
order 2 (plain Strang), across smooth, power-of-two, prime (convolution
form), rank-2, tiny and batched lattices.  Tolerances as for Strang runs:
relative L2 1e-11 (complex128), 1e-4 (complex64)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import TOL, _dtype, korobov_case, rel

pytestmark = pytest.mark.gpu


def gpu_split(lt, plan, v, u0, gamma, dt, steps, prec, order, **kw):
    import torch
    u = torch.tensor(np.asarray(u0), dtype=_dtype(prec), device="cuda")
    vv = torch.tensor(np.asarray(v), dtype=torch.float64, device="cuda")
    lt.splitting_run(plan, vv, u, gamma, dt, steps, order=order, **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.complex128)


def check_split(lt, Z, n, v, u0, gamma, dt, steps, I=None, orders=(4, 2), precs=("c128", "c64")):
    print(f"case N={int(np.prod(n))} r={len(n)} steps={steps} shape={np.shape(u0)}", flush=True)
    plan = lt.lattice_plan(Z, n, I)
    _, s, _ = O.index_set(Z, n, I)
    for order in orders:
        ref = O.composed_run(n, s, v, u0, gamma, dt, steps, order=order)
        for prec in precs:
            e = rel(gpu_split(lt, plan, v, u0, gamma, dt, steps, prec, order), ref)
            print(f"  order={order} {prec} bluestein={plan.info['bluestein']} rel_l2={e:.3e}", flush=True)
            assert e < TOL[prec], (order, prec, e)
    return plan


@pytest.mark.parametrize("N,d,seed", [(15360, 3, 1), (1 << 16, 4, 2), (65521, 4, 3), (1031, 3, 4),
                                      (4096, 3, 5)])
def test_composition_matches_oracle(lt, N, d, seed):
    check_split(lt, *korobov_case(N, d, 40 + seed, 7, dt=5e-3))


def test_tiny_lattices(lt):
    check_split(lt, np.array([[1, 34]]), np.array([55]), *korobov_case(55, 2, 45, 5)[2:])
    check_split(lt, np.array([[1]]), np.array([2]), np.array([0.3, -0.2]), np.array([1.0, 0.5j]), 0.2, 0.1, 3)


def test_rank2(lt):
    n1, n2, d = 1024, 64, 5
    H = W.hyperbolic_cross(d, 1)
    Z = W.cbc_rank2(H, n1, n2, np.random.default_rng(n1))
    n = np.array([n1, n2])
    num = W.point_numerators(Z, n)
    g = np.random.default_rng(46)
    v = W.cosine_series(d, 8, g).at(num, n1 * n2)
    u0 = W.seeded_packet(num, n1 * n2, g)
    check_split(lt, Z, n, v, u0, 0.05, 4e-3, 6, I=H)


def test_batch_shared_and_per_state_potential(lt):
    check_split(lt, *korobov_case(4096 * 3, 3, 47, 5, batch=3, shared=True))
    check_split(lt, *korobov_case(65521, 3, 48, 5, batch=2, shared=False), orders=(4,))


def test_order2_is_strang_and_reversible(lt):
    """Order 2 gives strang_run's result; the symmetric composition run with
    -dt undoes a run with dt; zero steps leave u unchanged."""
    import torch
    for N in (1031, 65521, 1 << 16):
        Z, n, v, u0, gamma, dt, _ = korobov_case(N, 3, 49, 1)
        plan = lt.lattice_plan(Z, n)
        vv = torch.tensor(v, device="cuda")
        a = torch.tensor(u0, dtype=torch.complex128, device="cuda")
        b = a.clone()
        lt.splitting_run(plan, vv, a, gamma, dt, 12, order=2)
        lt.strang_run(plan, vv, b, gamma, dt, 12)
        assert rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-12
        lt.splitting_run(plan, vv, a, gamma, dt, 9, order=4)
        lt.splitting_run(plan, vv, a, gamma, -dt, 9, order=4)
        lt.splitting_run(plan, vv, a, gamma, dt, 0, order=4)
        assert rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-12


def test_fourth_order_on_gpu(lt):
    """Against a fine-step run of the same scheme, halving dt divides the
    error of the complex128 composition by about 16."""
    import torch
    Z, n, v, u0, gamma, _, _ = korobov_case(1031, 2, 50, 1, gamma=0.3)
    plan = lt.lattice_plan(Z, n)
    vv = torch.tensor(v, device="cuda")
    T = 0.4

    def run(m):
        u = torch.tensor(u0, dtype=torch.complex128, device="cuda")
        lt.splitting_run(plan, vv, u, gamma, T / m, m, order=4)
        return u.cpu().numpy()

    ref = run(2048)
    errs = [np.linalg.norm(run(m) - ref) for m in (64, 128, 256)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("orders", orders, flush=True)
    assert np.all((orders > 3.8) & (orders < 4.2)), orders


def tdv_check(lt, Z, n, v, u0, gamma, dt, steps, v1, f, t0=0.1, I=None, orders=(2, 4), precs=("c128", "c64")):
    """v + f(t) v1 through the C-ABI (f sampled at splitting_times) against the
    oracle's time-dependent composition."""
    import torch
    print(f"tdv case N={int(np.prod(n))} r={len(n)} steps={steps} shape={np.shape(u0)}", flush=True)
    plan = lt.lattice_plan(Z, n, I)
    _, s, _ = O.index_set(Z, n, I)
    vv = torch.tensor(np.asarray(v), dtype=torch.float64, device="cuda")
    vv1 = torch.tensor(np.asarray(v1), dtype=torch.float64, device="cuda")
    for order in orders:
        fk = f(lt.splitting_times(order, steps, t0, dt))
        ref = O.composed_run(n, s, v, u0, gamma, dt, steps, order=order, v1=v1, f=f, t0=t0)
        for prec in precs:
            u = torch.tensor(np.asarray(u0), dtype=_dtype(prec), device="cuda")
            lt.splitting_run(plan, vv, u, gamma, dt, steps, order=order, v1=vv1, f=fk)
            torch.cuda.synchronize()
            e = rel(u.cpu().numpy().astype(np.complex128), ref)
            print(f"  order={order} {prec} bluestein={plan.info['bluestein']} rel_l2={e:.3e}", flush=True)
            assert e < TOL[prec], (order, prec, e)


def _field(case, seed):
    Z, n, v, u0, gamma, dt, steps = case
    N = int(np.prod(n))
    num = W.point_numerators(Z, n)
    g = np.random.default_rng(seed)
    d = Z.shape[1]
    v1 = W.cosine_series(d, 8, g).at(num, N)
    if np.ndim(v) == 2:
        v1 = np.stack([W.cosine_series(d, 8, g).at(num, N) for _ in range(v.shape[0])])
    return v1


def _f(t):
    return 1.0 + 2.0 * np.sin(5.0 * np.asarray(t))


@pytest.mark.parametrize("N,d,seed", [(15360, 3, 1), (1 << 16, 4, 2), (65521, 4, 3), (1031, 3, 4)])
def test_time_dependent_matches_oracle(lt, N, d, seed):
    case = korobov_case(N, d, 60 + seed, 6, dt=5e-3)
    tdv_check(lt, *case, v1=_field(case, seed), f=_f)


def test_time_dependent_rank2_tiny_and_batches(lt):
    n1, n2, d = 1024, 64, 5
    H = W.hyperbolic_cross(d, 1)
    Z = W.cbc_rank2(H, n1, n2, np.random.default_rng(n1))
    n = np.array([n1, n2])
    num = W.point_numerators(Z, n)
    g = np.random.default_rng(66)
    v = W.cosine_series(d, 8, g).at(num, n1 * n2)
    v1 = W.cosine_series(d, 8, g).at(num, n1 * n2)
    u0 = W.seeded_packet(num, n1 * n2, g)
    tdv_check(lt, Z, n, v, u0, 0.05, 4e-3, 5, v1=v1, f=_f, I=H)
    case = korobov_case(55, 2, 67, 5)
    tdv_check(lt, np.array([[1, 34]]), np.array([55]), *case[2:], v1=_field(case, 67), f=_f)
    case = korobov_case(4096 * 3, 3, 68, 4, batch=3, shared=True)
    tdv_check(lt, *case, v1=_field(case, 68), f=_f)
    case = korobov_case(65521, 3, 69, 4, batch=2, shared=False)
    tdv_check(lt, *case, v1=_field(case, 69), f=_f, orders=(4,))


def test_time_dependent_constant_coefficient(lt):
    """f = c gives the time-independent run under v + c v1."""
    import torch
    for N in (1031, 1 << 16):
        case = korobov_case(N, 3, 70, 1)
        Z, n, v, u0, gamma, dt, _ = case
        v1 = _field(case, 70)
        plan = lt.lattice_plan(Z, n)
        for order in (2, 4):
            a = torch.tensor(u0, dtype=torch.complex128, device="cuda")
            b = a.clone()
            fk = np.full(8 * (3 if order == 4 else 1) + 1, 0.7)
            lt.splitting_run(plan, torch.tensor(v, device="cuda"), a, gamma, dt, 8, order=order,
                             v1=torch.tensor(v1, device="cuda"), f=fk)
            lt.splitting_run(plan, torch.tensor(v + 0.7 * v1, device="cuda"), b, gamma, dt, 8, order=order)
            assert rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-12, (N, order)
