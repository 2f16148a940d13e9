"""strang_run_noalloc (the entry point for callers that cannot allocate: its
workspace is the library's static per-GPU scratch) against strang_run on the
same inputs, through the C-ABI: two calls in a row, the second with a smaller
input; plus its two refusals (workspace beyond the scratch, plan tables not
built), returned before any launch."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def case(N, d, seed, batch, per_state_v):
    g = np.random.default_rng(seed)
    z = W.korobov(N, d, g)
    Z, n = z.reshape(1, -1), np.array([N])
    num = W.point_numerators(Z, n)
    if per_state_v:
        v = np.stack([W.cosine_series(d, 16, g).at(num, N) for _ in range(batch)])
    else:
        v = W.cosine_series(d, 16, g).at(num, N)
    u0 = np.stack([W.seeded_packet(num, N, g) for _ in range(batch)])
    return Z, n, v, u0


def test_noalloc_equals_strang_run_twice(lt):
    import torch
    # first call: the 2^16-point chirp-z lattice (N = 65521), two states with
    # their own potentials; second call: a smaller input, N = 4099, one state
    calls = [(65521, 4, 11, 2, True, 0.05, 2e-3, 12), (4099, 3, 12, 1, False, 0.1, 5e-3, 7)]
    for N, d, seed, batch, per_state, gamma, dt, steps in calls:
        Z, n, v, u0 = case(N, d, seed, batch, per_state)
        plan = lt.lattice_plan(Z, n, prec_mask=lt.LT_C64 | lt.LT_C128)
        vv = torch.tensor(v, dtype=torch.float64, device="cuda")
        for dtype in (torch.complex128, torch.complex64):
            ua = torch.tensor(u0, dtype=dtype, device="cuda")
            ub = ua.clone()
            lt.strang_run_noalloc(plan, vv, ua, gamma, dt, steps)
            lt.strang_run(plan, vv, ub, gamma, dt, steps)
            torch.cuda.synchronize()
            err = float(torch.linalg.vector_norm(ua - ub) / torch.linalg.vector_norm(ub))
            print(f"  N={N} batch={batch} {dtype}: equal {torch.equal(ua, ub)}, rel {err:.1e}", flush=True)
            assert torch.equal(ua, ub), (N, dtype, err)


def test_noalloc_refusals(lt):
    import torch
    # per-state potential tables of three 2^22-point states need 192 MiB
    N = 1 << 22
    Z, n, v, u0 = case(N, 3, 13, 3, True)
    plan = lt.lattice_plan(Z, n, prec_mask=lt.LT_C64)
    vv = torch.tensor(v, dtype=torch.float64, device="cuda")
    u = torch.tensor(u0, dtype=torch.complex64, device="cuda")
    before = u.clone()
    assert lt.strang_workspace_size(plan, lt.LT_C64, 3, False) > lt.strang_run_noalloc_capacity()
    with pytest.raises(lt.LatticeError, match="scratch holds"):
        lt.strang_run_noalloc(plan, vv, u, 0.05, 1e-3, 3)
    # a plan whose complex128 tables were never built
    Z, n, v, u0 = case(65521, 4, 14, 1, False)
    plan = lt.lattice_plan(Z, n, prec_mask=0)
    vv = torch.tensor(v, dtype=torch.float64, device="cuda")
    u2 = torch.tensor(u0, dtype=torch.complex128, device="cuda")
    with pytest.raises(lt.LatticeError, match="not built"):
        lt.strang_run_noalloc(plan, vv, u2, 0.05, 1e-3, 3)
    torch.cuda.synchronize()
    assert torch.equal(u, before)
