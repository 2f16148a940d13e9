"""Runs on caller streams: a run on a side stream (default priority) equals
the run on the current stream; two plans, and one plan shared by two runs
with their own buffers and workspaces, run concurrently on two streams and
equal their serial results (plans are immutable after creation)."""
import numpy as np
import pytest

from test_gpu_parity import korobov_case, rel

pytestmark = pytest.mark.gpu


def _setup(lt, N, d, seed):
    import torch
    Z, n, v, u0, gamma, dt, _ = korobov_case(N, d, seed, 1)
    plan = lt.lattice_plan(Z, n)
    return plan, torch.tensor(v, device="cuda"), torch.tensor(u0, dtype=torch.complex128, device="cuda"), gamma, dt


def _serial(lt, plan, v, u0, gamma, dt, steps):
    import torch
    u = u0.clone()
    lt.strang_run(plan, v, u, gamma, dt, steps)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def test_side_stream_and_concurrent_plans(lt):
    import torch
    a = _setup(lt, 65521, 4, 91)
    b = _setup(lt, 1 << 16, 3, 92)
    ref_a = _serial(lt, *a, 30)
    ref_b = _serial(lt, *b, 30)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ua, ub = a[2].clone(), b[2].clone()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        lt.strang_run(a[0], a[1], ua, a[3], a[4], 30, stream=s1)
    with torch.cuda.stream(s2):
        lt.strang_run(b[0], b[1], ub, b[3], b[4], 30, stream=s2)
    torch.cuda.synchronize()
    assert rel(ua.cpu().numpy(), ref_a) < 1e-13
    assert rel(ub.cpu().numpy(), ref_b) < 1e-13


def test_one_plan_two_streams(lt):
    import torch
    plan, v, u0, gamma, dt = _setup(lt, 65521, 4, 93)
    ref = _serial(lt, plan, v, u0, gamma, dt, 25)
    u1 = u0.clone()
    u2 = torch.flip(u0, [0]).contiguous()
    ref2 = _serial(lt, plan, v, u2, gamma, dt, 25)
    nb = lt.strang_workspace_size(plan, lt.LT_C128, 1, True)
    w1 = torch.empty(nb, dtype=torch.uint8, device="cuda")
    w2 = torch.empty(nb, dtype=torch.uint8, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        lt.strang_run(plan, v, u1, gamma, dt, 25, work=w1, stream=s1)
    with torch.cuda.stream(s2):
        lt.strang_run(plan, v, u2, gamma, dt, 25, work=w2, stream=s2)
    torch.cuda.synchronize()
    assert rel(u1.cpu().numpy(), ref) < 1e-13
    assert rel(u2.cpu().numpy(), ref2) < 1e-13
