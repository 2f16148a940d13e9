"""Graph capture of strang_run.  With a caller workspace, and once an earlier
run has built the plan's device tables, a run enqueues kernel launches only
(no allocation, memset or synchronisation), so a caller can capture it into a
HIP graph and replay it.  Every replay is checked against the eager run, with
eager work and synchronisations between the replays."""
import numpy as np
import pytest

from test_gpu_parity import korobov_case, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,d", [(65521, 4), (1 << 16, 3), (1031, 2)])
def test_captured_run_replays_equal_eager(lt, N, d):
    """Chirp-z two-pass, power-of-two two-pass and one-workgroup schedules."""
    import torch
    Z, n, v, u0, gamma, dt, _ = korobov_case(N, d, 97, 1)
    plan = lt.lattice_plan(Z, n)
    vv = torch.tensor(v, device="cuda")
    steps = 12
    for dtype, prec in ((torch.complex128, lt.LT_C128), (torch.complex64, lt.LT_C64)):
        print(f"graph N={N} d={d} {dtype}", flush=True)
        u0d = torch.tensor(np.asarray(u0), dtype=dtype, device="cuda")
        ws = torch.empty(lt.strang_workspace_size(plan, prec, 1, True), dtype=torch.uint8, device="cuda")
        # eager references: one run, and two runs in a row (a run boundary
        # applies the two half potential steps separately, so two runs differ
        # from one run of twice the steps by rounding)
        refs = []
        u = u0d.clone()
        for k in (1, 2):
            lt.strang_run(plan, vv, u, gamma, dt, steps, work=ws)
            torch.cuda.synchronize()
            refs.append(u.cpu().numpy())
        u = u0d.clone()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            lt.strang_run(plan, vv, u, gamma, dt, steps, work=ws)
        torch.cuda.synchronize()
        for rep in range(3):
            u.copy_(u0d)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            e = rel(u.cpu().numpy(), refs[0])
            print(f"  replay {rep}: rel_l2 vs eager {e:.2e}", flush=True)
            assert e == 0.0, (rep, e)
        # two replays in a row equal two eager runs in a row
        u.copy_(u0d)
        g.replay()
        g.replay()
        torch.cuda.synchronize()
        e = rel(u.cpu().numpy(), refs[1])
        print(f"  two replays: rel_l2 vs eager {e:.2e}", flush=True)
        assert e == 0.0, e
        del g
