"""Second-order convergence in dt on a lattice of the paper's Table 1
(d = 2, n = 2^18, z = (1, 100135)), with the paper's Gaussian g1 and both of
its potentials (Sec. 3.2), following its protocol: T = 1, reference solution
with dt = 1/10000, runs with dt = 1/m (complex128 on the GPU)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("potential,gamma,ms", [("v1", 0.1, [20, 40, 80, 160]), ("v2", 0.5, [40, 80, 160, 320])])
def test_second_order_paper_lattice(lt, potential, gamma, ms):
    """The least-squares slope of log error against log dt lies in [1.85, 2.15].
    With v1 each halving of dt also gains a factor close to 4; v2 is
    continuous but not smooth on the torus, and its successive ratios
    oscillate around 4."""
    import torch
    Z, n = W.paper_lattice(2, 1 << 18)
    N = int(n[0])
    num = W.point_numerators(Z, n)
    v = W.v_smooth_paper(num, N) if potential == "v1" else W.v_harmonic_paper(num, N)
    u0 = W.paper_g1(num, N, gamma)
    plan = lt.lattice_plan(Z, n)
    vv = torch.tensor(v, device="cuda")

    def solve(m):
        u = torch.tensor(u0, dtype=torch.complex128, device="cuda")
        lt.strang_run(plan, vv, u, gamma, 1.0 / m, m)
        return u.cpu().numpy()

    ref = solve(10000)
    errs = [float(np.sqrt(np.mean(np.abs(solve(m) - ref) ** 2))) for m in ms]
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(ms) - 1)]
    slope = np.polyfit(np.log(1.0 / np.asarray(ms, dtype=float)), np.log(errs), 1)[0]
    print(f"  {potential}: errors {['%.2e' % e for e in errs]}, orders {['%.3f' % o for o in orders]}, "
          f"fitted order {slope:.3f}", flush=True)
    assert 1.85 < slope < 2.15, slope
    if potential == "v1":
        assert all(1.9 < o < 2.1 for o in orders), orders
