"""The largest lattices the path is built for (N about 2^22; the prime one
needs a chirp-z length of 2^23 = 2048 x 4096): properties that hold at any
size, since the oracle is too slow here -- unitarity, reversibility, the two
forms of the prime-N step agreeing, and complex64 agreeing with complex128."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def problem(N, d, seed):
    g = np.random.default_rng(seed)
    z = W.korobov_good(N, d, g)
    Z, n = z.reshape(1, -1), np.array([N])
    num = W.point_numerators(Z, n)
    return Z, n, W.cosine_series(d, 16, g).at(num, N), W.seeded_packet(num, N, g)


@pytest.mark.parametrize("N,d", [(4194301, 3), (1 << 22, 3)])
def test_largest_lattices(lt, N, d):
    import torch
    Z, n, v, u0 = problem(N, d, 41)
    plan = lt.lattice_plan(Z, n)
    info = plan.info
    print(f"N={N}: L={info['fft_len']} = {info['L1']} x {info['L2']}, chirp-z={info['bluestein']}", flush=True)
    vv = torch.tensor(v, device="cuda")
    gamma, dt, m = 0.05, 2e-3, 8

    def run(dtype, pieces, sign=1.0, u=None):
        u = torch.tensor(u0, dtype=dtype, device="cuda") if u is None else u
        for k in pieces:
            lt.strang_run(plan, vv, u, gamma, sign * dt, k)
        return u

    u = run(torch.complex128, [m])
    a = u.cpu().numpy()
    n0 = np.mean(np.abs(u0) ** 2)
    assert abs(np.mean(np.abs(a) ** 2) - n0) < 1e-12 * n0
    back = run(torch.complex128, [m], -1.0, u).cpu().numpy()
    assert rel(back, u0) < 1e-11
    if info["bluestein"]:
        # m steps in one call (convolution form) = m steps in calls of 2 (chirp-z pairs)
        b = run(torch.complex128, [2] * (m // 2)).cpu().numpy()
        e = rel(a, b)
        print(f"  convolution vs chirp-z form: {e:.2e}", flush=True)
        assert e < 1e-12
    c = run(torch.complex64, [m]).cpu().numpy().astype(np.complex128)
    e = rel(c, a)
    print(f"  complex64 vs complex128: {e:.2e}", flush=True)
    assert e < 1e-5
