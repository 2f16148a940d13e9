"""GPU parity of the initial discretization error (Sec. 3.4): the key sums
(sum_A |ghat|^2, sum_A |ghat - ghat_a|^2) of lattice_projection_error
against the oracle's, for the paper's Gaussian g1 on rank-1 (smooth,
power-of-two, prime) and rank-2 lattices and a batch.  Each side builds the
exact coefficients ghat from its own index set."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import _dtype

pytestmark = pytest.mark.gpu


def _coeffs(h_of_key, d, gamma):
    kmax = int(np.abs(h_of_key).max()) + 1
    tables, norm2 = W.paper_g1_coefficients(d, gamma, kmax)
    return W.coefficients_at(h_of_key.astype(np.int64), tables), norm2


def check(lt, Z, n, gammas, I=None):
    import torch
    N, d = int(np.prod(n)), Z.shape[1]
    print(f"case N={N} r={len(n)} d={d} batch={len(gammas)}", flush=True)
    plan = lt.lattice_plan(Z, n, I)
    _, _, h_lib = lt.lattice_plan_keys(plan)
    h_ref, _, _ = O.index_set(Z, n, I)   # representatives in key order
    num = W.point_numerators(Z, n)
    u = np.stack([W.paper_g1(num, N, gm, normalize=False) for gm in gammas])
    g_lib = np.stack([_coeffs(h_lib, d, gm)[0] for gm in gammas])
    g_ref = np.stack([_coeffs(h_ref, d, gm)[0] for gm in gammas])
    ref = O.projection_error(n, u, g_ref)
    for prec in ("c128", "c64"):
        out = lt.lattice_projection_error(plan, torch.tensor(u, dtype=_dtype(prec), device="cuda"),
                                          torch.tensor(g_lib, dtype=torch.complex128, device="cuda"))
        got = out.cpu().numpy()
        for b in range(len(gammas)):
            e0 = abs(got[b, 0] - ref[b, 0]) / ref[b, 0]
            e1 = abs(got[b, 1] - ref[b, 1])
            tol1 = 1e-10 * ref[b, 1] + 1e-15 * ref[b, 0] if prec == "c128" else 1e-4 * ref[b, 1] + 1e-9 * ref[b, 0]
            print(f"  {prec} gamma={gammas[b]} sums={got[b]} ref={ref[b]} rel0={e0:.1e} abs1={e1:.1e}", flush=True)
            assert e0 < 1e-12 and e1 < tol1, (prec, b, e0, e1)


def test_projection_fig1_and_smooth(lt):
    check(lt, np.array([[1, 34]]), np.array([55]), [1.0])
    z = W.korobov_good(15360, 3, np.random.default_rng(81))
    check(lt, z.reshape(1, -1), np.array([15360]), [1.0, 0.5])


def test_projection_power_of_two_and_prime(lt):
    z = W.korobov_good(1 << 16, 4, np.random.default_rng(82))
    check(lt, z.reshape(1, -1), np.array([1 << 16]), [1.0])
    z = W.korobov_good(65521, 4, np.random.default_rng(83))
    check(lt, z.reshape(1, -1), np.array([65521]), [1.0, 0.3])


def test_projection_rank2(lt):
    n1, n2, d = 1024, 64, 5
    H = W.hyperbolic_cross(d, 1)
    Z = W.cbc_rank2(H, n1, n2, np.random.default_rng(n1))
    check(lt, Z, np.array([n1, n2]), [1.0])
