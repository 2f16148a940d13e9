"""lattice_diagnostics (norm^2 and energy of Sec. 3.3) against the FP64
oracle's diagnostics, and the conservation experiment of Sec. 3.3 (gamma = 0.5,
d = 5, the paper's g1 and harmonic v2) through checkpointed runs."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 2e-6}


def lattices():
    g = np.random.default_rng(77)
    out = []
    for N, d in [(1031, 2), (15360, 3), (65521, 4), (1 << 16, 3)]:
        z = W.korobov_good(N, d, g)
        out.append((z.reshape(1, -1), np.array([N]), None))
    H = W.hyperbolic_cross(4, 1)
    out.append((W.cbc_rank2(H, 64, 16, np.random.default_rng(64)), np.array([64, 16]), H))
    H = W.hyperbolic_cross(5, 1)
    out.append((W.cbc_rank2(H, 1024, 64, np.random.default_rng(1024)), np.array([1024, 64]), H))
    return out


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_diagnostics_against_oracle(lt, prec):
    import torch
    dtype = torch.complex128 if prec == "c128" else torch.complex64
    for Z, n, I in lattices():
        N = int(np.prod(n))
        plan = lt.lattice_plan(Z, n, I)
        _, s, _ = O.index_set(Z, n, I)
        num = W.point_numerators(Z, n)
        g = np.random.default_rng(N)
        d = Z.shape[1]
        vs = np.stack([W.cosine_series(d, 8, g).at(num, N) + 1.0 for _ in range(3)])
        us = np.stack([W.seeded_packet(num, N, g) for _ in range(3)])
        got = lt.lattice_diagnostics(plan, torch.tensor(vs, device="cuda"),
                                     torch.tensor(us, dtype=dtype, device="cuda"), 0.3).cpu().numpy()
        ref = np.array([O.diagnostics(n, s, vs[b], us[b], 0.3) for b in range(3)])
        e = float(np.max(np.abs(got - ref) / np.abs(ref)))
        print(f"  N={N} r={len(n)} {prec}: max rel error of (norm^2, energy) {e:.2e}", flush=True)
        assert e < TOL[prec], (N, e)


def test_conservation_paper_setting(lt):
    """gamma = 0.5, d = 5, g1, v2 (Sec. 3.3): the norm and energy history of a
    run every 5 steps, from the checkpoints, against the oracle's history; the
    norm varies by less than 1e-13 relative (delta = (max - min) / mean)."""
    import torch
    N, d, gamma, dt, steps, every = 1 << 14, 5, 0.5, 1e-2, 40, 5
    z = W.korobov_good(N, d, np.random.default_rng(5))
    Z, n = z.reshape(1, -1), np.array([N])
    num = W.point_numerators(Z, n)
    v = W.v_harmonic_paper(num, N)
    u0 = W.paper_g1(num, N, gamma)
    plan = lt.lattice_plan(Z, n)
    _, s, _ = O.index_set(Z, n)
    _, hist = O.strang_run(n, s, v, u0, gamma, dt, steps, history=True)
    vv = torch.tensor(v, device="cuda")
    u = torch.tensor(u0, dtype=torch.complex128, device="cuda")
    nck = lt.num_checkpoints(steps, every)
    ck = torch.empty(nck * N, dtype=torch.complex128, device="cuda")
    lt.strang_run(plan, vv, u, gamma, dt, steps, ckpt=ck, ckpt_every=every)
    got = lt.lattice_diagnostics(plan, vv, ck.view(nck, N), gamma).cpu().numpy()
    ref = np.asarray(hist)[0, 0:steps:every, :2]
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-11
    norm = got[:, 0]
    delta = (norm.max() - norm.min()) / norm.mean()
    print(f"  norm delta {delta:.2e}, energy delta {(got[:, 1].max() - got[:, 1].min()) / got[:, 1].mean():.2e}",
          flush=True)
    assert delta < 1e-13
