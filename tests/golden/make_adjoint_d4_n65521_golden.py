"""Write tests/golden/adjoint_d4_n65521_oracle_grad.npz: the FP64 oracle's gradients for
the differentiation workload (d = 4, N = 65521, 32 states sharing a 64-term
cosine potential v, gamma = 0.05, dt = 2e-3, 500 steps).  The target of state
b is the oracle's run of u0_b under a hidden 64-term potential; the loss is the
full lattice L2 misfit J = sum_b (1/N) sum_k |u_b(T)_k - target_b,k|^2 over all
N points.  Stored: J, dJ/da for the 64 coefficients of v (a_t multiplies
cos(2 pi h_t . x)) with the conditioning of each coefficient's sum
kappa_t = sum_k |B_tk dJ/dv_k| / |sum_k B_tk dJ/dv_k|, the norm of dJ/dv,
dJ/dv at 1024 seeded points, and dJ/du0, u(T) and the target at 128 seeded
points per state.  Calls only oracle/ and workloads/.  Runtime: about
15 minutes on 8 cores."""
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

_C = {}


def setup():
    c = W.adjoint_d4_n65521()
    _, s, _ = O.index_set(c.Z, c.n, c.I)
    _C.update(c=c, s=s)


def state(b):
    if not _C:
        setup()
    c, s = _C["c"], _C["s"]
    t = time.time()
    target = O.strang_run(c.n, s, c.meta["v_hidden"], c.u0[b], c.gamma, c.dt, c.steps)
    uT = O.strang_run(c.n, s, c.v, c.u0[b], c.gamma, c.dt, c.steps)
    gT = (2.0 / c.N) * (uT - target)
    J = float(np.sum(np.abs(uT - target) ** 2) / c.N)
    g0, gv = O.strang_vjp(c.n, s, c.v, c.u0[b], gT, c.gamma, c.dt, c.steps)
    print(f"state {b}: J_b={J:.6e} {time.time() - t:.0f}s", flush=True)
    return b, target, uT, J, g0, gv


def main():
    setup()
    c = _C["c"]
    B, N = c.u0.shape[0], c.N
    g = np.random.default_rng(20180604)
    idx_u = np.sort(g.choice(N, 128, replace=False))
    idx_v = np.sort(g.choice(N, 1024, replace=False))
    with Pool(int(os.environ.get("GOLDEN_PROCS", "8"))) as pool:
        res = sorted(pool.map(state, range(B)), key=lambda r: r[0])
    # the batch sum of dJ/dv in a fixed order (state 0 first)
    gv = np.zeros(N)
    for r in res:
        gv += r[5]
    basis = c.meta["series"].basis(c.meta["num"], N)
    dJ_da = basis @ gv
    kappa = (np.abs(basis) @ np.abs(gv)) / np.abs(dJ_da)
    np.savez_compressed(
        os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_d4_n65521_oracle_grad.npz"),
        J=sum(r[3] for r in res), dJ_da=dJ_da, kappa=kappa, dJ_dv_norm=np.linalg.norm(gv),
        idx_v=idx_v, dJ_dv=gv[idx_v], idx_u=idx_u,
        dJ_du0=np.stack([r[4][idx_u] for r in res]), uT=np.stack([r[2][idx_u] for r in res]),
        target=np.stack([r[1][idx_u] for r in res]))


if __name__ == "__main__":
    main()
