"""Write tests/golden/adjoint_d4_n65521_oracle_grad.npz: the FP64 oracle's gradients for
the differentiation workload (d = 4, N = 65521, 32 states sharing a 64-term
cosine potential v, gamma = 0.05, dt = 2e-3, 500 steps).  The target of state
b is the oracle's run of u0_b under a hidden 64-term potential; the loss is the
full lattice L2 misfit J = sum_b (1/N) sum_k |u_b(T)_k - target_b,k|^2 over all
N points.  Stored: J, dJ/da for the 64 coefficients of v (a_t multiplies
cos(2 pi h_t . x)) with the conditioning of each coefficient's sum
kappa_t = sum_k |B_tk dJ/dv_k| / |sum_k B_tk dJ/dv_k| and of the reduction
as a whole (||B||_2 ||dJ/dv|| / ||dJ/da||), the conditioning of dJ/dv's sums
over steps and states (kappa_v), the norm of dJ/dv,
dJ/dv at 1024 seeded points, and dJ/du0, u(T) and the target at 128 seeded
points per state; and the same gradients with both potentials shifted by a
constant (J and its gradients unchanged in exact arithmetic, so the two
results differ by the oracle's own rounding).  Calls only oracle/ and
workloads/.  Runtime: about 15 minutes per part on 8 cores."""
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


# Both potentials shifted by the same constant: every state and the target
# pick up the same global phase exp(-i SHIFT T / gamma) (a constant commutes
# with the Laplacian), so J and its gradients are unchanged in exact
# arithmetic; the oracle's results under the shift differ from the unshifted
# ones by its own rounding alone, which measures the oracle's noise floor.
SHIFT = 0.375


def state(b, shift=0.0):
    if not _C:
        setup()
    c, s = _C["c"], _C["s"]
    t = time.time()
    target = O.strang_run(c.n, s, c.meta["v_hidden"] + shift, c.u0[b], c.gamma, c.dt, c.steps)
    uT = O.strang_run(c.n, s, c.v + shift, c.u0[b], c.gamma, c.dt, c.steps)
    gT = (2.0 / c.N) * (uT - target)
    J = float(np.sum(np.abs(uT - target) ** 2) / c.N)
    g0, gv, ga = O.strang_vjp(c.n, s, c.v + shift, c.u0[b], gT, c.gamma, c.dt, c.steps, return_abs=True)
    print(f"state {b}: J_b={J:.6e} {time.time() - t:.0f}s", flush=True)
    return b, target, uT, J, g0, gv, ga


def state_shifted(b):
    return state(b, SHIFT)


def gradients(fn):
    c = _C["c"]
    B, N = c.u0.shape[0], c.N
    with Pool(int(os.environ.get("GOLDEN_PROCS", "8"))) as pool:
        res = sorted(pool.map(fn, range(B)), key=lambda r: r[0])
    # the batch sums of dJ/dv and of its terms' absolute values, in a fixed
    # order (state 0 first)
    gv, ga = np.zeros(N), np.zeros(N)
    for r in res:
        gv += r[5]
        ga += r[6]
    return res, gv, ga


def main(part):
    setup()
    c = _C["c"]
    N = c.N
    g = np.random.default_rng(20180604)
    idx_u = np.sort(g.choice(N, 128, replace=False))
    idx_v = np.sort(g.choice(N, 1024, replace=False))
    basis = c.meta["series"].basis(c.meta["num"], N)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_d4_n65521_oracle_grad.npz")
    out = dict(np.load(path)) if part != "all" and os.path.exists(path) else {}
    if part in ("all", "base"):
        res, gv, ga = gradients(state)
        dJ_da = basis @ gv
        # conditioning: of dJ/dv's sums over steps and states (norm-wise,
        # ||sum |terms| || / ||dJ/dv||) and of the 64-term reduction B dJ/dv
        # (per coefficient, and norm-wise ||B||_2 ||dJ/dv|| / ||dJ/da||)
        out.update(J=sum(r[3] for r in res), dJ_da=dJ_da,
                   kappa_v=np.linalg.norm(ga) / np.linalg.norm(gv),
                   kappa=(np.abs(basis) @ np.abs(gv)) / np.abs(dJ_da),
                   kappa_norm=np.linalg.norm(basis, 2) * np.linalg.norm(gv) / np.linalg.norm(dJ_da),
                   dJ_dv_norm=np.linalg.norm(gv), idx_v=idx_v, dJ_dv=gv[idx_v], idx_u=idx_u,
                   dJ_du0=np.stack([r[4][idx_u] for r in res]), uT=np.stack([r[2][idx_u] for r in res]),
                   target=np.stack([r[1][idx_u] for r in res]))
    if part in ("all", "shift"):
        res, gv, _ = gradients(state_shifted)
        dJ_da = basis @ gv
        out.update(shift=SHIFT, J_shift=sum(r[3] for r in res), dJ_da_shift=dJ_da, dJ_dv_shift=gv[idx_v],
                   dJ_du0_shift=np.stack([r[4][idx_u] for r in res]))
    np.savez_compressed(path, **out)


if __name__ == "__main__":
    # --part base | shift | all (default): shift adds the shifted-potential
    # gradients to an existing file
    main(sys.argv[sys.argv.index("--part") + 1] if "--part" in sys.argv else "all")
