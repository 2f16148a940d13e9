"""Write tests/golden/wide_oracle_samples.npz: the FP64 oracle's state for
two lattices whose transform needs rows of 8192 points (L = 2^25 = 4096 x
8192): the paper's Table 1 lattice d = 3, n = 2^25, z = (1, 12386359,
15699201) (Sec. 3.2) with g1, the smooth potential v1, gamma = 0.5,
dt = 1e-3, 4 steps; and the rank-1 lattice of prime N = 8388617, d = 2,
best-of-8 Korobov (seed 3), chirp-z length 2^25, with the harmonic v2,
gamma = 0.5, dt = 1e-3, 4 steps (the convolution form of a step); and the Table 1
lattices d = 4, 6, 8, 10, 12 with n = 2^25 (z the first d components of the
d = 12 vector) under the paper's g1 or g2 and v1 or v2, gamma = 0.5,
dt = 1e-3, 4 steps.  Stored: the state at 4096 seeded points plus the first
64, and the full-vector norm^2.  Calls only oracle/ and workloads/.  Runtime:
about 30 minutes on two cores (up to 12 GB per case).  Arguments: case names
to recompute alone, keeping the other stored cases."""
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

GAMMA, DT, STEPS = 0.5, 1e-3, 4


# the Table 1 lattices of d = 4 ... 12 (n = 2^25, z the first d components of
# the d = 12 vector), each with one of the paper's initial conditions and
# potentials (Sec. 3.2); d = 12 is also the largest minimal-l2 set the planner
# builds (2^25 keys in 12 dimensions)
TABLE1_HIGH = {4: ("g2", "v2"), 6: ("g1", "v1"), 8: ("g1", "v2"), 10: ("g2", "v1"), 12: ("g1", "v2")}


def cases():
    Z, n = W.paper_lattice(3, 1 << 25)
    yield "table1_d3", Z, n, W.v_smooth_paper, W.paper_g1
    N = 8388617
    z = W.korobov_good(N, 2, np.random.default_rng(3))
    yield "prime_d2", z.reshape(1, -1), np.array([N]), W.v_harmonic_paper, W.paper_g1
    for d, (g, v) in TABLE1_HIGH.items():
        Z, n = W.paper_lattice(d, 1 << 25)
        yield (f"table1_d{d}", Z, n, W.v_smooth_paper if v == "v1" else W.v_harmonic_paper,
               W.paper_g1 if g == "g1" else W.paper_g2)


def run_case(case):
    name, Z, n, vfun, gfun = case
    t = time.time()
    N = int(n[0])
    _, s, _ = O.index_set(Z, n)
    num = W.point_numerators(Z, n)
    v = vfun(num, N)
    u0 = gfun(num, N, GAMMA)
    del num
    u = O.strang_run(n, s, v, u0, GAMMA, DT, STEPS)
    g = np.random.default_rng(20250125)
    idx = np.unique(np.concatenate([np.arange(64), g.choice(N, 4096, replace=False)]))
    out = {f"{name}_z": Z[0], f"{name}_N": N, f"{name}_idx": idx, f"{name}_u": u[idx],
           f"{name}_norm2": float(np.mean(np.abs(u) ** 2))}
    print(f"{name}: {time.time() - t:.0f}s norm2={out[f'{name}_norm2']:.15f}", flush=True)
    return out


def main(only):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wide_oracle_samples.npz")
    out = dict(np.load(path)) if only and os.path.exists(path) else {}
    todo = [c for c in cases() if not only or c[0] in only]
    with Pool(int(os.environ.get("GOLDEN_PROCS", "2"))) as pool:  # 2^25-point states: a few GB each
        for part in pool.imap_unordered(run_case, todo):
            out.update(part)
    out["steps"] = STEPS
    out["gamma"] = GAMMA
    out["dt"] = DT
    np.savez_compressed(path, **out)


if __name__ == "__main__":
    # optional case names: recompute only those and keep the other stored cases
    main(sys.argv[1:])
