"""Write tests/golden/wide_oracle_samples.npz: the FP64 oracle's state for
two lattices whose transform needs rows of 8192 points (L = 2^25 = 4096 x
8192): the paper's Table 1 lattice d = 3, n = 2^25, z = (1, 12386359,
15699201) (Sec. 3.2) with g1, the smooth potential v1, gamma = 0.5,
dt = 1e-3, 4 steps; and the rank-1 lattice of prime N = 8388617, d = 2,
best-of-8 Korobov (seed 3), chirp-z length 2^25, with the harmonic v2,
gamma = 0.5, dt = 1e-3, 4 steps (the convolution form of a step).  Stored: the
state at 4096 seeded points plus the first 64, and the full-vector norm^2.
Calls only oracle/ and workloads/.  Runtime: about 10 minutes on one core."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

GAMMA, DT, STEPS = 0.5, 1e-3, 4


def cases():
    Z, n = W.paper_lattice(3, 1 << 25)
    yield "table1_d3", Z, n, W.v_smooth_paper
    N = 8388617
    z = W.korobov_good(N, 2, np.random.default_rng(3))
    yield "prime_d2", z.reshape(1, -1), np.array([N]), W.v_harmonic_paper


def main():
    out = {}
    for name, Z, n, vfun in cases():
        t = time.time()
        N = int(n[0])
        _, s, _ = O.index_set(Z, n)
        num = W.point_numerators(Z, n)
        v = vfun(num, N)
        u0 = W.paper_g1(num, N, GAMMA)
        u = O.strang_run(n, s, v, u0, GAMMA, DT, STEPS)
        g = np.random.default_rng(20250125)
        idx = np.unique(np.concatenate([np.arange(64), g.choice(N, 4096, replace=False)]))
        out[f"{name}_z"] = Z[0]
        out[f"{name}_N"] = N
        out[f"{name}_idx"] = idx
        out[f"{name}_u"] = u[idx]
        out[f"{name}_norm2"] = float(np.mean(np.abs(u) ** 2))
        print(f"{name}: {time.time() - t:.0f}s norm2={out[f'{name}_norm2']:.15f}", flush=True)
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "wide_oracle_samples.npz"), **out)


if __name__ == "__main__":
    main()
