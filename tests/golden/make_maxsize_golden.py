"""Write tests/golden/maxsize_oracle_samples.npz: the FP64 oracle's state after
8 steps on the largest single lattices of the build (workloads.maxsize_d3):
d = 3, N = 4194301 (prime; chirp-z length 2^23) and N = 2^22, 16-term cosine
potential, seeded packet, gamma = 0.05, dt = 2e-3.  Stored per lattice: the
state at 4096 seeded points plus the first 64 and the last 64, and the
full-vector norm^2.  Calls only oracle/ and workloads/.  Runtime: a few
minutes on one core."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

SIZES = (4194301, 1 << 22)


def main():
    out = {}
    for N in SIZES:
        t = time.time()
        c = W.maxsize_d3(N)
        _, s, _ = O.index_set(c.Z, c.n, c.I)
        u = O.strang_run(c.n, s, c.v, c.u0, c.gamma, c.dt, c.steps)
        g = np.random.default_rng(20260422 + N % 1000)
        idx = np.unique(np.concatenate([np.arange(64), np.arange(N - 64, N), g.choice(N, 4096, replace=False)]))
        out[f"n{N}_z"] = c.Z[0]
        out[f"n{N}_idx"] = idx
        out[f"n{N}_u"] = u[idx]
        out[f"n{N}_norm2"] = float(np.mean(np.abs(u) ** 2))
        print(f"N={N}: {time.time() - t:.0f}s norm2={out[f'n{N}_norm2']:.15f}", flush=True)
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "maxsize_oracle_samples.npz"),
                        **out)


if __name__ == "__main__":
    main()
