"""Write tests/golden/cross_d6_n1048573_oracle_samples.npz: the FP64 oracle's state for
the benchmark workload (d = 6, N = 1048573, hyperbolic cross R = 10 completed
with minimal-l2 representatives, gamma = 0.05, dt = 1e-3) after 100 and 1000
Strang steps, at 8192 seeded sample points plus the first 64 points, with
the full-vector norm^2 and energy.  Calls only oracle/ and workloads/.
Runtime: about 30 minutes on one core."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main():
    c = W.cross_d6_n1048573(steps=1000)
    _, s, _ = O.index_set(c.Z, c.n, c.I)
    g = np.random.default_rng(20181808)
    idx = np.unique(np.concatenate([np.arange(64), g.choice(c.N, 8192, replace=False)]))
    out = {"idx": idx, "z": c.Z[0], "N": c.N}
    u = c.u0.copy()
    done = 0
    for mark in (100, 1000):
        t = time.time()
        u = O.strang_run(c.n, s, c.v, u, c.gamma, c.dt, mark - done)
        done = mark
        nn, E = O.diagnostics(c.n, s, c.v, u, c.gamma)
        out[f"u{mark}"] = u[idx]
        out[f"norm2_{mark}"] = nn
        out[f"energy_{mark}"] = E
        print(f"step {mark}: {time.time() - t:.0f}s norm2={nn:.15f} energy={E:.12f}", flush=True)
    nn0, E0 = O.diagnostics(c.n, s, c.v, c.u0, c.gamma)
    out["norm2_0"], out["energy_0"] = nn0, E0
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                     "cross_d6_n1048573_oracle_samples.npz"), **out)


if __name__ == "__main__":
    main()
