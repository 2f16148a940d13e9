"""Write tests/golden/rank2_d10_n4096x256_oracle_samples.npz: the FP64 oracle's state for
the rank-2 workload (d = 10, n = (4096, 256), cross {-1,0,1}^10 completed with
minimal-l2 representatives, gamma = 0.05, 32-term cosine potential,
dt = 2e-3) after 100 and 500 Strang steps, at 4096 seeded sample points plus
the first 64, with the full-vector norm^2.  Calls only oracle/ and
workloads/.  Runtime: several minutes on one core."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main():
    c = W.rank2_d10_n4096x256()
    t = time.time()
    _, s, _ = O.index_set(c.Z, c.n, c.I)
    print(f"index set {time.time() - t:.0f}s", flush=True)
    g = np.random.default_rng(20180603)
    idx = np.unique(np.concatenate([np.arange(64), g.choice(c.N, 4096, replace=False)]))
    out = {"idx": idx, "Z": c.Z}
    u = c.u0.copy()
    done = 0
    for mark in (100, 500):
        t = time.time()
        u = O.strang_run(c.n, s, c.v, u, c.gamma, c.dt, mark - done)
        done = mark
        out[f"u{mark}"] = u[idx]
        out[f"norm2_{mark}"] = float(np.mean(np.abs(u) ** 2))
        print(f"step {mark}: {time.time() - t:.0f}s norm2={out[f'norm2_{mark}']:.15f}", flush=True)
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                     "rank2_d10_n4096x256_oracle_samples.npz"), **out)


if __name__ == "__main__":
    main()
