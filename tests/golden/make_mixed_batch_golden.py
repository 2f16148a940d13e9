"""Write tests/golden/mixed_batch_oracle_samples.npz: the FP64 oracle's state
after 200 Strang steps for every one of the 256 problems of the batched
workload (d in 2..10, N between 2^12 and 2^18, best-of-8 Korobov lattices
with minimal-l2 full index sets, 16-term cosine potentials, gamma in
[0.02, 0.2], dt = 5e-3).  Stored per problem: 64 seeded sample points plus
the first 8, the state there and the norm^2 of the full vector.  Calls only
oracle/ and workloads/.  Runtime: about 10 minutes on 8 cores."""
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

STEPS = 200
INSTS = []


def run(i):
    c = INSTS[i]
    t = time.time()
    _, s, _ = O.index_set(c.Z, c.n, c.I)
    u = O.strang_run(c.n, s, c.v, c.u0, c.gamma, c.dt, STEPS)
    g = np.random.default_rng(20180602 + i)
    idx = np.unique(np.concatenate([np.arange(8), g.choice(c.N, 64, replace=False)]))
    nn, _ = O.diagnostics(c.n, s, c.v, u, c.gamma)
    print(f"problem {i}: d={c.d} N={c.N} {time.time() - t:.0f}s norm2={nn:.15f}", flush=True)
    return i, idx, u[idx], nn


def main():
    t = time.time()
    INSTS.extend(W.mixed_batch())
    print(f"inputs {time.time() - t:.0f}s", flush=True)
    order = sorted(range(len(INSTS)), key=lambda i: -INSTS[i].N)  # longest first
    with Pool(int(os.environ.get("GOLDEN_PROCS", "8"))) as pool:
        res = sorted(pool.imap_unordered(run, order), key=lambda r: r[0])
    out = {"instances": np.arange(len(INSTS)), "steps": STEPS}
    for i, idx, ui, nn in res:
        out[f"idx_{i}"] = idx.astype(np.int32)
        out[f"u_{i}"] = ui
        out[f"norm2_{i}"] = nn
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                     "mixed_batch_oracle_samples.npz"), **out)


if __name__ == "__main__":
    main()
