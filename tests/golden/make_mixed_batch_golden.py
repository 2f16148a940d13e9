"""Write tests/golden/mixed_batch_oracle_samples.npz: the FP64 oracle's state
after 200 Strang steps for six instances of the batched workload (256
problems, d in 2..10, N between 2^12 and 2^18, best-of-8 Korobov lattices
with minimal-l2 full index sets, 16-term cosine potentials, gamma in
[0.02, 0.2], dt = 5e-3): the largest prime N, the largest composite N, the
smallest N, the first d = 10 and d = 2 problems and problem 0.  Stored per
instance: 256 seeded sample points, the state there and the norm^2 of the
full vector.  Calls only oracle/ and workloads/.  Runtime: a few minutes on
six cores."""
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


def pick(shapes):
    Ns = np.array([N for _, N in shapes])
    ds = np.array([d for d, _ in shapes])
    prime = np.arange(len(shapes)) % 2 == 0
    sel = [int(np.flatnonzero(prime)[np.argmax(Ns[prime])]),
           int(np.flatnonzero(~prime)[np.argmax(Ns[~prime])]),
           int(np.argmin(Ns)), int(np.flatnonzero(ds == 10)[0]), int(np.flatnonzero(ds == 2)[0]), 0]
    return sorted(set(sel))


def run(i):
    shapes = W.mixed_batch_shapes()
    insts = W.mixed_batch(shapes=shapes[: i + 1])  # the generators draw in order: build the prefix
    c = insts[i]
    t = time.time()
    _, s, _ = O.index_set(c.Z, c.n, c.I)
    u = O.strang_run(c.n, s, c.v, c.u0, c.gamma, c.dt, STEPS)
    g = np.random.default_rng(20180602 + i)
    idx = np.unique(np.concatenate([np.arange(16), g.choice(c.N, 240, replace=False)]))
    nn, _ = O.diagnostics(c.n, s, c.v, u, c.gamma)
    print(f"instance {i}: d={c.d} N={c.N} {time.time() - t:.0f}s norm2={nn:.15f}", flush=True)
    return i, idx, u[idx], nn


def main():
    sel = pick(W.mixed_batch_shapes())
    with Pool(len(sel)) as pool:
        res = pool.map(run, sel)
    out = {"instances": np.array(sel), "steps": STEPS}
    for i, idx, ui, nn in res:
        out[f"idx_{i}"] = idx
        out[f"u_{i}"] = ui
        out[f"norm2_{i}"] = nn
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                     "mixed_batch_oracle_samples.npz"), **out)


if __name__ == "__main__":
    main()
