"""The largest single lattices the path is built for (d = 3, N about 2^22; the
prime one needs a chirp-z length of 2^23 = 2048 x 4096): the state after 8
steps against the FP64 oracle's at stored sample points (both forms of the
prime-N step: the convolution form of one call and the chirp-z pairs of calls
of 2 steps), in both precisions, plus unitarity and reversibility."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "maxsize_oracle_samples.npz")
TOL = {"c128": 1e-11, "c64": 1e-4}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("N", [4194301, 1 << 22])
def test_largest_lattices(lt, N):
    import torch
    gold = np.load(GOLD)
    c = W.maxsize_d3(N)
    assert np.array_equal(gold[f"n{N}_z"], c.Z[0])
    idx, ref = gold[f"n{N}_idx"], gold[f"n{N}_u"]
    plan = lt.lattice_plan(c.Z, c.n, c.I)
    info = plan.info
    print(f"N={N}: L={info['fft_len']} = {info['L1']} x {info['L2']}, chirp-z={info['bluestein']}", flush=True)
    vv = torch.tensor(c.v, device="cuda")
    m = c.steps

    def run(dtype, pieces, sign=1.0, u=None):
        u = torch.tensor(c.u0, dtype=dtype, device="cuda") if u is None else u
        for k in pieces:
            lt.strang_run(plan, vv, u, c.gamma, sign * c.dt, k)
        return u

    forms = [("one call", [m])]
    if info["bluestein"]:
        forms.append(("calls of 2 (chirp-z pairs)", [2] * (m // 2)))
    for prec, dtype in (("c128", torch.complex128), ("c64", torch.complex64)):
        for name, pieces in forms:
            u = run(dtype, pieces)
            a = u.cpu().numpy().astype(np.complex128)
            e = rel(a[idx], ref)
            print(f"  {prec} {name}: sampled rel_l2 vs oracle {e:.2e}", flush=True)
            assert e < TOL[prec], (prec, name, e)
            n2 = float(np.mean(np.abs(a) ** 2))
            assert abs(n2 - float(gold[f"n{N}_norm2"])) < 2 * TOL[prec], (prec, n2)
            if prec == "c128" and name == "one call":
                back = run(dtype, [m], -1.0, u).cpu().numpy()
                assert rel(back, c.u0) < 1e-11
