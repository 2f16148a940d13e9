"""The register-staged passes store the state with write-through when a
launch's working set fits the Infinity Cache and with write-back beyond it.
The policy changes no arithmetic: a state run alone (write-through) and the
same state inside a batch beyond the threshold (write-back) end bit for bit
equal, and both match the oracle."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,batch", [("c64", 200), ("c128", 100)])
def test_write_through_and_write_back_agree(lt, prec, batch):
    import torch
    dtype = torch.complex64 if prec == "c64" else torch.complex128
    N, d, steps, gamma, dt = 65521, 4, 9, 0.05, 2e-3
    g = np.random.default_rng(41)
    z = W.korobov(N, d, g)
    Z, n = z.reshape(1, -1), np.array([N])
    num = W.point_numerators(Z, n)
    v = W.cosine_series(d, 16, g).at(num, N)
    u0 = W.seeded_packet(num, N, g)
    plan = lt.lattice_plan(Z, n)
    L = plan.info["fft_len"]
    S = 8 if prec == "c64" else 16
    # the batch's working set is beyond the 192 MB threshold, the single state's within
    assert batch * L * S + 32 * L > (192 << 20) and L * S + 32 * L <= (192 << 20)
    vv = torch.tensor(v, device="cuda")
    one = torch.tensor(u0, dtype=dtype, device="cuda").reshape(1, N)
    lt.strang_run(plan, vv, one, gamma, dt, steps)
    many = torch.tensor(u0, dtype=dtype, device="cuda").reshape(1, N).repeat(batch, 1)
    lt.strang_run(plan, vv, many, gamma, dt, steps)
    torch.cuda.synchronize()
    print(f"  {prec}: batch {batch} x L {L}: states equal to the single run "
          f"{[bool(torch.equal(many[i], one[0])) for i in (0, batch // 2, batch - 1)]}", flush=True)
    assert torch.equal(many[0], one[0])
    assert torch.equal(many[batch - 1], one[0])
    _, s, _ = O.index_set(Z, n)
    ref = O.strang_run(n, s, v, u0, gamma, dt, steps)
    got = one[0].cpu().numpy().astype(np.complex128)
    e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert e < (1e-4 if prec == "c64" else 1e-11), e
    del many
    torch.cuda.empty_cache()
