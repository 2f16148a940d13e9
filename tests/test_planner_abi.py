"""Host-side tests of the C-ABI library: exports, planner tables bit-exact
against the oracle, argument and lattice errors.  No GPU call is made."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_1808_06357_amd import _capi as C


def test_library_exports_every_header_function():
    names = C.header_functions()
    assert "strang_run" in names and "lattice_plan" in names and len(names) >= 12
    for name in names:
        assert hasattr(C.lib, name), name


def _planner_matches_oracle(Z, n, I=None):
    p = C.lattice_plan(Z, n, I)
    k, s, h = C.lattice_plan_keys(p)
    ho, so, fromI = O.index_set(Z, n, I)
    assert np.array_equal(s, so)
    assert np.array_equal(h, ho)
    if I is not None:
        assert np.array_equal(k, O.keys(Z, n, I))
        assert p.info["n_index"] == len(I) and p.info["n_completed"] == p.N - len(I)
    assert p.info["max_s"] == so.max()
    return p


def test_planner_fig1_and_box_d2_n1031_bitexact():
    _planner_matches_oracle(np.array([[1, 34]]), np.array([55]))
    c = W.box_d2_n1031()
    p = _planner_matches_oracle(c.Z, c.n, c.I)
    assert p.N == 1031


def test_planner_rank2_bitexact():
    _planner_matches_oracle(np.array([[1, 5, 7], [0, 1, 3]]), np.array([12, 4]))
    Z = W.cbc_rank2(W.hyperbolic_cross(4, 2), 64, 16, np.random.default_rng(3))
    _planner_matches_oracle(Z, np.array([64, 16]), W.hyperbolic_cross(4, 2))


def test_planner_adjoint_d4_n65521_lattice_bitexact():
    """d = 4, N = 65521, Korobov z, full minimal-l2 set (no user set)."""
    z = W.korobov(65521, 4, W.rng(4, "z"))
    _planner_matches_oracle(z.reshape(1, -1), np.array([65521]))


@pytest.mark.slow
def test_planner_cross_d6_n1048573_lattice_bitexact():
    """The benchmark lattice: d = 6, N = 1048573, hyperbolic cross R = 10
    completed with minimal-l2 representatives (bin map bit-exact)."""
    c1 = W.cross_d6_n1048573(steps=1)
    _planner_matches_oracle(c1.Z, c1.n, c1.I)


def test_points_match_workload_numerators():
    for Z, n in [(np.array([[1, 32]]), np.array([1031])), (np.array([[1, 5, 7], [0, 1, 3]]), np.array([12, 4]))]:
        p = C.lattice_plan(Z, n)
        assert np.array_equal(C.lattice_plan_points(p), W.point_numerators(Z, n))
        assert np.array_equal(C.lattice_plan_points(p, 5, 3), W.point_numerators(Z, n)[5:8])


def test_plan_errors():
    with pytest.raises(C.LatticeError) as e:
        C.lattice_plan(np.array([[1, 3], [1, 1]]), np.array([4, 8]))     # 8 does not divide 4
    assert e.value.status == "LT_E_NOT_CANONICAL"
    with pytest.raises(C.LatticeError) as e:
        C.lattice_plan(np.array([[1, 3]]), np.array([7]), np.array([[0, 0], [7, 0]]))
    assert e.value.status == "LT_E_NOT_INJECTIVE"
    with pytest.raises(C.LatticeError) as e:
        C.lattice_plan(np.array([[2, 4]]), np.array([8]))               # gcd 2: points repeat
    assert e.value.status == "LT_E_INCOMPLETE"
    with pytest.raises(C.LatticeError) as e:
        C.lattice_plan(np.array([[1, 1, 1], [1, 1, 1]]), np.array([4, 4]))  # rank-2 all odd: repeats
    assert e.value.status == "LT_E_INCOMPLETE"
    out = ctypes.c_void_p()
    assert C.lib.lattice_plan(0, 1, None, None, None, 0, 1, 0, ctypes.byref(out)) == 1
    assert b"d must be" in C.lib.lt_last_error()


def test_plan_complete_flag():
    """complete = 0 accepts an index set only when it owns every key; the
    config-0 box owns 1024 of 1031 keys (A7) and is rejected, while the full
    minimal-l2 set of the same lattice, given as H, plans to the same keys."""
    c = W.box_d2_n1031()
    with pytest.raises(C.LatticeError) as e:
        C.lattice_plan(c.Z, c.n, c.I, complete=False)
    assert e.value.status == "LT_E_INCOMPLETE"
    assert b"1024 of 1031" in C.lib.lt_last_error()
    full = C.lattice_plan(c.Z, c.n)
    _, s_full, h_full = C.lattice_plan_keys(full)
    again = C.lattice_plan(c.Z, c.n, h_full, complete=False)
    k, s, h = C.lattice_plan_keys(again)
    assert again.info["n_completed"] == 0 and again.info["n_index"] == c.N
    assert np.array_equal(k, np.arange(c.N)) and np.array_equal(s, s_full) and np.array_equal(h, h_full)
    out = ctypes.c_void_p()
    Z = np.ascontiguousarray(c.Z, dtype=np.int64)
    n = np.ascontiguousarray(c.n, dtype=np.int64)
    assert C.lib.lattice_plan(2, 1, Z.ctypes.data, n.ctypes.data, None, 0, 2, 0, ctypes.byref(out)) == 1
    assert C.lib.lattice_plan(2, 1, Z.ctypes.data, n.ctypes.data, None, 0, 1, 4, ctypes.byref(out)) == 1
    assert b"prec_mask" in C.lib.lt_last_error()


def test_run_argument_errors_before_any_gpu_call():
    p = C.lattice_plan(np.array([[1, 34]]), np.array([55]))
    h = p.handle
    # NULL buffers, bad gamma, bad precision, negative steps: rejected on the host
    assert C.lib.strang_run(h, 1, 1, None, 0, None, 0.1, 0.01, 5, None, 0, None, 0, None) == 1
    assert C.lib.strang_run(h, 1, 1, None, 0, None, -0.1, 0.01, 5, None, 0, None, 0, None) == 1
    assert C.lib.strang_run(h, 3, 1, None, 0, None, 0.1, 0.01, 5, None, 0, None, 0, None) == 1
    assert C.lib.strang_run(h, 1, 1, None, 0, None, 0.1, 0.01, -1, None, 0, None, 0, None) == 1
    assert C.lib.strang_run(None, 1, 1, None, 0, None, 0.1, 0.01, 1, None, 0, None, 0, None) == 1
    assert C.lib.strang_run(h, 1, 1, None, 0, None, 0.1, float("nan"), 1, None, 0, None, 0, None) == 1
    # zero steps / zero batch are no-ops that touch nothing
    assert C.lib.strang_run(h, 2, 0, None, 0, None, 0.1, 0.01, 5, None, 0, None, 0, None) == 0
    assert C.lib.strang_run(h, 2, 1, None, 0, None, 0.1, 0.01, 0, None, 0, None, 0, None) == 0
    assert C.lib.strang_adjoint(h, 2, 1, None, 0, None, None, 0.1, 0.01, 3, None, 0, None, None,
                                None, 0, None) == 1


def test_schedules():
    """Transform layouts: chirp-z for prime N, two passes for long transforms."""
    c = W.box_d2_n1031()
    p = C.lattice_plan(c.Z, c.n, c.I)
    assert p.info["bluestein"] == 1 and p.info["passes"] == 1 and p.info["fft_len"] >= 2 * 1031 - 1
    p = C.lattice_plan(np.array([[1, 253]]), np.array([1 << 16]))
    assert p.info["bluestein"] == 0 and p.info["passes"] == 2
    assert p.info["L1"] * p.info["L2"] == 1 << 16
    p = C.lattice_plan(np.array([[1, 5, 7], [0, 1, 3]]), np.array([12, 4]))
    assert p.info["passes"] == 1 and p.info["fft_len"] == 48
    # forward runs: a kinetic table, plus a transform buffer for two-pass chirp-z
    small = C.strang_workspace_size(p, C.LT_C128, 2, True)
    assert 0 < small <= 4096
    assert C.strang_adjoint_workspace_size(p, C.LT_C128, 2, True) > small
    c1 = C.lattice_plan(np.array([[1, 253]]), np.array([65521]))
    assert C.strang_workspace_size(c1, C.LT_C64, 3, True) >= 3 * c1.info["fft_len"] * 8
    # kernel selection is host state: set / get without a GPU
    assert C.lattice_plan_get_kernels_batch(c1, C.LT_C64, 64) == (1, 1)
    C.lattice_plan_set_kernels(c1, C.LT_C64, 2, 0)
    assert C.lattice_plan_get_kernels(c1, C.LT_C64) == (2, 0)
    # a forced choice holds for single-state and many-state launches alike
    for batch in (1, 2, 8, 64, 4096):
        assert C.lattice_plan_get_kernels_batch(c1, C.LT_C64, batch) == (2, 0)
    # complex128 columns of at most 2048 points default to variant 5
    assert c1.info["L1"] <= 2048
    assert C.lattice_plan_get_kernels_batch(c1, C.LT_C128, 64) == (5, 1)
    with pytest.raises(C.LatticeError):
        C.lattice_plan_set_kernels(c1, C.LT_C64, 6, 0)
    with pytest.raises(C.LatticeError):
        C.lattice_plan_set_kernels(c1, C.LT_C64, 1, 6)
    with pytest.raises(C.LatticeError):
        C.lattice_plan_get_kernels_batch(c1, C.LT_C64, 0)


def test_swapped_rank2_schedule():
    """Rank-2 tensors whose n1-point columns are long run transposed: the
    plan says so, and a run's workspace holds the transposed state and v."""
    for n1, n2, swapped in [(2048, 64, 1), (4096, 256, 1), (1024, 64, 0), (2048, 1024, 0), (64, 16, 0)]:
        H = W.hyperbolic_cross(4, 1)
        Z = W.cbc_rank2(H, n1, n2, np.random.default_rng(n1 + n2))
        p = C.lattice_plan(Z, np.array([n1, n2]), H)
        assert p.info["swapped"] == swapped, (n1, n2)
        if swapped:
            N = n1 * n2
            assert C.strang_workspace_size(p, C.LT_C64, 1, True) >= N * 8 + N * 8
            assert C.strang_workspace_size(p, C.LT_C128, 3, False) >= 3 * N * 16 + 3 * N * 8
    p = C.lattice_plan(np.array([[1, 253]]), np.array([1 << 16]))
    assert p.info["swapped"] == 0


def test_plan_poor_lattice_fails_within_budget():
    """z = (1, ..., 1): keys are coordinate sums, so minimal-l2 representatives
    of far keys lie far out; the planner stops at its enumeration budget with
    a clear error instead of exhausting host memory."""
    with pytest.raises(C.LatticeError) as e:
        C.lattice_plan(np.ones((1, 6), dtype=np.int64), np.array([200003]))
    assert e.value.status == "LT_E_UNSUPPORTED"
    assert "short dual vectors" in str(e.value)


def test_batched_argument_errors_on_host():
    p = C.lattice_plan(np.array([[1, 34]]), np.array([55]))
    arr = (ctypes.c_void_p * 1)(p.handle)
    assert C.lib.strang_run_batched(-1, None, 1, None, None, None, None, None, None, 0, None) == 1
    assert C.lib.strang_run_batched(1, None, 1, None, None, None, None, None, None, 0, None) == 1
    assert C.lib.strang_run_batched(0, None, 1, None, None, None, None, None, None, 0, None) == 0
    g = (ctypes.c_double * 1)(-0.1)
    dt = (ctypes.c_double * 1)(0.01)
    st = (ctypes.c_int64 * 1)(3)
    nul = (ctypes.c_void_p * 1)(None)
    assert C.lib.strang_run_batched(1, arr, 1, nul, nul, g, dt, st, None, 0, None) == 1  # gamma <= 0
    g[0] = 0.1
    assert C.lib.strang_run_batched(1, arr, 1, nul, nul, g, dt, st, None, 0, None) == 1  # NULL u, v
    size = ctypes.c_size_t()
    assert C.lib.strang_batched_workspace_size(1, arr, 1, ctypes.byref(size)) == 0 and size.value > 0


@pytest.mark.slow
def test_mixed_batch_lattices_bitexact_on_golden_instances():
    """Planner bin maps of six problems of the batched workload (best-of-8
    Korobov lattices, minimal-l2 full sets) equal the oracle's."""
    shapes = W.mixed_batch_shapes()
    Ns = np.array([N for _, N in shapes])
    ds = np.array([d for d, _ in shapes])
    prime = np.arange(len(shapes)) % 2 == 0
    # the largest prime and composite N, the smallest N, the first d = 10 and
    # d = 2 problems, problem 0
    sel = sorted({int(np.flatnonzero(prime)[np.argmax(Ns[prime])]),
                  int(np.flatnonzero(~prime)[np.argmax(Ns[~prime])]),
                  int(np.argmin(Ns)), int(np.flatnonzero(ds == 10)[0]), int(np.flatnonzero(ds == 2)[0]), 0})
    insts = W.mixed_batch(shapes=shapes[: max(sel) + 1])
    for i in sel:
        _planner_matches_oracle(insts[i].Z, insts[i].n)


def test_diagnostics_argument_errors_on_host():
    p = C.lattice_plan(np.array([[1, 34]]), np.array([55]))
    h = p.handle
    assert C.lib.lattice_diagnostics(h, 1, 1, None, 0, None, 0.1, None, None, 0, None) == 1   # NULL buffers
    assert C.lib.lattice_diagnostics(h, 1, 1, None, 0, None, -0.1, None, None, 0, None) == 1  # gamma <= 0
    assert C.lib.lattice_diagnostics(h, 3, 1, None, 0, None, 0.1, None, None, 0, None) == 1   # precision
    assert C.lib.lattice_diagnostics(h, 2, 0, None, 0, None, 0.1, None, None, 0, None) == 0   # empty batch
    assert C.lattice_diagnostics_workspace_size(p, C.LT_C128, 4) > C.lattice_diagnostics_workspace_size(p, C.LT_C128, 1)


def test_splitting_argument_errors_on_host():
    p = C.lattice_plan(np.array([[1, 34]]), np.array([55]))
    h = p.handle
    r = C.lib.splitting_run

    def call(prec=2, batch=1, v1=None, f=None, steps=5, order=4, gamma=0.1):
        return r(h, prec, batch, None, v1, 0, f, None, gamma, 0.01, steps, order, None, 0, None)
    assert call(order=3) == 1 and b"order" in C.lib.lt_last_error()
    assert call() == 1                       # NULL v, u
    assert call(prec=3) == 1                 # precision
    assert call(steps=-1) == 1
    assert call(gamma=0.0) == 1
    assert call(batch=0) == 0                # empty batch
    assert call(steps=0) == 0                # no steps
    with pytest.raises(C.LatticeError):
        C.splitting_workspace_size(p, C.LT_C128, 1, True, 6)
    s2 = C.splitting_workspace_size(p, C.LT_C64, 1, True, 2)
    s4 = C.splitting_workspace_size(p, C.LT_C64, 1, True, 4)
    assert s4 > s2 > 0


def test_splitting_times():
    """Substep boundaries: order 2 is the plain grid t0 + k dt; order 4 steps
    through t0 + (k + c_i) dt with c = (0, w1, w1 + w0) and ends at t0 + m dt."""
    assert np.array_equal(C.splitting_times(2, 4, 1.0, 0.25), 1.0 + 0.25 * np.arange(5))
    w1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
    tau = C.splitting_times(4, 2, 0.5, 0.1)
    c = np.array([0.0, w1, 1.0 - w1])
    assert tau.shape == (7,)
    assert np.allclose(tau[:6], 0.5 + 0.1 * (np.repeat([0.0, 1.0], 3) + np.tile(c, 2)), rtol=0, atol=1e-15)
    assert abs(tau[6] - 0.7) < 1e-15
    assert tau[2] < tau[1]                   # the middle substep runs backwards
    with pytest.raises(C.LatticeError):
        C.splitting_times(3, 2, 0.0, 0.1)
