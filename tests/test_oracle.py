"""Pins for the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them retypes the oracle's
formula: they use closed forms, brute force on tiny inputs, independent dense
linear algebra (scipy expm) or library FFTs (numpy) as the outside opinion.
"""
import itertools

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

import oracle as O
import workloads as W

PI = np.pi


# ----------------------------------------------------------------- helpers
def brute_min_l2(Z, n, box_r, fixed=None):
    """Pure-Python argmin over a box: for every key the (||h||^2, lex h) least
    vector (Lemma 4, eq. (hrepresenter)); `fixed` maps keys to owners."""
    Z = np.atleast_2d(Z)
    n = np.atleast_1d(n)
    d = Z.shape[1]
    best = {}
    for h in itertools.product(range(-box_r, box_r + 1), repeat=d):
        chi = 0
        for i in range(Z.shape[0]):
            chi = chi * int(n[i]) + (sum(a * int(b) for a, b in zip(h, Z[i])) % int(n[i]))
        if fixed is not None and chi in fixed:
            continue
        s = sum(a * a for a in h)
        if chi not in best or (s, h) < best[chi]:
            best[chi] = (s, h)
    return best


def grid_strang(vgrid, u0grid, gamma, dt, steps, freqs):
    """Independent split-step solver on a tensor grid using numpy.fft.fftn
    (the classical Fourier pseudo-spectral method the paper generalises,
    Sec. 2.2): kinetic phase exp(-i 2 pi^2 gamma dt |f|^2) per grid frequency."""
    s = sum(f ** 2 for f in freqs)
    K = np.exp(-1j * 2 * PI * PI * gamma * dt * s)
    P = np.exp(-1j * dt * vgrid / (2 * gamma))
    u = u0grid.astype(np.complex128)
    for _ in range(steps):
        u = P * u
        u = np.fft.ifftn(K * np.fft.fftn(u))
        u = P * u
    return u


# ----------------------------------------------------------------- keys
def test_fig1_example_full_minimal_set():
    """Sec. 2.1, Fig. 1: n = 55, z = (1, 34) has an anti-aliasing set of full
    cardinality; the minimal-l2 owners equal a brute-force argmin."""
    Z, n = np.array([[1, 34]]), np.array([55])
    h, s, _ = O.index_set(Z, n)
    k = O.keys(Z, n, h)
    assert np.array_equal(np.sort(k), np.arange(55))
    assert np.array_equal(k, np.arange(55))          # h_of_key[chi] has key chi
    best = brute_min_l2(Z, n, 12)
    assert len(best) == 55
    for chi in range(55):
        assert s[chi] == best[chi][0]
        assert tuple(h[chi]) == best[chi][1]


def test_box_d2_n1031_initial_condition_is_projected_onto_the_index_set():
    """Config 0's u0 is the Gaussian packet projected onto I: its lattice DFT
    vanishes on the seven completed keys and carries, on each key of I, the
    packet's closed-form Fourier coefficient (the transform of a Gaussian,
    shifted to the centre and the carrier k0), up to the common scale."""
    c = W.box_d2_n1031()
    N = int(c.n[0])
    coef = np.fft.fft(c.u0) / N  # u_k = sum_xi coef_xi exp(2 pi i xi k / N)
    k = O.keys(c.Z, c.n, c.I)
    others = np.setdiff1d(np.arange(N), k)
    assert others.size == 7
    assert np.max(np.abs(coef[others])) < 1e-14 * np.max(np.abs(coef))
    sigma, centre, k0 = 0.1, np.array([0.5, 0.5]), np.array([2, 0])
    dh = c.I.astype(np.float64) - k0
    exact = np.prod(sigma * np.sqrt(2 * np.pi) * np.exp(-2 * np.pi ** 2 * sigma ** 2 * dh ** 2), axis=1) \
        * np.exp(-2j * np.pi * dh @ centre)
    ratio = coef[k] / exact
    big = np.abs(exact) > 1e-4 * np.abs(exact).max()
    assert big.sum() > 50 and np.allclose(ratio[big], ratio[big][0], rtol=1e-11, atol=0)
    # unit lattice-rule norm
    assert abs(np.mean(np.abs(c.u0) ** 2) - 1.0) < 1e-14


def test_box_d2_n1031_box_keys_and_completion():
    """Def. 2 on the box {-15..16}^2 with z = (1, 32), N = 1031: injective
    (1024 keys), the seven unowned keys are completed with their minimal-l2
    representatives (brute force)."""
    c = W.box_d2_n1031()
    k = O.keys(c.Z, c.n, c.I)
    assert np.unique(k).size == 1024
    h, s, fromI = O.index_set(c.Z, c.n, c.I)
    missing = np.where(~fromI)[0]
    assert missing.tolist() == list(range(529, 536))
    best = brute_min_l2(c.Z, c.n, 25, fixed=set(k.tolist()))
    for chi in missing:
        assert (s[chi], tuple(h[chi])) == best[chi]
    # box elements keep their keys
    assert np.array_equal(h[k], c.I)


def test_rank2_minimal_set_bruteforce():
    """Sec. 2.5: rank-2 keys chi = xi_1 n_2 + xi_2; minimal-l2 owners by brute force."""
    Z = np.array([[1, 5, 7], [0, 1, 3]])
    n = np.array([12, 4])
    h, s, _ = O.index_set(Z, n)
    best = brute_min_l2(Z, n, 6)
    assert len(best) == 48
    for chi in range(48):
        assert (s[chi], tuple(h[chi])) == best[chi]
    assert np.array_equal(O.keys(Z, n, h), np.arange(48))


def test_not_injective_and_unreachable():
    """Def. 2 violated -> error 2; points not distinct (gcd(N, z) > 1, Sec. 2.1)
    -> error 3."""
    Z, n = np.array([[1, 3]]), np.array([7])
    with pytest.raises(O.OracleError) as e:
        O.index_set(Z, n, np.array([[0, 0], [7, 0]]))
    assert e.value.code == 2
    with pytest.raises(O.OracleError) as e:
        O.index_set(np.array([[2, 4]]), np.array([8]))
    assert e.value.code == 3


def test_character_property():
    """Eq. (char): (1/n) sum_p exp(2 pi i h.p) is 1 on the dual lattice, 0 off it."""
    g = np.random.default_rng(7)
    for Z, n in [(np.array([[1, 34]]), np.array([55])),
                 (np.array([[1, 5, 7], [0, 1, 3]]), np.array([12, 4]))]:
        x = O.points(Z, n)
        N = x.shape[0]
        assert np.unique(np.round(x * N).astype(np.int64), axis=0).shape[0] == N
        for _ in range(200):
            hv = g.integers(-40, 41, size=Z.shape[1])
            val = np.mean(np.exp(2j * PI * (x @ hv)))
            dual = all((hv @ Z[i]) % n[i] == 0 for i in range(len(n)))
            assert abs(val - (1.0 if dual else 0.0)) < 1e-12


def test_points_match_workload_numerators():
    c = W.box_d2_n1031()
    x = O.points(c.Z, c.n)
    num = W.point_numerators(c.Z, c.n)
    assert np.array_equal(x, num / c.N)
    Z = np.array([[1, 5, 7], [0, 1, 3]])
    n = np.array([12, 4])
    assert np.array_equal(O.points(Z, n), W.point_numerators(Z, n) / 48)


# ----------------------------------------------------------------- transforms
@pytest.mark.parametrize("L", [1, 2, 3, 7, 16, 60, 97, 256, 1031])
def test_direct_dft_matches_numpy(L):
    g = np.random.default_rng(L)
    x = g.standard_normal(L) + 1j * g.standard_normal(L)
    assert np.allclose(O.dft_direct(x, -1), np.fft.fft(x), rtol=0, atol=1e-11 * max(1, L))
    assert np.allclose(O.dft_direct(x, +1), np.fft.ifft(x) * L, rtol=0, atol=1e-11 * max(1, L))


@pytest.mark.parametrize("L,method", [(2, "radix2"), (64, "radix2"), (4096, "radix2"),
                                      (1 << 16, "radix2"), (1031, "bluestein"),
                                      (4099, "bluestein"), (65521, "bluestein"),
                                      (3000, "bluestein"), (1031, "auto"), (12, "auto")])
def test_fast_transforms_match_numpy(L, method):
    g = np.random.default_rng(L)
    x = g.standard_normal(L) + 1j * g.standard_normal(L)
    for sign, ref in [(-1, np.fft.fft(x)), (+1, np.fft.ifft(x) * L)]:
        y = O.fft(x, sign, method)
        err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        assert err < 1e-14


def test_fftn_matches_numpy():
    g = np.random.default_rng(3)
    for shape in [(8, 4), (12, 4), (31, 32), (1031,)]:
        x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
        y = O.fftn(x.reshape(-1), shape, -1).reshape(shape)
        assert np.linalg.norm(y - np.fft.fftn(x)) / np.linalg.norm(y) < 1e-14


def test_single_mode_maps_to_its_key():
    """Thm. 1(iii) with eqs. (Fnx)/(Fn): the lattice samples of exp(2 pi i h.x)
    have unitary DFT sqrt(n) * delta at chi(h) (this fixes the sign)."""
    for Z, n in [(np.array([[1, 32]]), np.array([1031])),
                 (np.array([[1, 5, 7], [0, 1, 3]]), np.array([12, 4]))]:
        x = O.points(Z, n)
        N = x.shape[0]
        for hv in [np.array([16, 16] if Z.shape[1] == 2 else [1, -2, 3]),
                   np.array([-9, 16] if Z.shape[1] == 2 else [0, 0, 1])]:
            u = np.exp(2j * PI * (x @ hv))
            U = O.fftn(u, n, -1) / np.sqrt(N)
            chi = O.keys(Z, n, hv[None, :].astype(np.int32))[0]
            e = np.zeros(N, complex)
            e[chi] = np.sqrt(N)
            assert np.max(np.abs(U - e)) < 1e-10


# ----------------------------------------------------------------- Strang
def _plane_waves(Z, n, hs, coeffs):
    x = O.points(Z, n)
    return sum(c * np.exp(2j * PI * (x @ h)) for h, c in zip(hs, coeffs)), x


def test_unitarity_box_d2_n1031():
    """||S||_2 = 1 (proof of Thm. 3; Sec. 3.3): the norm is conserved to rounding."""
    c = W.box_d2_n1031()
    _, s, _ = O.index_set(c.Z, c.n, c.I)
    u, hist = O.strang_run(c.n, s, c.v, c.u0, c.gamma, c.dt, c.steps, history=True)
    n0 = np.mean(np.abs(c.u0) ** 2)
    assert abs(np.mean(np.abs(u) ** 2) - n0) / n0 < 1e-13
    assert np.max(np.abs(hist[0, :, 0] - n0)) < 1e-13


def test_free_evolution_closed_form():
    """v = 0: every mode evolves by exp(-i 2 pi^2 gamma ||h||^2 t) (eq. (Fourier-ODE)
    with f = 0; the exact propagator of Sec. 2.4 with W = 0)."""
    c = W.box_d2_n1031()
    h, s, _ = O.index_set(c.Z, c.n, c.I)
    g = np.random.default_rng(0)
    keys = g.choice(c.N, 12, replace=False)
    hs = h[keys].astype(np.int64)
    coeffs = g.standard_normal(12) + 1j * g.standard_normal(12)
    u0, x = _plane_waves(c.Z, c.n, hs, coeffs)
    T = c.dt * 37
    uT = O.strang_run(c.n, s, np.zeros(c.N), u0, c.gamma, c.dt, 37)
    exact = sum(cf * np.exp(-1j * 2 * PI * PI * c.gamma * (hh @ hh) * T) * np.exp(2j * PI * (x @ hh))
                for hh, cf in zip(hs, coeffs))
    assert np.linalg.norm(uT - exact) / np.linalg.norm(exact) < 1e-13


def test_constant_potential_global_phase():
    """v = v0 commutes with the Laplacian: an extra phase exp(-i v0 t / gamma)."""
    c = W.box_d2_n1031()
    h, s, _ = O.index_set(c.Z, c.n, c.I)
    g = np.random.default_rng(1)
    keys = g.choice(c.N, 8, replace=False)
    hs = h[keys].astype(np.int64)
    coeffs = g.standard_normal(8) + 1j * g.standard_normal(8)
    u0, x = _plane_waves(c.Z, c.n, hs, coeffs)
    v0, steps = 0.731, 25
    T = c.dt * steps
    uT = O.strang_run(c.n, s, np.full(c.N, v0), u0, c.gamma, c.dt, steps)
    exact = sum(cf * np.exp(-1j * (2 * PI * PI * c.gamma * (hh @ hh) + v0 / c.gamma) * T)
                * np.exp(2j * PI * (x @ hh)) for hh, cf in zip(hs, coeffs))
    assert np.linalg.norm(uT - exact) / np.linalg.norm(exact) < 1e-13


def _dense_coefficient_strang(Z, n, s, v, u0, gamma, dt, steps):
    """Eq. (StrangTDSE) in the coefficient domain with dense matrices:
    W_n = F V F^{-1} (eq. (Vn)), D_n = diag(4 pi^2 s) (eq. (Dn)), matrix
    exponentials by scipy.linalg.expm, F from its definition (eq. (Fn))."""
    N = u0.size
    shape = tuple(int(a) for a in np.atleast_1d(n))
    # r-D unitary DFT matrix as a Kronecker product of 1-D ones (eq. (Fnx))
    F = np.ones((1, 1), complex)
    for L in shape:
        k = np.arange(L)
        F = np.kron(F, np.exp(-2j * PI * np.outer(k, k) / L) / np.sqrt(L))
    Fi = F.conj().T
    Wn = F @ np.diag(v) @ Fi
    Dn = np.diag(4 * PI * PI * s.astype(float))
    Ew = scipy.linalg.expm(-1j * Wn * dt / (2 * gamma))
    Ed = scipy.linalg.expm(-1j * gamma * Dn * dt / 2)
    S = Ew @ Ed @ Ew
    uh = F @ u0
    for _ in range(steps):
        uh = S @ uh
    return Fi @ uh, (F, Fi, Wn, Dn)


@pytest.mark.parametrize("Z,n", [(np.array([[1, 34]]), np.array([55])),
                                 (np.array([[1, 5, 7], [0, 1, 3]]), np.array([12, 4]))])
def test_dense_bruteforce(Z, n):
    """Algorithm 1 against dense matrix exponentials (tiny n)."""
    h, s, _ = O.index_set(Z, n)
    num = W.point_numerators(Z, n)
    N = num.shape[0]
    v = W.v_product(num, N, 0.7) + 0.3 * W.v_sum_one_minus_cos(num, N)
    g = np.random.default_rng(2)
    u0 = g.standard_normal(N) + 1j * g.standard_normal(N)
    ref, _ = _dense_coefficient_strang(Z, n, s, v, u0, 0.2, 0.05, 20)
    got = O.strang_run(n, s, v, u0, 0.2, 0.05, 20)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13


def test_second_order_against_exact_propagator():
    """Thm. 3(ii): the Strang error against exp(-(i/gamma) W t - (i gamma/2) D t)
    (Sec. 2.4) falls by ~4 per halving of dt."""
    Z, n = np.array([[1, 34]]), np.array([55])
    h, s, _ = O.index_set(Z, n)
    num = W.point_numerators(Z, n)
    v = W.v_sum_one_minus_cos(num, 55)
    x = O.points(Z, n)
    u0 = np.exp(-np.sum((x - 0.5) ** 2, axis=1) / 0.05).astype(complex)
    gamma, T = 0.3, 0.4
    _, (F, Fi, Wn, Dn) = _dense_coefficient_strang(Z, n, s, v, u0, gamma, 0.1, 0)
    exact = Fi @ (scipy.linalg.expm(-1j * (Wn / gamma + gamma * Dn / 2) * T) @ (F @ u0))
    errs = []
    for m in (8, 16, 32, 64):
        errs.append(np.linalg.norm(O.strang_run(n, s, v, u0, gamma, T / m, m) - exact))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 1.9) & (orders < 2.1)), orders


def test_fourth_order_composition_against_exact_propagator():
    """The triple jump of Strang steps (weights summing to 1, w1^3 + w0^3 + w1^3
    = 0) converges at fourth order against the exact propagator of the
    lattice Hamiltonian: the error falls by ~16 per halving of dt."""
    Z, n = np.array([[1, 34]]), np.array([55])
    h, s, _ = O.index_set(Z, n)
    num = W.point_numerators(Z, n)
    v = W.v_sum_one_minus_cos(num, 55)
    x = O.points(Z, n)
    u0 = np.exp(-np.sum((x - 0.5) ** 2, axis=1) / 0.05).astype(complex)
    gamma, T = 0.3, 0.4
    _, (F, Fi, Wn, Dn) = _dense_coefficient_strang(Z, n, s, v, u0, gamma, 0.1, 0)
    exact = Fi @ (scipy.linalg.expm(-1j * (Wn / gamma + gamma * Dn / 2) * T) @ (F @ u0))
    w = O.composition_weights(4)
    assert abs(sum(w) - 1.0) < 1e-15 and abs(sum(x ** 3 for x in w)) < 1e-14
    errs = [np.linalg.norm(O.composed_run(n, s, v, u0, gamma, T / m, m) - exact) for m in (16, 32, 64, 128)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 3.85) & (orders < 4.15)), orders
    # order 2 is the plain Strang run
    assert np.allclose(O.composed_run(n, s, v, u0, gamma, 0.05, 3, order=2),
                       O.strang_run(n, s, v, u0, gamma, 0.05, 3), rtol=0, atol=1e-13)


def _tdv_case():
    Z, n = np.array([[1, 34]]), np.array([55])
    h, s, _ = O.index_set(Z, n)
    num = W.point_numerators(Z, n)
    v = W.v_sum_one_minus_cos(num, 55)
    v1 = W.v_product(num, 55, 0.7)
    x = O.points(Z, n)
    u0 = np.exp(-np.sum((x - 0.5) ** 2, axis=1) / 0.05).astype(complex)
    return Z, n, s, v, v1, u0


def test_time_dependent_special_cases():
    """A constant coefficient f = c is the time-independent run under v + c v1;
    a spatially constant v1 with f linear in t only adds the global phase
    exp(-(i/gamma) int f dt) (the substep boundaries' trapezoid sums are exact
    for linear f, also across the backward middle substep of order 4)."""
    Z, n, s, v, v1, u0 = _tdv_case()
    gamma, dt, m = 0.3, 0.05, 6
    for order in (2, 4):
        a = O.composed_run(n, s, v, u0, gamma, dt, m, order=order, v1=v1, f=lambda t: 0.8)
        b = O.composed_run(n, s, v + 0.8 * v1, u0, gamma, dt, m, order=order)
        assert np.allclose(a, b, rtol=0, atol=1e-13), order
        t0, T = 0.2, m * dt
        lin = lambda t: 1.5 - 2.0 * t
        integral = 1.5 * T - (((t0 + T) ** 2) - t0 ** 2)
        a = O.composed_run(n, s, v, u0, gamma, dt, m, order=order, v1=np.ones(55), f=lin, t0=t0)
        b = O.composed_run(n, s, v, u0, gamma, dt, m, order=order) * np.exp(-1j * integral / gamma)
        assert np.allclose(a, b, rtol=0, atol=1e-13), order


def test_time_dependent_orders_against_ode_solution():
    """v(x, t) = v(x) + f(t) v1(x) with f(t) = 1 + 2 sin 5t: against a DOP853
    solution (rtol 1e-13) of the lattice ODE i gamma u' = (gamma^2/2)
    F^-1 D_n F u + v(., t) u, the composition converges at order 2 (Strang)
    and 4 (triple jump)."""
    Z, n, s, v, v1, u0 = _tdv_case()
    gamma, T = 0.3, 0.4
    _, (F, Fi, Wn, Dn) = _dense_coefficient_strang(Z, n, s, v, u0, gamma, 0.1, 0)
    Kpt = Fi @ (gamma * Dn / 2) @ F
    f = lambda t: 1.0 + 2.0 * np.sin(5.0 * t)
    sol = scipy.integrate.solve_ivp(lambda t, y: -1j * ((v + f(t) * v1) / gamma * y + Kpt @ y), (0, T), u0,
                                    method="DOP853", rtol=1e-13, atol=1e-13)
    ref = sol.y[:, -1]
    for order, ms, lo, hi in ((2, (16, 32, 64), 1.95, 2.05), (4, (32, 64, 128), 3.85, 4.15)):
        errs = [np.linalg.norm(O.composed_run(n, s, v, u0, gamma, T / m, m, order=order, v1=v1, f=f) - ref)
                for m in ms]
        orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert np.all((orders > lo) & (orders < hi)), (order, orders)


def test_projection_error_trigonometric_polynomial_and_aliased_mode():
    """Sec. 3.4: a trigonometric polynomial on the index set is reproduced
    exactly (both error terms vanish); a single mode outside it aliases onto
    its key, giving e_total^2 = 1 (its own coefficient) + 1 (the aliased one)."""
    Z, n = np.array([[1, 34]]), np.array([55])
    h, s, _ = O.index_set(Z, n)
    num = W.point_numerators(Z, n)
    keys = O.keys(Z, n, h)
    g = np.random.default_rng(5)
    pick = g.choice(55, 6, replace=False)
    c = g.standard_normal(6) + 1j * g.standard_normal(6)
    u = np.zeros(55, dtype=complex)
    ghat = np.zeros(55, dtype=complex)
    for i, ck in zip(pick, c):
        u += ck * np.exp(2j * np.pi * ((num @ h[i]) % 55) / 55)
        ghat[keys[i]] = ck
    s0, s1 = O.projection_error(n, u, ghat)[0]
    assert abs(s0 - np.sum(np.abs(c) ** 2)) < 1e-12 and s1 < 1e-24
    e2 = np.sum(np.abs(c) ** 2) - s0 + s1
    assert abs(e2) < 1e-12
    # h_out = h + (55, 0) has the key of h but is not in the minimal set
    h_in = h[pick[0]]
    h_out = h_in + np.array([55, 0])
    assert O.keys(Z, n, h_out[None])[0] == keys[pick[0]]
    u = np.exp(2j * np.pi * (num @ h_out) / 55.0)
    s0, s1 = O.projection_error(n, u, np.zeros(55))[0]
    assert s0 == 0.0 and abs(s1 - 1.0) < 1e-13
    assert abs((1.0 - s0 + s1) - 2.0) < 1e-13


def test_projection_error_gaussian_against_direct_integral():
    """e_total^2 of the paper's g1 on the Fig. 1 lattice, from the key sums,
    against the definition int |g - g_a|^2 dx by a tensor Gauss-Legendre rule
    (g_a the trigonometric polynomial on the index set with the lattice
    coefficients)."""
    Z, n = np.array([[1, 34]]), np.array([55])
    h, s, _ = O.index_set(Z, n)
    keys = O.keys(Z, n, h)
    hk = np.empty_like(h)
    hk[keys] = h
    num = W.point_numerators(Z, n)
    gamma = 1.0
    tables, norm2 = W.paper_g1_coefficients(2, gamma, 64)
    ghat = W.coefficients_at(hk, tables)
    u = W.paper_g1(num, 55, gamma, normalize=False)
    s0, s1 = O.projection_error(n, u, ghat)[0]
    e2 = norm2 - s0 + s1
    ga = O.fftn(u, n) / 55.0                    # lattice coefficients in key order
    t, w = np.polynomial.legendre.leggauss(300)
    x, w = 0.5 * (t + 1.0), 0.5 * w
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    gx = np.exp(-((2 * np.pi * X1 - 1.5 * np.pi) ** 2 + (2 * np.pi * X2 - np.pi) ** 2) / gamma)
    gax = sum(ga[kk] * np.exp(2j * np.pi * (hk[kk, 0] * X1 + hk[kk, 1] * X2)) for kk in range(55))
    direct = float(np.sum(np.outer(w, w) * np.abs(gx - gax) ** 2))
    assert direct > 1e-6
    assert abs(e2 - direct) < 1e-12 * max(1.0, norm2), (e2, direct)


def test_box_d2_n1031_second_order_paper_protocol():
    """Sec. 3.2 protocol: reference at dt = 1e-4, errors at larger dt, T fixed,
    observed order 2 (here T = 0.2 so the reference stays cheap)."""
    c = W.box_d2_n1031()
    _, s, _ = O.index_set(c.Z, c.n, c.I)
    T = 0.2
    ref = O.strang_run(c.n, s, c.v, c.u0, c.gamma, 1e-4, int(round(T / 1e-4)))
    errs = []
    for dt in (0.04, 0.02, 0.01, 0.005):
        m = int(round(T / dt))
        errs.append(np.sqrt(np.mean(np.abs(O.strang_run(c.n, s, c.v, c.u0, c.gamma, dt, m) - ref) ** 2)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 1.9) & (orders < 2.1)), orders


def test_rank1_equals_tensor_grid_d2():
    """Regular grids are lattices (Sec. 2.1): z = (32, 31), N = 992 samples
    exactly the 31 x 32 grid (p_k = (k/31, k/32) mod 1), and the box
    {-15..15} x {-15..16} is a full anti-aliasing set, so the rank-1 solver
    equals a 2-D grid split-step solver built on numpy.fft."""
    Z, n = np.array([[32, 31]]), np.array([992])
    I = np.array([[a, b] for a in range(-15, 16) for b in range(-15, 17)], dtype=np.int32)
    h, s, fromI = O.index_set(Z, n, I)
    assert fromI.all()
    num = W.point_numerators(Z, n)
    k = np.arange(992)
    a, b = k % 31, k % 32
    assert np.array_equal(num[:, 0], (a * 32) % 992) and np.array_equal(num[:, 1], (b * 31) % 992)
    x1, x2 = np.arange(31) / 31, np.arange(32) / 32
    X1, X2 = np.meshgrid(x1, x2, indexing="ij")
    vgrid = (1 - np.cos(2 * PI * X1)) + 0.5 * np.cos(2 * PI * (X1 + 2 * X2))
    u0grid = np.exp(-((X1 - 0.4) ** 2 + (X2 - 0.6) ** 2) / 0.02) * np.exp(2j * PI * 3 * X1)
    f1 = np.fft.fftfreq(31, 1 / 31)
    f2 = np.fft.fftfreq(32, 1 / 32)
    F1, F2 = np.meshgrid(f1, f2, indexing="ij")
    F2 = np.where(F2 == -16, 16, F2)   # the box owns +16, not -16
    ref = grid_strang(vgrid, u0grid, 0.1, 0.01, 50, (F1, F2))
    got = O.strang_run(n, s, vgrid[a, b], u0grid[a, b], 0.1, 0.01, 50)
    assert np.linalg.norm(got - ref[a, b]) / np.linalg.norm(ref) < 1e-12


def test_rank2_regular_grid_equals_tensor_solver():
    """A rank-2 lattice with Z = I is the regular 8 x 4 grid (Sec. 2.1, 2.5);
    with the box as index set the rank-2 solver equals the numpy grid solver."""
    Z, n = np.array([[1, 0], [0, 1]]), np.array([8, 4])
    I = np.array([[a, b] for a in range(-3, 5) for b in range(-1, 3)], dtype=np.int32)
    h, s, fromI = O.index_set(Z, n, I)
    assert fromI.all()
    X1, X2 = np.meshgrid(np.arange(8) / 8, np.arange(4) / 4, indexing="ij")
    vgrid = 1 + np.cos(2 * PI * X1) * np.sin(2 * PI * X2)
    u0grid = np.exp(2j * PI * X1) + 0.3 * np.exp(-2j * PI * X2)
    F1 = np.fft.fftfreq(8, 1 / 8)
    F1 = np.where(F1 == -4, 4, F1)
    F2 = np.fft.fftfreq(4, 1 / 4)
    F2 = np.where(F2 == -2, 2, F2)
    G1, G2 = np.meshgrid(F1, F2, indexing="ij")
    ref = grid_strang(vgrid, u0grid, 0.25, 0.02, 30, (G1, G2))
    got = O.strang_run(n, s, vgrid.reshape(-1), u0grid.reshape(-1), 0.25, 0.02, 30)
    assert np.linalg.norm(got - ref.reshape(-1)) / np.linalg.norm(ref) < 1e-13


def test_reversibility():
    """The Strang scheme is symmetric (Sec. 2.3): S(-dt) S(dt) = I."""
    c = W.box_d2_n1031()
    _, s, _ = O.index_set(c.Z, c.n, c.I)
    u = O.strang_run(c.n, s, c.v, c.u0, c.gamma, c.dt, 40)
    back = O.strang_run(c.n, s, c.v, u, c.gamma, -c.dt, 40)
    assert np.linalg.norm(back - c.u0) / np.linalg.norm(c.u0) < 1e-13


def test_diagnostics_single_mode():
    """Sec. 3.3: for u = exp(2 pi i h.x) (h in A), ||u||^2 = 1 and
    <Hu, u> = 2 pi^2 gamma ||h||^2 + mean(v)/gamma."""
    c = W.box_d2_n1031()
    h, s, _ = O.index_set(c.Z, c.n, c.I)
    hv = h[123].astype(np.int64)
    x = O.points(c.Z, c.n)
    u = np.exp(2j * PI * (x @ hv))
    nn, E = O.diagnostics(c.n, s, c.v, u, c.gamma)
    assert abs(nn - 1) < 1e-13
    assert abs(E - (2 * PI * PI * c.gamma * (hv @ hv) + np.mean(c.v) / c.gamma)) < 1e-10


def test_bluestein_steps_against_long_double():
    """A prime lattice (N = 4099, Bluestein transforms) stepped 400 times
    against the same steps in long double (the kinetic part of a step as the
    cyclic convolution with the kernel F^-1 K F, evaluated by long-double FFTs
    through scipy.fft): the chirp-z tables enter every transform, so their
    rounding adds up over the steps unless they are exact to double
    precision; the drift stays at the level of the double data path."""
    import scipy.fft as sf
    N, d, m, gamma, dt = 4099, 3, 400, 0.05, 2e-3
    g = np.random.default_rng(3)
    z = W.korobov(N, d, g)
    Z, n = z.reshape(1, -1), np.array([N])
    num = W.point_numerators(Z, n)
    _, s, _ = O.index_set(Z, n)
    v = W.cosine_series(d, 16, g).at(num, N)
    u0 = W.seeded_packet(num, N, g)
    L = 16384
    pil = np.longdouble("3.14159265358979323846264338327950288")
    th = 2 * pil ** 2 * np.longdouble(gamma) * np.longdouble(dt)
    k = sf.ifft(np.exp(-1j * (th * s.astype(np.longdouble))).astype(np.clongdouble))
    gk = np.zeros(L, np.clongdouble)
    gk[:N] = k
    gk[L - N + 1:] = k[1:]
    G = sf.fft(gk)
    P = np.exp(-1j * (np.longdouble(dt) * v.astype(np.longdouble) / (2 * np.longdouble(gamma))))
    x = u0.astype(np.clongdouble)
    for _ in range(m):
        xp = np.zeros(L, np.clongdouble)
        xp[:N] = x * P
        x = sf.ifft(sf.fft(xp) * G)[:N] * P
    got = O.strang_run(n, s, v, u0, gamma, dt, m)
    e = float(np.linalg.norm(got - x) / np.linalg.norm(x))
    assert e < 1.5e-13, e


def test_history_potential_term():
    """The history's third column is the potential term (1/(gamma N)) sum v |u|^2
    of <Hu, u> (Sec. 3.3).  A single mode has |u| = 1 at every point and the
    lattice rule integrates cos(2 pi x_j) to 0 (z_j != 0 mod N), so under
    v = sum_j (1 - cos 2 pi x_j) the term of u0 is d / gamma; under a constant
    v0 it is v0 ||u||^2 / gamma at every step."""
    c = W.box_d2_n1031()
    h, s, _ = O.index_set(c.Z, c.n, c.I)
    hv = h[77].astype(np.int64)
    x = O.points(c.Z, c.n)
    u0 = np.exp(2j * PI * (x @ hv))
    _, hist = O.strang_run(c.n, s, c.v, u0, c.gamma, c.dt, 3, history=True)
    assert abs(hist[0, 0, 2] - 2.0 / c.gamma) < 1e-12
    assert abs(hist[0, 0, 1] - (2 * PI * PI * c.gamma * (hv @ hv) + 2.0 / c.gamma)) < 1e-9
    v0 = 0.75
    _, hist = O.strang_run(c.n, s, np.full(c.N, v0), c.u0, c.gamma, c.dt, 9, history=True)
    assert np.max(np.abs(hist[0, :, 2] - v0 * hist[0, :, 0] / c.gamma)) < 1e-12


# ----------------------------------------------------------------- adjoint
def _small_problem(batch=1, shared=True):
    Z, n = np.array([[1, 34]]), np.array([55])
    h, s, _ = O.index_set(Z, n)
    num = W.point_numerators(Z, n)
    g = np.random.default_rng(11)
    v = W.v_sum_one_minus_cos(num, 55) + 0.2 * g.standard_normal(55)
    if not shared:
        v = np.stack([v + 0.1 * k for k in range(batch)])
    u0 = g.standard_normal((batch, 55)) + 1j * g.standard_normal((batch, 55))
    return n, s, v, u0


def test_vjp_abs_sums_single_step_dense():
    """gv_abs (the conditioning output of the VJP) on one step, N = 55: with
    dense matrices (DFT matrix F, K, P), a = P u0, b = F^H K F a,
    y = conj(P) gT, mu = F^H conj(K) F y, the two terms per point are
    t1 = c Im(conj(y) b) and t2 = c Im(conj(mu) a) (c = dt / (2 gamma)):
    gv = t1 + t2 and gv_abs = |t1| + |t2|; over several steps and states
    gv_abs >= |gv|."""
    n, s, v, u0 = _small_problem(batch=1)
    N, gamma, dt = 55, 0.3, 0.07
    g = np.random.default_rng(12)
    gT = g.standard_normal(N) + 1j * g.standard_normal(N)
    _, gv, ga = O.strang_vjp(n, s, v, u0[0], gT, gamma, dt, 1, return_abs=True)
    k = np.arange(N)
    F = np.exp(-2j * PI * np.outer(k, k) / N) / np.sqrt(N)
    K = np.exp(-1j * 2 * PI * PI * gamma * dt * s)
    P = np.exp(-1j * dt * v / (2 * gamma))
    c = dt / (2 * gamma)
    a = P * u0[0]
    b = F.conj().T @ (K * (F @ a))
    y = np.conj(P) * gT
    mu = F.conj().T @ (np.conj(K) * (F @ y))
    t1, t2 = c * np.imag(np.conj(y) * b), c * np.imag(np.conj(mu) * a)
    assert np.max(np.abs(gv - (t1 + t2))) < 1e-13
    assert np.max(np.abs(ga - (np.abs(t1) + np.abs(t2)))) < 1e-13
    n, s, v, u0 = _small_problem(batch=3)
    gT = g.standard_normal(u0.shape) + 1j * g.standard_normal(u0.shape)
    _, gv, ga = O.strang_vjp(n, s, v, u0, gT, gamma, dt, 9, return_abs=True)
    assert np.all(ga >= np.abs(gv) - 1e-15) and np.max(ga - np.abs(gv)) > 0


def test_vjp_dot_product():
    """The state map is linear: Re<y, S^m x> = Re<(S^m)^H y, x>."""
    n, s, v, u0 = _small_problem(batch=2)
    g = np.random.default_rng(5)
    y = g.standard_normal(u0.shape) + 1j * g.standard_normal(u0.shape)
    Sx = O.strang_run(n, s, v, u0, 0.2, 0.03, 60)
    g0, _ = O.strang_vjp(n, s, v, u0, y, 0.2, 0.03, 60)
    assert abs(np.vdot(y, Sx) - np.vdot(g0, u0)) < 1e-11 * np.linalg.norm(y) * np.linalg.norm(u0)


@pytest.mark.parametrize("shared", [True, False])
def test_vjp_potential_central_differences(shared):
    """dJ/dv_k against FP64 central differences, J = (1/N) sum |u(T) - t|^2."""
    n, s, v, u0 = _small_problem(batch=2, shared=shared)
    g = np.random.default_rng(6)
    tgt = g.standard_normal(u0.shape) + 1j * g.standard_normal(u0.shape)
    gamma, dt, m = 0.2, 0.03, 60   # 60 > 50 exercises the checkpoint segments
    N = 55

    def J(vv):
        uT = O.strang_run(n, s, vv, u0, gamma, dt, m)
        return np.sum(np.abs(uT - tgt) ** 2) / N

    uT = O.strang_run(n, s, v, u0, gamma, dt, m)
    g0, gv = O.strang_vjp(n, s, v, u0, 2.0 * (uT - tgt) / N, gamma, dt, m)
    eps = 1e-6
    for k in (0, 7, 31, 54):
        if shared:
            e = np.zeros_like(v); e[k] = eps
            fd = (J(v + e) - J(v - e)) / (2 * eps)
            assert abs(fd - gv[k]) < 1e-7 * max(1.0, abs(fd))
        else:
            for b in range(2):
                e = np.zeros_like(v); e[b, k] = eps
                fd = (J(v + e) - J(v - e)) / (2 * eps)
                assert abs(fd - gv[b, k]) < 1e-7 * max(1.0, abs(fd))
    # gradient with respect to u0 (real and imaginary parts)
    for k in (3, 40):
        e = np.zeros_like(u0); e[1, k] = eps

        def Ju(uu):
            return np.sum(np.abs(O.strang_run(n, s, v, uu, gamma, dt, m) - tgt) ** 2) / N
        fr = (Ju(u0 + e) - Ju(u0 - e)) / (2 * eps)
        fi = (Ju(u0 + 1j * e) - Ju(u0 - 1j * e)) / (2 * eps)
        assert abs(fr - g0[1, k].real) < 1e-7 and abs(fi - g0[1, k].imag) < 1e-7
