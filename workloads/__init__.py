"""Seeded synthetic inputs shaped like the workloads of arXiv:1808.06357.

This module is shared by the oracle side and the product side.  It holds none
of the method's arithmetic: it only builds the *inputs* of Algorithm 1 -- a
lattice (generating vectors, moduli), an index set, the potential v and the
initial condition g evaluated at the lattice points, gamma, dt and the step
count.  Lattice points are produced from their exact integer definition
(Sec. 2.1, Def. 1): coordinate j of point kappa is num_j(kappa) / n with

    num_j(kappa) = (sum_i z_{i,j} k_i (n / n_i)) mod n,

so every periodic input function is evaluated through the integer numerator
(cos(2 pi h.x) uses (h . num) mod n, never a rounded x).

Generating vectors for the hyperbolic-cross configurations come from a seeded
component-by-component search for a *reconstructing* lattice (the index set
must map injectively to keys).  It plays the role of the paper's external
construction script (Sec. 3.1); both the oracle and the product planner check
injectivity of its result independently.

Seeds: each workload has a seed index i (box_d2_n1031 0, cross_d6_n1048573 1,
mixed_batch 2, rank2_d10_n4096x256 3, adjoint_d4_n65521 4) and draws from numpy
PCG64(SeedSequence(1808_06357 + i)), spawned into the sub-streams [z-search, v,
u0, batch-shapes, hidden-v].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 1808_06357
_STREAMS = {"z": 0, "v": 1, "u0": 2, "shapes": 3, "hidden_v": 4}


def rng(seed_index: int, stream: str) -> np.random.Generator:
    ss = np.random.SeedSequence(SEED_BASE + seed_index).spawn(len(_STREAMS))[_STREAMS[stream]]
    return np.random.Generator(np.random.PCG64(ss))


# ---------------------------------------------------------------- lattice inputs
def point_numerators(Z, n) -> np.ndarray:
    """Integer numerators num (N x d, int64) of the lattice points in kappa
    order (Def. 1 and the lexicographic ordering of Sec. 2.5)."""
    Z = np.atleast_2d(np.asarray(Z, dtype=np.int64))
    n = np.atleast_1d(np.asarray(n, dtype=np.int64))
    r, d = Z.shape
    N = int(np.prod(n))
    kappa = np.arange(N, dtype=np.int64)
    num = np.zeros((N, d), dtype=np.int64)
    rem = kappa.copy()
    ks = []
    for i in range(r - 1, -1, -1):
        ks.append(rem % n[i])
        rem //= n[i]
    ks = ks[::-1]
    for i in range(r):
        scale = N // int(n[i])
        for j in range(d):
            zj = int(Z[i, j]) % int(n[i])
            num[:, j] = (num[:, j] + (ks[i] * zj % int(n[i])) * scale) % N
    return num


def box(lo: int, hi: int, d: int) -> np.ndarray:
    """All h in {lo..hi}^d, lexicographic."""
    axes = [np.arange(lo, hi + 1, dtype=np.int32)] * d
    g = np.meshgrid(*axes, indexing="ij")
    return np.stack([a.reshape(-1) for a in g], axis=1)


def hyperbolic_cross(d: int, R: int) -> np.ndarray:
    """{h in Z^d : prod_j max(1, |h_j|) <= R}, lexicographic."""
    out: List[List[int]] = []

    def rec(prefix, budget):
        if len(prefix) == d:
            out.append(list(prefix))
            return
        for a in range(-budget, budget + 1):
            rec(prefix + [a], budget // max(1, abs(a)))

    rec([], R)
    return np.asarray(out, dtype=np.int32).reshape(-1, d)


def _unique_count(keys: np.ndarray) -> int:
    return int(np.unique(keys).size)


def cbc_rank1(H: np.ndarray, N: int, g: np.random.Generator, tries: int = 4000) -> np.ndarray:
    """Seeded reconstructing CBC: z_1 = 1; component j takes the first seeded
    candidate in [1, N-1] coprime to N for which h -> h.z mod N is injective on
    the projection of H onto coordinates 1..j."""
    d = H.shape[1]
    z = [1]
    for j in range(1, d):
        proj = np.unique(H[:, : j + 1], axis=0).astype(np.int64)
        base = (proj[:, :j] @ np.asarray(z, dtype=np.int64)) % N
        for _ in range(tries):
            c = int(g.integers(1, N))
            if math.gcd(c, N) != 1:
                continue
            if _unique_count((base + proj[:, j] * c) % N) == proj.shape[0]:
                z.append(c)
                break
        else:
            raise RuntimeError(f"CBC failed at component {j + 1}")
    return np.asarray(z, dtype=np.int64)


def cbc_rank2(H: np.ndarray, n1: int, n2: int, g: np.random.Generator, tries: int = 4000):
    """Seeded reconstructing CBC for a rank-2 lattice with power-of-two moduli
    (n1, n2); keys (h.z1 mod n1) * n2 + (h.z2 mod n2) injective on the
    projections of H.  z1 = (1, odd, ...), z2 = (0, odd, ...): if every
    component of both vectors were odd, k = (n1/2, n2/2) would map to the
    origin and only n/2 points would be distinct; the leading (1, 0) column
    makes all n1 * n2 points distinct."""
    d = H.shape[1]
    z1, z2 = [1], [0]
    for j in range(1, d):
        proj = np.unique(H[:, : j + 1], axis=0).astype(np.int64)
        b1 = (proj[:, :j] @ np.asarray(z1, dtype=np.int64)) % n1
        b2 = (proj[:, :j] @ np.asarray(z2, dtype=np.int64)) % n2
        for _ in range(tries):
            c1 = int(g.integers(0, n1 // 2)) * 2 + 1
            c2 = int(g.integers(0, n2 // 2)) * 2 + 1
            k = ((b1 + proj[:, j] * c1) % n1) * n2 + (b2 + proj[:, j] * c2) % n2
            if _unique_count(k) == proj.shape[0]:
                z1.append(c1)
                z2.append(c2)
                break
        else:
            raise RuntimeError(f"rank-2 CBC failed at component {j + 1}")
    return np.stack([np.asarray(z1, dtype=np.int64), np.asarray(z2, dtype=np.int64)])


def korobov(N: int, d: int, g: np.random.Generator) -> np.ndarray:
    """z = (1, a, a^2, ..., a^{d-1}) mod N with a seeded a coprime to N."""
    while True:
        a = int(g.integers(2, N))
        if math.gcd(a, N) == 1:
            break
    z = [1]
    for _ in range(d - 1):
        z.append(z[-1] * a % N)
    return np.asarray(z, dtype=np.int64)


def l2_ball_radius2(d: int, count: int) -> int:
    """Smallest R^2 such that {h in Z^d : ||h||^2 <= R^2} holds >= count vectors
    (counts per squared norm, one coordinate at a time)."""
    smax = 4
    while True:
        c = np.zeros(smax + 1, dtype=np.int64)
        c[0] = 1
        for _ in range(d):
            nxt = c.copy()
            x = 1
            while x * x <= smax:
                nxt[x * x:] += 2 * c[: smax + 1 - x * x]
                x += 1
            c = nxt
        hit = np.nonzero(np.cumsum(c) >= count)[0]
        if hit.size:
            return int(hit[0])
        smax *= 2


def l2_ball(d: int, r2: int) -> np.ndarray:
    """All h in Z^d with ||h||^2 <= r2 (unordered)."""
    a = math.isqrt(r2)
    xs = np.arange(-a, a + 1, dtype=np.int64)
    pts = np.zeros((1, 0), dtype=np.int64)
    norms = np.zeros(1, dtype=np.int64)
    for _ in range(d):
        nn = norms[:, None] + xs[None, :] ** 2
        i, j = np.nonzero(nn <= r2)
        pts = np.concatenate([pts[i], xs[j, None]], axis=1)
        norms = nn[i, j]
    return pts


def korobov_good(N: int, d: int, g: np.random.Generator, candidates: int = 8) -> np.ndarray:
    """The best of `candidates` seeded Korobov vectors: the one whose keys
    h.z mod N cover the most distinct values on the l2 ball of about N/2
    frequencies.  Poor vectors (short dual vectors, e.g. a of small
    multiplicative order) leave many keys uncovered there, which makes their
    minimal-l2 completion reach far out and cost a large enumeration."""
    ball = l2_ball(d, l2_ball_radius2(d, N // 2)).astype(np.float64)  # exact: |h.z| < 2^53
    best, best_cov = None, -1
    for _ in range(candidates):
        z = korobov(N, d, g)
        keys = np.mod(ball @ z.astype(np.float64), N).astype(np.int64)
        cov = int(np.count_nonzero(np.bincount(keys, minlength=N)))
        if cov > best_cov:
            best, best_cov = z, cov
    return best


# ---------------------------------------------------------------- input functions
def _cos2pi(num_mod: np.ndarray, N: int) -> np.ndarray:
    return np.cos(2.0 * np.pi * (num_mod % N).astype(np.float64) / N)


def v_sum_one_minus_cos(num: np.ndarray, N: int) -> np.ndarray:
    """v(x) = sum_j (1 - cos 2 pi x_j)."""
    return np.sum(1.0 - _cos2pi(num, N), axis=1)


def v_product(num: np.ndarray, N: int, amp: float = 0.5) -> np.ndarray:
    """v(x) = prod_j (1 + amp cos 2 pi x_j) - 1."""
    return np.prod(1.0 + amp * _cos2pi(num, N), axis=1) - 1.0


def v_smooth_paper(num: np.ndarray, N: int) -> np.ndarray:
    """The paper's smooth potential v1 = prod_j (1 - cos 2 pi x_j) (Sec. 3.2)."""
    return np.prod(1.0 - _cos2pi(num, N), axis=1)


def v_harmonic_paper(num: np.ndarray, N: int) -> np.ndarray:
    """The paper's harmonic potential v2 = 1/2 sum_j (2 pi x_j - pi)^2 (Sec. 3.2)."""
    x = num.astype(np.float64) / N
    return 0.5 * np.sum((2.0 * np.pi * x - np.pi) ** 2, axis=1)


@dataclass
class CosineSeries:
    """v(x) = sum_t a_t cos(2 pi h_t . x)."""
    h: np.ndarray          # (T, d) int64
    a: np.ndarray          # (T,) float64

    def at(self, num: np.ndarray, N: int) -> np.ndarray:
        v = np.zeros(num.shape[0])
        for t in range(self.h.shape[0]):
            v += self.a[t] * _cos2pi(num @ self.h[t], N)
        return v

    def basis(self, num: np.ndarray, N: int) -> np.ndarray:
        """B[t, k] = cos(2 pi h_t . p_k): dv_k / da_t."""
        return np.stack([_cos2pi(num @ self.h[t], N) for t in range(self.h.shape[0])])


def cosine_series(d: int, terms: int, g: np.random.Generator, hmax: int = 2) -> CosineSeries:
    hs = []
    while len(hs) < terms:
        h = g.integers(-hmax, hmax + 1, size=d)
        if np.any(h != 0):
            hs.append(h)
    a = g.uniform(-0.5, 0.5, size=terms)
    return CosineSeries(np.asarray(hs, dtype=np.int64), a)


def gaussian_packet(num: np.ndarray, N: int, center, k0, sigma: float = 0.1) -> np.ndarray:
    """Periodised Gaussian packet prod_j G(x_j - c_j) * exp(2 pi i k0 . x),
    G(t) = sum_{m=-3..3} exp(-(t-m)^2 / (2 sigma^2)), sampled at the points and
    scaled so that (1/N) sum_k |u_k|^2 = 1 (the lattice-rule L2 norm)."""
    x = num.astype(np.float64) / N
    amp = np.ones(num.shape[0])
    for j in range(num.shape[1]):
        t = x[:, j] - center[j]
        G = np.zeros_like(t)
        for m in range(-3, 4):
            G += np.exp(-((t - m) ** 2) / (2.0 * sigma * sigma))
        amp *= G
    ph = (num @ np.asarray(k0, dtype=np.int64)) % N
    u = amp * np.exp(2j * np.pi * ph.astype(np.float64) / N)
    u /= np.sqrt(np.mean(np.abs(u) ** 2))
    return u.astype(np.complex128)


def projected_packet(Z: np.ndarray, n: np.ndarray, I: np.ndarray, center, k0, sigma: float = 0.1) -> np.ndarray:
    """The periodised Gaussian packet of gaussian_packet projected onto the
    span of exp(2 pi i h.x), h in I: its exact Fourier coefficients
    prod_j sigma sqrt(2 pi) exp(-2 pi^2 sigma^2 (h_j - k0_j)^2)
    exp(-2 pi i (h_j - k0_j) c_j) on I (zero elsewhere), summed at the
    lattice points (Def. 1, rank 1 or 2) and scaled so that
    (1/N) sum_k |u_k|^2 = 1."""
    Z = np.asarray(Z, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    I = np.asarray(I, dtype=np.int64)
    N = int(np.prod(n))
    num = point_numerators(Z, n)
    dh = I - np.asarray(k0, dtype=np.int64)[None, :]
    c = np.asarray(center, dtype=np.float64)
    coef = np.prod(sigma * np.sqrt(2.0 * np.pi) * np.exp(-2.0 * np.pi ** 2 * sigma ** 2 * dh.astype(np.float64) ** 2),
                   axis=1) * np.exp(-2j * np.pi * (dh.astype(np.float64) @ c))
    u = np.zeros(num.shape[0], dtype=np.complex128)
    for t in range(I.shape[0]):
        ph = (num @ I[t]) % N  # h.x_k = (h.num_k mod N) / N for the point numerators
        u += coef[t] * np.exp(2j * np.pi * ph.astype(np.float64) / N)
    u /= np.sqrt(np.mean(np.abs(u) ** 2))
    return u


def seeded_packet(num: np.ndarray, N: int, g: np.random.Generator, sigma: float = 0.1):
    d = num.shape[1]
    c = g.uniform(0.3, 0.7, size=d)
    k0 = g.integers(-2, 3, size=d)
    return gaussian_packet(num, N, c, k0, sigma)


def paper_g1(num: np.ndarray, N: int, gamma: float, normalize: bool = True) -> np.ndarray:
    """The paper's Gaussian initial condition g1 (Sec. 3.2) at the lattice
    points, scaled to unit lattice-rule norm unless normalize is False."""
    x = num.astype(np.float64) / N
    e = (2 * np.pi * x[:, 0] - 1.5 * np.pi) ** 2 + np.sum((2 * np.pi * x[:, 1:] - np.pi) ** 2, axis=1)
    u = np.exp(-e / gamma).astype(np.complex128)
    if normalize:
        u /= np.sqrt(np.mean(np.abs(u) ** 2))
    return u


def paper_g2(num: np.ndarray, N: int, gamma: float, normalize: bool = True) -> np.ndarray:
    """The paper's hat initial condition g2 (Sec. 3.2) at the lattice points:
    prod_j max(0, 1 - |y_j| / a) with y_1 = 2 pi x_1 - 3 pi / 2,
    y_j = 2 pi x_j - pi (j >= 2) and a = pi sqrt(gamma) / 2, the tent whose
    normalising factor (3 / (pi sqrt(gamma)))^(d/2) makes it unit-norm on
    [0, 2 pi]^d; scaled to unit lattice-rule norm unless normalize is False.
    The tent is supported inside the cell for gamma <= 1, so it is periodic,
    continuous and only Lipschitz (kinks at its peak and edges)."""
    x = num.astype(np.float64) / N
    a = 0.5 * np.pi * np.sqrt(gamma)
    u = np.maximum(0.0, 1.0 - np.abs(2 * np.pi * x[:, 0] - 1.5 * np.pi) / a)
    for j in range(1, num.shape[1]):
        u = u * np.maximum(0.0, 1.0 - np.abs(2 * np.pi * x[:, j] - np.pi) / a)
    u = u.astype(np.complex128)
    if normalize:
        u /= np.sqrt(np.mean(np.abs(u) ** 2))
    return u


def paper_g1_coefficients(d: int, gamma: float, kmax: int, nodes: int = 4096):
    """Fourier coefficients of the (unscaled) g1 on [0,1)^d: g1 is a product of
    1-D factors exp(-(2 pi x - c)^2 / gamma) (c = 3 pi / 2 in the first
    coordinate, pi in the others), so ghat(h) = prod_j I_j(h_j) with
    I_j(k) = int_0^1 exp(-(2 pi x - c_j)^2 / gamma) exp(-2 pi i k x) dx.
    Returns (tables (d, 2 kmax + 1) complex, I_j(k) at column k + kmax; the
    squared L2 norm of g1), both from a Gauss-Legendre rule with `nodes`
    points on [0, 1] (exact to rounding for |k| well below nodes / 2)."""
    t, w = np.polynomial.legendre.leggauss(nodes)
    x, w = 0.5 * (t + 1.0), 0.5 * w
    k = np.arange(-kmax, kmax + 1)
    tables = np.empty((d, 2 * kmax + 1), dtype=np.complex128)
    norm2 = 1.0
    for j in range(d):
        c = 1.5 * np.pi if j == 0 else np.pi
        f = np.exp(-(2 * np.pi * x - c) ** 2 / gamma)
        tables[j] = np.exp(-2j * np.pi * np.outer(k, x)) @ (w * f)
        norm2 *= float(np.sum(w * f * f))
    return tables, norm2


def coefficients_at(h: np.ndarray, tables: np.ndarray) -> np.ndarray:
    """prod_j tables[j, h_j + kmax] for integer vectors h (rows), the Fourier
    coefficient of a product function at frequencies h."""
    kmax = (tables.shape[1] - 1) // 2
    out = np.ones(h.shape[0], dtype=np.complex128)
    for j in range(h.shape[1]):
        out *= tables[j, h[:, j] + kmax]
    return out


# ---------------------------------------------------------------- configurations
@dataclass
class Instance:
    """One Strang problem: lattice, index set, v and u0 at the points."""
    d: int
    Z: np.ndarray                   # (r, d) int64
    n: np.ndarray                   # (r,) int64
    I: Optional[np.ndarray]         # user index set (nI, d) int32, or None = minimal-l2 set
    gamma: float
    dt: float
    steps: int
    v: np.ndarray                   # (N,) float64
    u0: np.ndarray                  # (N,) or (B, N) complex128
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    @property
    def r(self) -> int:
        return int(self.n.size)


def box_d2_n1031() -> Instance:
    """d = 2, N = 1031, z = (1, 32), I = {-15..16}^2, gamma = 0.1,
    v = sum_j (1 - cos 2 pi x_j), Gaussian packet at (1/2, 1/2) with k0 = (2, 0)
    projected onto I, dt = 0.01, 100 steps."""
    Z = np.array([[1, 32]], dtype=np.int64)
    n = np.array([1031], dtype=np.int64)
    num = point_numerators(Z, n)
    I = box(-15, 16, 2)
    v = v_sum_one_minus_cos(num, 1031)
    u0 = projected_packet(Z, n, I, (0.5, 0.5), (2, 0), 0.1)
    return Instance(2, Z, n, I, 0.1, 0.01, 100, v, u0, {"name": "box_d2_n1031"})


def cross_d6_n1048573(steps: int = 1000) -> Instance:
    """d = 6, N = 1048573 (prime), z by seeded reconstructing CBC on the
    hyperbolic cross R = 10 (70,173 frequencies), gamma = 0.05,
    v = prod_j (1 + cos(2 pi x_j)/2) - 1, seeded packet, dt = 1e-3."""
    N = 1048573
    H = hyperbolic_cross(6, 10)
    z = cbc_rank1(H, N, rng(1, "z"))
    Z = z.reshape(1, -1)
    n = np.array([N], dtype=np.int64)
    num = point_numerators(Z, n)
    v = v_product(num, N)
    u0 = seeded_packet(num, N, rng(1, "u0"))
    return Instance(6, Z, n, H, 0.05, 1e-3, steps, v, u0, {"name": "cross_d6_n1048573", "R": 10})


def smooth7(x: int) -> int:
    """Smallest 7-smooth integer >= x."""
    best = None
    p2 = 1
    while p2 < 2 * x:
        p3 = p2
        while p3 < 2 * x:
            p5 = p3
            while p5 < 2 * x:
                p7 = p5
                while p7 < 2 * x:
                    if p7 >= x and (best is None or p7 < best):
                        best = p7
                    p7 *= 7
                p5 *= 5
            p3 *= 3
        p2 *= 2
    return best


def next_prime(x: int) -> int:
    def isprime(m):
        if m < 2:
            return False
        if m % 2 == 0:
            return m == 2
        f = 3
        while f * f <= m:
            if m % f == 0:
                return False
            f += 2
        return True
    while not isprime(x):
        x += 1
    return x


def mixed_batch_shapes(count: int = 256):
    """(d_i, N_i) for the batched configuration: d ~ U{2..10}, N log-uniform in
    [2^12, 2^18], primes at even i and 7-smooth composites at odd i."""
    g = rng(2, "shapes")
    out = []
    for i in range(count):
        d = int(g.integers(2, 11))
        target = int(round(2.0 ** g.uniform(12.0, 18.0)))
        N = next_prime(target) if i % 2 == 0 else smooth7(target)
        out.append((d, N))
    return out


def mixed_batch(count: int = 256, steps: int = 200, shapes=None) -> List[Instance]:
    """Batched complex64: per instance the best of 8 seeded Korobov vectors
    (korobov_good), minimal-l2 full index set,
    16-term cosine potential (|h_j| <= 2, a ~ U(-1/2, 1/2)), gamma ~ U(0.02, 0.2),
    seeded packet, dt = 5e-3, 200 steps."""
    shapes = shapes if shapes is not None else mixed_batch_shapes(count)
    gz, gv, gu, gs = rng(2, "z"), rng(2, "v"), rng(2, "u0"), rng(2, "hidden_v")
    out = []
    for i, (d, N) in enumerate(shapes):
        z = korobov_good(N, d, gz)
        Z = z.reshape(1, -1)
        n = np.array([N], dtype=np.int64)
        num = point_numerators(Z, n)
        v = cosine_series(d, 16, gv).at(num, N)
        u0 = seeded_packet(num, N, gu)
        gamma = float(gs.uniform(0.02, 0.2))
        out.append(Instance(d, Z, n, None, gamma, 5e-3, steps, v, u0, {"name": f"mixed_batch[{i}]"}))
    return out


def rank2_d10_n4096x256(steps: int = 500) -> Instance:
    """d = 10, rank-2 lattice n = (4096, 256), odd generating vectors by seeded
    rank-2 CBC on the cross {-1,0,1}^10 (59,049 frequencies), completed to
    2^20 keys; gamma = 0.05, 32-term cosine potential, seeded packet, dt = 2e-3."""
    H = hyperbolic_cross(10, 1)
    Z = cbc_rank2(H, 4096, 256, rng(3, "z"))
    n = np.array([4096, 256], dtype=np.int64)
    num = point_numerators(Z, n)
    N = 4096 * 256
    v = cosine_series(10, 32, rng(3, "v")).at(num, N)
    u0 = seeded_packet(num, N, rng(3, "u0"))
    return Instance(10, Z, n, H, 0.05, 2e-3, steps, v, u0, {"name": "rank2_d10_n4096x256", "R": 1})


# Generating vectors the paper prints for its experiments (Sec. 3.1, Table 1):
# (d, n) -> z.  For d >= 4 the paper takes the first d components of the
# 12-component vector at n = 2^25.
_TABLE1_Z12 = (1, 12386359, 15699201, 6807287, 13966305, 6107923, 4432603, 2304135, 7323801, 5705679,
               5643703, 3867405)
PAPER_TABLE1 = {(2, 1 << 18): (1, 100135), (2, 1 << 20): (1, 443165), (3, 1 << 22): (1, 1737355, 261247),
                (3, 1 << 25): (1, 12386359, 15699201)}
PAPER_TABLE1.update({(d, 1 << 25): _TABLE1_Z12[:d] for d in range(4, 13)})


def paper_lattice(d: int, n: int):
    """(Z, n) of a Table 1 lattice as rank-1 arrays."""
    z = np.asarray(PAPER_TABLE1[(d, n)], dtype=np.int64)
    return z.reshape(1, -1), np.array([n], dtype=np.int64)


def adjoint_d4_n65521(batch: int = 32, steps: int = 500):
    """d = 4, N = 65521 (prime), Korobov z, minimal-l2 full set, batch of
    seeded packets sharing a 64-term cosine potential; a hidden 64-term
    potential defines the target.  gamma = 0.05, dt = 2e-3, checkpoints every 50."""
    N, d = 65521, 4
    z = korobov(N, d, rng(4, "z"))
    Z = z.reshape(1, -1)
    n = np.array([N], dtype=np.int64)
    num = point_numerators(Z, n)
    series = cosine_series(d, 64, rng(4, "v"))
    hidden = cosine_series(d, 64, rng(4, "hidden_v"))
    gu = rng(4, "u0")
    u0 = np.stack([seeded_packet(num, N, gu) for _ in range(batch)])
    inst = Instance(d, Z, n, None, 0.05, 2e-3, steps, series.at(num, N), u0,
                    {"name": "adjoint_d4_n65521", "ckpt_every": 50, "series": series, "hidden": hidden,
                     "v_hidden": hidden.at(num, N), "num": num})
    return inst


def maxsize_d3(N: int, seed: int = 41) -> Instance:
    """The largest single lattices of the build: d = 3 rank-1 with N near 2^22
    (prime 4194301, whose chirp-z length is 2^23, or 2^22 itself), best-of-8
    Korobov z, 16-term cosine potential, seeded packet, gamma = 0.05,
    dt = 2e-3, 8 steps."""
    g = np.random.default_rng(seed)
    d = 3
    z = korobov_good(N, d, g)
    Z, n = z.reshape(1, -1), np.array([N], dtype=np.int64)
    num = point_numerators(Z, n)
    v = cosine_series(d, 16, g).at(num, N)
    u0 = seeded_packet(num, N, g)
    return Instance(d, Z, n, None, 0.05, 2e-3, 8, v, u0, {"name": f"maxsize_d3_n{N}"})


def conservation_d5_n2p20(steps: int = 1000) -> Instance:
    """The conservation setting of Sec. 3.3: gamma = 0.5, d = 5, the paper's g1
    and harmonic v2, on a rank-1 lattice of 2^20 points (best of 8 Korobov
    vectors, seed 33; Table 1 lists no d = 5 vector), dt = 1e-3, checkpoints
    every 10 steps."""
    N, d = 1 << 20, 5
    z = korobov_good(N, d, np.random.default_rng(33))
    Z, n = z.reshape(1, -1), np.array([N], dtype=np.int64)
    num = point_numerators(Z, n)
    return Instance(d, Z, n, None, 0.5, 1e-3, steps, v_harmonic_paper(num, N), paper_g1(num, N, 0.5),
                    {"name": "conservation_d5_n2p20", "ckpt_every": 10})


def table1_run(d: int, n: int, potential: str = "v1", gamma: float = 0.5, dt: float = 1e-3,
               steps: int = 100, initial: str = "g1") -> Instance:
    """A Table 1 lattice (Sec. 3.1) with its minimal-l2 index set, the paper's
    g1 (Gaussian) or g2 (hat) and v1 (smooth) or v2 (harmonic) (Sec. 3.2)."""
    Z, nn = paper_lattice(d, n)
    num = point_numerators(Z, nn)
    vfun = v_smooth_paper if potential == "v1" else v_harmonic_paper
    gfun = paper_g1 if initial == "g1" else paper_g2
    return Instance(d, Z, nn, None, gamma, dt, steps, vfun(num, n), gfun(num, n, gamma),
                    {"name": f"table1_d{d}_n{n}_{initial}_{potential}"})


def splitting_modulation(t):
    """f(t) of the time-dependent potential v(x, t) = v(x) + f(t) v(x) on the
    benchmark lattice: 0.5 sin(20 t)."""
    return 0.5 * np.sin(20.0 * np.asarray(t, dtype=np.float64))
