"""FP64 CPU oracle for Strang splitting on rank-1 / rank-r lattices.

TEST INFRASTRUCTURE ONLY.  The product package never imports this module;
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` do.  The arithmetic lives in ``oracle.c`` (plain C, double
precision); this file only marshals numpy arrays through ctypes.

Paper references (arXiv:1808.06357):
  * keys / anti-aliasing sets: Sec. 2.1, Def. 2; Thm. 1(iii);
  * minimal-l2 representatives: Lemma 4, eq. (hrepresenter);
  * unitary DFT: Sec. 2.2, eqs. (Fnx), (Fn);
  * Strang step: Sec. 2.4, eq. (StrangTDSE); Algorithm 1;
  * rank-r orderings: Sec. 2.5;
  * norm / energy: Sec. 3.3;
  * initial discretization error: Sec. 3.4;
  * fourth-order composition of Strang steps and time-dependent potentials:
    the two continuations named in Sec. 5 (the composition taken as Yoshida's
    symmetric triple jump, time advanced with the kinetic flow).

Every function here is pinned by ``tests/test_oracle.py`` against values the
paper and the mathematics fix (closed forms, brute force, library routines).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "liboracle.so")
_lock = threading.Lock()
_lib = None

STATUS = {0: "ok", 1: "argument error", 2: "index set not injective",
          3: "keys unreachable (lattice points not distinct)", 4: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (ISO C11, so no FP contraction)."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
            sig = {
                "or_key": (i64, [ctypes.c_int, ctypes.c_int, P, P, P]),
                "or_keys": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, P, P, P, i64, P]),
                "or_points": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, P, P, P]),
                "or_index_set": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, P, P, P, i64, P, P, P]),
                "or_dft_direct": (ctypes.c_int, [i64, P, P, ctypes.c_int]),
                "or_fft_radix2": (ctypes.c_int, [i64, P, ctypes.c_int]),
                "or_fft_bluestein": (ctypes.c_int, [i64, P, ctypes.c_int]),
                "or_fft": (ctypes.c_int, [i64, P, ctypes.c_int, ctypes.c_int]),
                "or_fftn": (ctypes.c_int, [ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int]),
                "or_diagnostics": (ctypes.c_int, [ctypes.c_int, P, P, P, P, f64, ctypes.c_int, P, P]),
                "or_strang_run": (ctypes.c_int, [ctypes.c_int, P, P, i64, P, i64, P, f64, f64, i64,
                                                 ctypes.c_int, P]),
                "or_strang_vjp": (ctypes.c_int, [ctypes.c_int, P, P, i64, P, i64, P, P, f64, f64, i64,
                                                 ctypes.c_int, P, P, P]),
            }
            for name, (res, args) in sig.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(code: int, what: str):
    if code != 0:
        raise OracleError(code, what)


def _lattice(Z, n):
    Z = np.ascontiguousarray(np.atleast_2d(np.asarray(Z, dtype=np.int64)))
    n = np.ascontiguousarray(np.atleast_1d(np.asarray(n, dtype=np.int64)))
    if Z.shape[0] != n.shape[0]:
        raise ValueError("Z must have one row per generating vector (r x d)")
    return Z, n


_METHODS = {"auto": 0, "direct": 1, "radix2": 2, "bluestein": 3}


# ---------------------------------------------------------------- lattice
def keys(Z, n, H) -> np.ndarray:
    """chi(h) for each row of H (Def. 2, Thm. 1(iii), Sec. 2.5 ordering)."""
    Z, n = _lattice(Z, n)
    H = np.ascontiguousarray(np.atleast_2d(np.asarray(H, dtype=np.int32)))
    out = np.empty(H.shape[0], dtype=np.int64)
    _check(_load().or_keys(Z.shape[1], Z.shape[0], _p(Z), _p(n), _p(H), H.shape[0], _p(out)), "keys")
    return out


def points(Z, n) -> np.ndarray:
    """Lattice points p_kappa (N x d) in kappa order (Def. 1, Sec. 2.5)."""
    Z, n = _lattice(Z, n)
    N = int(np.prod(n))
    x = np.empty((N, Z.shape[1]), dtype=np.float64)
    _check(_load().or_points(Z.shape[1], Z.shape[0], _p(Z), _p(n), _p(x)), "points")
    return x


def index_set(Z, n, I=None):
    """Full anti-aliasing set: I owns its keys, the rest get minimal-l2
    representatives (Lemma 4).  Returns (h_of_key (N x d), s_of_key (N),
    from_I (N bool))."""
    Z, n = _lattice(Z, n)
    d, r = Z.shape[1], Z.shape[0]
    N = int(np.prod(n))
    if I is None:
        I = np.zeros((0, d), dtype=np.int32)
    I = np.ascontiguousarray(np.asarray(I, dtype=np.int32).reshape(-1, d))
    h = np.zeros((N, d), dtype=np.int32)
    s = np.zeros(N, dtype=np.int64)
    fromI = np.zeros(N, dtype=np.uint8)
    _check(_load().or_index_set(d, r, _p(Z), _p(n), _p(I), I.shape[0], _p(h), _p(s), _p(fromI)),
           "index_set")
    return h, s, fromI.astype(bool)


# ---------------------------------------------------------------- transforms
def dft_direct(x, sign=-1) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.complex128)
    X = np.empty_like(x)
    _check(_load().or_dft_direct(x.size, _p(x), _p(X), sign), "dft_direct")
    return X


def fft(x, sign=-1, method="auto") -> np.ndarray:
    """Unnormalised 1-D DFT, kernel exp(sign 2 pi i k xi / L)."""
    y = np.array(x, dtype=np.complex128, copy=True, order="C")
    _check(_load().or_fft(y.size, _p(y), sign, _METHODS[method]), "fft")
    return y


def fftn(x, n, sign=-1, method="auto") -> np.ndarray:
    """Unnormalised r-D DFT of the row-major tensor with shape n (flat in/out)."""
    n = np.ascontiguousarray(np.atleast_1d(np.asarray(n, dtype=np.int64)))
    y = np.array(x, dtype=np.complex128, copy=True, order="C").reshape(-1)
    _check(_load().or_fftn(n.size, _p(n), _p(y), sign, _METHODS[method]), "fftn")
    return y


# ---------------------------------------------------------------- Strang
def strang_run(n, s_of_key, v, u0, gamma, dt, steps, method="auto", history=False):
    """m Strang steps on lattice values (eq. (StrangTDSE), Algorithm 1).

    n: moduli (rank r); s_of_key: ||h_chi||^2 per key; v: (N,) shared or
    (batch, N); u0: (N,) or (batch, N) complex.  Returns u(T) with the shape
    of u0, and optionally the (batch, steps+1, 3) history of norm^2, energy
    and the energy's potential term (1/(gamma N)) sum v |u|^2 (Sec. 3.3)."""
    n = np.ascontiguousarray(np.atleast_1d(np.asarray(n, dtype=np.int64)))
    N = int(np.prod(n))
    s = np.ascontiguousarray(s_of_key, dtype=np.int64)
    u = np.array(u0, dtype=np.complex128, copy=True, order="C")
    shape = u.shape
    u = u.reshape(-1, N)
    batch = u.shape[0]
    v = np.ascontiguousarray(v, dtype=np.float64)
    v_stride = 0 if v.ndim == 1 else N
    if v.ndim != 1 and v.shape[0] != batch:
        raise ValueError("v must be (N,) or (batch, N)")
    hist = np.zeros((batch, steps + 1, 3)) if history else None
    _check(_load().or_strang_run(n.size, _p(n), _p(s), batch, _p(v), v_stride, _p(u), float(gamma),
                                 float(dt), int(steps), _METHODS[method],
                                 _p(hist) if history else None), "strang_run")
    u = u.reshape(shape)
    return (u, hist) if history else u


def strang_vjp(n, s_of_key, v, u0, gT, gamma, dt, steps, method="auto", return_abs=False):
    """Reverse-mode derivative of u(T) = S^m u0: returns (g0, gv) given the
    cotangent gT = dJ/dRe u(T) + i dJ/dIm u(T).  gv is summed over the batch
    when v is shared.  return_abs: also return gv_abs, the same sums of the
    terms' absolute values (gv_abs / |gv| is the conditioning of each sum)."""
    n = np.ascontiguousarray(np.atleast_1d(np.asarray(n, dtype=np.int64)))
    N = int(np.prod(n))
    s = np.ascontiguousarray(s_of_key, dtype=np.int64)
    u0 = np.ascontiguousarray(u0, dtype=np.complex128)
    gT = np.ascontiguousarray(gT, dtype=np.complex128)
    shape = u0.shape
    u0 = u0.reshape(-1, N)
    gT = gT.reshape(-1, N)
    batch = u0.shape[0]
    v = np.ascontiguousarray(v, dtype=np.float64)
    v_stride = 0 if v.ndim == 1 else N
    g0 = np.empty_like(u0)
    gv = np.zeros((1 if v_stride == 0 else batch, N))
    ga = np.zeros_like(gv) if return_abs else None
    _check(_load().or_strang_vjp(n.size, _p(n), _p(s), batch, _p(v), v_stride, _p(u0), _p(gT),
                                 float(gamma), float(dt), int(steps), _METHODS[method], _p(g0),
                                 _p(gv), _p(ga) if return_abs else None), "strang_vjp")
    out = (g0.reshape(shape), (gv[0] if v_stride == 0 else gv))
    if return_abs:
        out = out + ((ga[0] if v_stride == 0 else ga),)
    return out


def composition_weights(order):
    """Step fractions of a symmetric composition of Strang steps: (1,) for
    order 2; for order 4 the triple jump w1, w0, w1 with w1 = 1/(2 - 2^(1/3))
    and w0 = 1 - 2 w1, so that the weights sum to 1 and their cubes to 0."""
    if order == 2:
        return (1.0,)
    if order != 4:
        raise ValueError("order must be 2 or 4")
    w1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
    return (w1, 1.0 - 2.0 * w1, w1)


def composed_run(n, s_of_key, v, u0, gamma, dt, steps, order=4, v1=None, f=None, t0=0.0, method="auto"):
    """`steps` steps of the composition: each step runs one Strang step of
    length w dt per weight w, in order (no merging of the potential halves).

    Time-dependent potential v(x, t) = v(x) + f(t) v1(x) (v1 shaped as v, f a
    function of t): time advances with the kinetic part, so a substep of
    length h starting at tau applies exp(-i h v(., tau) / (2 gamma)), the
    kinetic flow of length h (a Strang step with zero potential), then
    exp(-i h v(., tau + h) / (2 gamma)); tau runs through t0 + (k + partial
    sums of the weights) dt."""
    u = np.array(u0, dtype=np.complex128, copy=True)
    if v1 is None:
        for _ in range(steps):
            for w in composition_weights(order):
                u = strang_run(n, s_of_key, v, u, gamma, w * dt, 1, method=method)
        return u
    v = np.asarray(v, dtype=np.float64)
    v1 = np.asarray(v1, dtype=np.float64)
    zero = np.zeros(v.shape[-1])
    for k in range(steps):
        tau = t0 + k * dt
        for w in composition_weights(order):
            h = w * dt
            u = np.exp(-1j * h * (v + f(tau) * v1) / (2.0 * gamma)) * u
            u = strang_run(n, s_of_key, zero, u, gamma, h, 1, method=method)
            tau += h
            u = np.exp(-1j * h * (v + f(tau) * v1) / (2.0 * gamma)) * u
    return u


def projection_error(n, u, ghat, method="auto"):
    """The two key sums of the initial discretization error (Sec. 3.4):
    (sum_A |ghat|^2, sum_A |ghat - ghat_a|^2) with ghat_a(h_xi) = (1/N) times
    the lattice DFT of the point values u at key xi (eq. (Fn) / (Fnx) without
    the 1/sqrt(N)), for u and ghat of shape (N,) or (batch, N) in key order.
    e_total^2 = ||g||^2 - first + second."""
    n = np.ascontiguousarray(np.atleast_1d(np.asarray(n, dtype=np.int64)))
    N = int(np.prod(n))
    u = np.asarray(u, dtype=np.complex128).reshape(-1, N)
    g = np.asarray(ghat, dtype=np.complex128).reshape(-1, N)
    out = np.empty((u.shape[0], 2))
    for b in range(u.shape[0]):
        ga = fftn(u[b], n, -1, method) / N
        out[b] = (np.sum(np.abs(g[b]) ** 2), np.sum(np.abs(g[b] - ga) ** 2))
    return out


def diagnostics(n, s_of_key, v, u, gamma, method="auto"):
    """(norm^2, energy) of lattice values u (Sec. 3.3)."""
    n = np.ascontiguousarray(np.atleast_1d(np.asarray(n, dtype=np.int64)))
    s = np.ascontiguousarray(s_of_key, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.complex128)
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(_load().or_diagnostics(n.size, _p(n), _p(s), _p(v), _p(u), float(gamma),
                                  _METHODS[method], ctypes.byref(a), ctypes.byref(b), None), "diagnostics")
    return a.value, b.value
