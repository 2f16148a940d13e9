"""ctypes binding of include/lattice_tdse.h (argument marshalling only).

Every function here has the name of the C entry point it calls.  Device
buffers are torch tensors on the current HIP device; the library does all of
the work.  If the compiled library is missing this module raises ImportError:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblattice_tdse.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "lattice_tdse.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(python -c 'import __graft_entry__ as g; g.build()')")

# PyTorch ships its own HIP runtime under the same soname as the system one.
# Loading torch first lets the library bind to that runtime, so the process
# holds one HIP/HSA runtime; loaded the other way round, torch maps a second
# copy and the runtime that initialises second finds no device.
try:
    import torch  # noqa: F401
except ImportError:
    pass

lib = ctypes.CDLL(LIB_PATH)

LT_C64, LT_C128 = 1, 2
STATUS = {0: "LT_OK", 1: "LT_E_ARG", 2: "LT_E_NOT_CANONICAL", 3: "LT_E_NOT_INJECTIVE",
          4: "LT_E_INCOMPLETE", 5: "LT_E_NOMEM", 6: "LT_E_HIP", 7: "LT_E_UNSUPPORTED"}


class LatticeError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib.lt_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class PlanInfo(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("r", ctypes.c_int32), ("n", ctypes.c_int64 * 4),
                ("N", ctypes.c_int64), ("n_index", ctypes.c_int64), ("n_completed", ctypes.c_int64),
                ("max_s", ctypes.c_int64), ("bluestein", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("fft_len", ctypes.c_int64), ("L1", ctypes.c_int32), ("L2", ctypes.c_int32),
                ("cols", ctypes.c_int32), ("rows", ctypes.c_int32), ("L3", ctypes.c_int32),
                ("swapped", ctypes.c_int32)]


_P, _i32, _i64, _f64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_SIGS = {
    "lattice_plan": [_i32, _i32, _P, _P, _P, _i64, _i32, _i32, ctypes.POINTER(_P)],
    "lattice_plan_info": [_P, ctypes.POINTER(PlanInfo)],
    "lattice_plan_keys": [_P, _P, _P, _P],
    "lattice_plan_points": [_P, _i64, _i64, _P],
    "lattice_plan_destroy": [_P],
    "strang_workspace_size": [_P, _i32, _i32, _i32, ctypes.POINTER(_sz)],
    "strang_run": [_P, _i32, _i32, _P, _i64, _P, _f64, _f64, _i64, _P, _i64, _P, _sz, _P],
    "strang_run_sums_workspace_size": [_P, _i32, _i32, _i32, _i64, ctypes.POINTER(_sz)],
    "strang_run_noalloc_capacity": [ctypes.POINTER(_sz)],
    "strang_run_noalloc": [_P, _i32, _i32, _P, _i64, _P, _f64, _f64, _i64, _P],
    "strang_run_sums": [_P, _i32, _i32, _P, _i64, _P, _f64, _f64, _i64, _P, _i64, _P, _P, _sz, _P],
    "strang_adjoint_workspace_size": [_P, _i32, _i32, _i32, ctypes.POINTER(_sz)],
    "strang_adjoint": [_P, _i32, _i32, _P, _i64, _P, _P, _f64, _f64, _i64, _P, _i64, _P, _P, _P, _sz, _P],
    "strang_batched_workspace_size": [_i32, _P, _i32, ctypes.POINTER(_sz)],
    "strang_batch_create": [_i32, _P, _i32, _P, _P, _P, _P, _P, _P, ctypes.POINTER(_P)],
    "strang_batch_run": [_P, _P],
    "strang_batch_autotune": [_P, _i32, _P],
    "strang_batch_kernels": [_P, ctypes.POINTER(_i32), _P, _P, _i32],
    "strang_batch_destroy": [_P],
    "strang_run_batched": [_i32, _P, _i32, _P, _P, _P, _P, _P, _P, _sz, _P],
    "lattice_projection_error_workspace_size": [_P, _i32, _i32, ctypes.POINTER(_sz)],
    "lattice_projection_error": [_P, _i32, _i32, _P, _P, _P, _P, _sz, _P],
    "splitting_workspace_size": [_P, _i32, _i32, _i32, _i32, ctypes.POINTER(_sz)],
    "splitting_run": [_P, _i32, _i32, _P, _P, _i64, _P, _P, _f64, _f64, _i64, _i32, _P, _sz, _P],
    "splitting_times": [_i32, _i64, _f64, _f64, _P],
    "lattice_diagnostics_workspace_size": [_P, _i32, _i32, ctypes.POINTER(_sz)],
    "lattice_diagnostics": [_P, _i32, _i32, _P, _i64, _P, _f64, _P, _P, _sz, _P],
    "lattice_plan_autotune": [_P, _i32, _i32, _P],
    "lattice_plan_set_kernels": [_P, _i32, _i32, _i32],
    "lattice_plan_get_kernels": [_P, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "lattice_plan_get_kernels_batch": [_P, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "lt_timing_enable": [_i32],
    "lt_timing_summary": [_i32, ctypes.POINTER(_i64), ctypes.POINTER(_f64)],
    "lt_last_error": [],
}
for _name, _args in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.argtypes = _args
    _fn.restype = (ctypes.c_char_p if _name == "lt_last_error"
                   else None if _name in ("lattice_plan_destroy", "strang_batch_destroy") else ctypes.c_int)


def header_functions() -> list:
    """Names of the functions include/lattice_tdse.h declares."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(\w+)\s*\(", txt)) - {"if", "sizeof"})


def _check(code: int, where: str):
    if code != 0:
        raise LatticeError(code, where)


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_P)


# ---------------------------------------------------------------- plans
class Plan:
    """Owner of an lt_plan*; the C plan is destroyed with this object."""

    def __init__(self, handle: int, d: int, r: int):
        self._h = _P(handle)
        self.d, self.r = d, r
        self.info = lattice_plan_info(self)
        self.N = int(self.info["N"])

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        try:
            if h is not None and h.value:
                lib.lattice_plan_destroy(h)
                self._h = _P(0)
        except Exception:  # interpreter shutdown: module globals may already be torn down
            pass


def lattice_plan(Z, n, H=None, complete: bool = True, prec_mask: int = 0) -> Plan:
    """Plan a rank-r lattice (Z: r x d generating vectors, n: r moduli) with
    optional index set H (nh x d); complete: give keys H leaves unowned their
    minimal-l2 representatives; prec_mask: LT_C64 | LT_C128 precisions whose
    device tables are built now; see lattice_plan in lattice_tdse.h."""
    Z = np.ascontiguousarray(np.atleast_2d(np.asarray(Z, dtype=np.int64)))
    n = np.ascontiguousarray(np.atleast_1d(np.asarray(n, dtype=np.int64)))
    r, d = Z.shape
    if H is not None:
        H = np.ascontiguousarray(np.asarray(H, dtype=np.int32).reshape(-1, d))
    out = _P()
    _check(lib.lattice_plan(d, r, _np_ptr(Z), _np_ptr(n), _np_ptr(H), 0 if H is None else H.shape[0],
                            1 if complete else 0, int(prec_mask), ctypes.byref(out)), "lattice_plan")
    return Plan(out.value, d, r)


def lattice_plan_info(plan: Plan) -> dict:
    info = PlanInfo()
    _check(lib.lattice_plan_info(plan.handle, ctypes.byref(info)), "lattice_plan_info")
    out = {k: getattr(info, k) for k, _ in PlanInfo._fields_}
    out["n"] = list(info.n)[: info.r]
    return out


def lattice_plan_keys(plan: Plan):
    """(key_of_h, s_of_key, h_of_key) as numpy arrays (host copies)."""
    nh = int(plan.info["n_index"])
    k = np.empty(nh, dtype=np.int64)
    s = np.empty(plan.N, dtype=np.int64)
    h = np.empty((plan.N, plan.d), dtype=np.int32)
    _check(lib.lattice_plan_keys(plan.handle, _np_ptr(k), _np_ptr(s), _np_ptr(h)), "lattice_plan_keys")
    return k, s, h


def lattice_plan_points(plan: Plan, first: int = 0, count: Optional[int] = None) -> np.ndarray:
    """Integer numerators of the lattice points (p = num / N)."""
    count = plan.N - first if count is None else count
    num = np.empty((count, plan.d), dtype=np.int64)
    _check(lib.lattice_plan_points(plan.handle, first, count, _np_ptr(num)), "lattice_plan_points")
    return num


# ---------------------------------------------------------------- runs
def _prec_of(t) -> int:
    import torch
    if t.dtype == torch.complex64:
        return LT_C64
    if t.dtype == torch.complex128:
        return LT_C128
    raise TypeError("state must be torch.complex64 or torch.complex128")


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return _P(stream.cuda_stream)


def _dev_ptr(t):
    return None if t is None else _P(t.data_ptr())


def _check_dev(t, name, dtype=None, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")


def strang_workspace_size(plan: Plan, prec: int, batch: int, shared_v: bool) -> int:
    n = _sz()
    _check(lib.strang_workspace_size(plan.handle, prec, batch, int(bool(shared_v)), ctypes.byref(n)),
           "strang_workspace_size")
    return n.value


def strang_adjoint_workspace_size(plan: Plan, prec: int, batch: int, shared_v: bool) -> int:
    n = _sz()
    _check(lib.strang_adjoint_workspace_size(plan.handle, prec, batch, int(bool(shared_v)),
                                             ctypes.byref(n)), "strang_adjoint_workspace_size")
    return n.value


def num_checkpoints(steps: int, every: int) -> int:
    return 0 if every <= 0 else (steps + every - 1) // every


def strang_run(plan: Plan, v, u, gamma: float, dt: float, steps: int, ckpt=None, ckpt_every: int = 0,
               work=None, stream=None):
    """In-place Strang run of u (device, (N,) or (batch, N), complex64/128)
    under v (device float64, (N,) shared or (batch, N))."""
    import torch
    N = plan.N
    prec = _prec_of(u)
    batch = u.numel() // N
    _check_dev(u, "u", numel=batch * N)
    _check_dev(v, "v", torch.float64)
    if v.numel() not in (N, batch * N):
        raise ValueError("v must hold N or batch*N values")
    v_stride = 0 if v.numel() == N else N
    if ckpt is not None:
        _check_dev(ckpt, "ckpt", u.dtype, num_checkpoints(steps, ckpt_every) * batch * N)
    wb = 0
    if work is not None:
        _check_dev(work, "work")
        wb = work.numel() * work.element_size()
    _check(lib.strang_run(plan.handle, prec, batch, _dev_ptr(v), v_stride, _dev_ptr(u), float(gamma),
                          float(dt), int(steps), _dev_ptr(ckpt), int(ckpt_every), _dev_ptr(work), wb,
                          _stream(stream)), "strang_run")
    return u


def strang_run_noalloc_capacity() -> int:
    n = _sz()
    _check(lib.strang_run_noalloc_capacity(ctypes.byref(n)), "strang_run_noalloc_capacity")
    return n.value


def strang_run_noalloc(plan: Plan, v, u, gamma: float, dt: float, steps: int, stream=None):
    """strang_run on the library's static per-GPU scratch: allocates nothing
    (the plan's tables must exist: prec_mask at planning, or an earlier run)."""
    import torch
    N = plan.N
    prec = _prec_of(u)
    batch = u.numel() // N
    _check_dev(u, "u", numel=batch * N)
    _check_dev(v, "v", torch.float64)
    if v.numel() not in (N, batch * N):
        raise ValueError("v must hold N or batch*N values")
    v_stride = 0 if v.numel() == N else N
    _check(lib.strang_run_noalloc(plan.handle, prec, batch, _dev_ptr(v), v_stride, _dev_ptr(u), float(gamma),
                                  float(dt), int(steps), _stream(stream)), "strang_run_noalloc")
    return u


def strang_run_sums_workspace_size(plan: Plan, prec: int, batch: int, shared_v: bool, steps: int) -> int:
    n = _sz()
    _check(lib.strang_run_sums_workspace_size(plan.handle, prec, batch, int(bool(shared_v)), int(steps),
                                              ctypes.byref(n)), "strang_run_sums_workspace_size")
    return n.value


def strang_run_sums(plan: Plan, v, u, gamma: float, dt: float, steps: int, sums=None, ckpt=None,
                    ckpt_every: int = 0, work=None, stream=None):
    """strang_run that also returns the per-step sums (device float64,
    (batch, steps + 1, 2)): (1/N) sum |u_j|^2 and (1/(gamma N)) sum v |u_j|^2
    at every step boundary j."""
    import torch
    N = plan.N
    prec = _prec_of(u)
    batch = u.numel() // N
    _check_dev(u, "u", numel=batch * N)
    _check_dev(v, "v", torch.float64)
    if v.numel() not in (N, batch * N):
        raise ValueError("v must hold N or batch*N values")
    v_stride = 0 if v.numel() == N else N
    if ckpt is not None:
        _check_dev(ckpt, "ckpt", u.dtype, num_checkpoints(steps, ckpt_every) * batch * N)
    if sums is None:
        sums = torch.empty((batch, steps + 1, 2), dtype=torch.float64, device=u.device)
    _check_dev(sums, "sums", torch.float64, batch * (steps + 1) * 2)
    wb = 0
    if work is not None:
        _check_dev(work, "work")
        wb = work.numel() * work.element_size()
    _check(lib.strang_run_sums(plan.handle, prec, batch, _dev_ptr(v), v_stride, _dev_ptr(u), float(gamma),
                               float(dt), int(steps), _dev_ptr(ckpt), int(ckpt_every), _dev_ptr(sums),
                               _dev_ptr(work), wb, _stream(stream)), "strang_run_sums")
    return sums


def strang_adjoint(plan: Plan, v, uT, gT, gamma: float, dt: float, steps: int, ckpt, ckpt_every: int,
                   g0=None, gv=None, work=None, stream=None):
    """Returns (g0, gv): dJ/du(0) and dJ/dv for the cotangent gT of u(T)."""
    import torch
    N = plan.N
    prec = _prec_of(uT)
    batch = uT.numel() // N
    _check_dev(uT, "uT", numel=batch * N)
    _check_dev(gT, "gT", uT.dtype, batch * N)
    _check_dev(v, "v", torch.float64)
    v_stride = 0 if v.numel() == N else N
    if g0 is None:
        g0 = torch.empty_like(uT)
    if gv is None:
        gv = torch.empty(N if v_stride == 0 else (batch, N), dtype=torch.float64, device=uT.device)
    if ckpt is not None:
        _check_dev(ckpt, "ckpt", uT.dtype, num_checkpoints(steps, ckpt_every) * batch * N)
    wb = 0
    if work is not None:
        _check_dev(work, "work")
        wb = work.numel() * work.element_size()
    _check(lib.strang_adjoint(plan.handle, prec, batch, _dev_ptr(v), v_stride, _dev_ptr(uT), _dev_ptr(gT),
                              float(gamma), float(dt), int(steps), _dev_ptr(ckpt), int(ckpt_every),
                              _dev_ptr(g0), _dev_ptr(gv), _dev_ptr(work), wb, _stream(stream)),
           "strang_adjoint")
    return g0, gv


def strang_batched_workspace_size(plans: Sequence[Plan], prec: int) -> int:
    arr = (_P * len(plans))(*[p.handle for p in plans])
    n = _sz()
    _check(lib.strang_batched_workspace_size(len(plans), arr, prec, ctypes.byref(n)),
           "strang_batched_workspace_size")
    return n.value


def strang_run_batched(plans: Sequence[Plan], vs, us, gammas, dts, steps, work=None, stream=None):
    """Advance B unrelated problems together (each u in place)."""
    import torch
    B = len(plans)
    if not (len(vs) == len(us) == len(gammas) == len(dts) == len(steps) == B):
        raise ValueError("all per-problem sequences must have length B")
    prec = _prec_of(us[0]) if B else LT_C64
    for b in range(B):
        _check_dev(us[b], f"u[{b}]", us[0].dtype, plans[b].N)
        _check_dev(vs[b], f"v[{b}]", torch.float64, plans[b].N)
    parr = (_P * B)(*[p.handle for p in plans])
    varr = (_P * B)(*[v.data_ptr() for v in vs])
    uarr = (_P * B)(*[u.data_ptr() for u in us])
    g = np.ascontiguousarray(gammas, dtype=np.float64)
    dtt = np.ascontiguousarray(dts, dtype=np.float64)
    st = np.ascontiguousarray(steps, dtype=np.int64)
    wb = 0
    if work is not None:
        _check_dev(work, "work")
        wb = work.numel() * work.element_size()
    _check(lib.strang_run_batched(B, parr, prec, varr, uarr, _np_ptr(g), _np_ptr(dtt), _np_ptr(st),
                                  _dev_ptr(work), wb, _stream(stream)), "strang_run_batched")
    return us


class Batch:
    """Owner of an lt_batch*: the problems of strang_run_batched planned once.
    Holds references to the plans, potentials and states it points to."""

    def __init__(self, handle: int, plans, vs, us):
        self._h = handle
        self._keep = (list(plans), list(vs), list(us))

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            lib.strang_batch_destroy(h)


def strang_batch_create(plans: Sequence[Plan], vs, us, gammas, dts, steps, stream=None) -> Batch:
    """Plan B unrelated problems once (tables built on the device); the
    returned object advances the states us in place on every strang_batch_run."""
    import torch
    B = len(plans)
    if not (len(vs) == len(us) == len(gammas) == len(dts) == len(steps) == B):
        raise ValueError("all per-problem sequences must have length B")
    prec = _prec_of(us[0]) if B else LT_C64
    for b in range(B):
        _check_dev(us[b], f"u[{b}]", us[0].dtype, plans[b].N)
        _check_dev(vs[b], f"v[{b}]", torch.float64, plans[b].N)
    parr = (_P * max(B, 1))(*[p.handle for p in plans])
    varr = (_P * max(B, 1))(*[v.data_ptr() for v in vs])
    uarr = (_P * max(B, 1))(*[u.data_ptr() for u in us])
    g = np.ascontiguousarray(gammas, dtype=np.float64)
    dtt = np.ascontiguousarray(dts, dtype=np.float64)
    st = np.ascontiguousarray(steps, dtype=np.int64)
    h = _P()
    _check(lib.strang_batch_create(B, parr, prec, varr, uarr, _np_ptr(g), _np_ptr(dtt), _np_ptr(st),
                                   _stream(stream), ctypes.byref(h)), "strang_batch_create")
    return Batch(h.value, plans, vs, us)


def strang_batch_run(batch: Batch, stream=None) -> None:
    _check(lib.strang_batch_run(batch.handle, _stream(stream)), "strang_batch_run")


def strang_batch_autotune(batch: Batch, reps: int = 5, stream=None) -> None:
    _check(lib.strang_batch_autotune(batch.handle, int(reps), _stream(stream)), "strang_batch_autotune")


def strang_batch_kernels(batch: Batch):
    """[(key, variant)] per register-staged class: key > 0 a column class of
    that column length, key < 0 a row class (-key = 2 L2 + multiplier kind)."""
    n = _i32()
    _check(lib.strang_batch_kernels(batch.handle, ctypes.byref(n), None, None, 0), "strang_batch_kernels")
    key = np.zeros(max(n.value, 1), dtype=np.int32)
    var = np.zeros(max(n.value, 1), dtype=np.int32)
    _check(lib.strang_batch_kernels(batch.handle, ctypes.byref(n), _np_ptr(key), _np_ptr(var), n.value),
           "strang_batch_kernels")
    return [(int(k), int(v)) for k, v in zip(key[:n.value], var[:n.value])]


def splitting_workspace_size(plan: Plan, prec: int, batch: int, shared_v: bool, order: int) -> int:
    n = _sz()
    _check(lib.splitting_workspace_size(plan.handle, prec, batch, int(bool(shared_v)), order, ctypes.byref(n)),
           "splitting_workspace_size")
    return n.value


def lattice_projection_error_workspace_size(plan: Plan, prec: int, batch: int) -> int:
    n = _sz()
    _check(lib.lattice_projection_error_workspace_size(plan.handle, prec, batch, ctypes.byref(n)),
           "lattice_projection_error_workspace_size")
    return n.value


def lattice_projection_error(plan: Plan, u, ghat, out=None, work=None, stream=None):
    """(sum_A |ghat|^2, sum_A |ghat - ghat_a|^2) per state (device float64,
    (batch, 2)) for point values u (device, (N,) or (batch, N)) and the exact
    coefficients ghat (device complex128, same shape, key order)."""
    import torch
    N = plan.N
    prec = _prec_of(u)
    batch = u.numel() // N
    _check_dev(u, "u", numel=batch * N)
    _check_dev(ghat, "ghat", torch.complex128, batch * N)
    if out is None:
        out = torch.empty((batch, 2), dtype=torch.float64, device=u.device)
    _check_dev(out, "out", torch.float64, 2 * batch)
    wb = 0
    if work is not None:
        _check_dev(work, "work")
        wb = work.numel() * work.element_size()
    _check(lib.lattice_projection_error(plan.handle, prec, batch, _dev_ptr(u), _dev_ptr(ghat), _dev_ptr(out),
                                        _dev_ptr(work), wb, _stream(stream)), "lattice_projection_error")
    return out


def splitting_times(order: int, steps: int, t0: float, dt: float):
    """Substep boundaries tau (numpy, steps * P + 1) at which splitting_run
    samples the coefficient f of a time-dependent field."""
    import numpy as np
    P = 3 if order == 4 else 1
    tau = np.empty(max(0, steps) * P + 1)
    _check(lib.splitting_times(int(order), int(steps), float(t0), float(dt),
                               tau.ctypes.data_as(ctypes.c_void_p)), "splitting_times")
    return tau


def splitting_run(plan: Plan, v, u, gamma: float, dt: float, steps: int, order: int = 4, v1=None, f=None,
                  work=None, stream=None):
    """In-place run of a symmetric composition of Strang steps (order 2 or 4)
    under v, or under v + f(tau) v1 when v1 (device float64, shaped as v) and
    f (host values at splitting_times(order, steps, t0, dt)) are given."""
    import numpy as np
    import torch
    N = plan.N
    prec = _prec_of(u)
    batch = u.numel() // N
    _check_dev(u, "u", numel=batch * N)
    _check_dev(v, "v", torch.float64)
    if v.numel() not in (N, batch * N):
        raise ValueError("v must hold N or batch*N values")
    fh = None
    if v1 is not None:
        _check_dev(v1, "v1", torch.float64, v.numel())
        if f is None:
            raise ValueError("a time-dependent field v1 needs its coefficients f")
        fh = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        if fh.size != steps * (3 if order == 4 else 1) + 1:
            raise ValueError("f must hold steps * P + 1 values (P = 3 for order 4, else 1)")
    wb = 0
    if work is not None:
        _check_dev(work, "work")
        wb = work.numel() * work.element_size()
    _check(lib.splitting_run(plan.handle, prec, batch, _dev_ptr(v), _dev_ptr(v1), 0 if v.numel() == N else N,
                             None if fh is None else fh.ctypes.data_as(ctypes.c_void_p), _dev_ptr(u),
                             float(gamma), float(dt), int(steps), int(order), _dev_ptr(work), wb,
                             _stream(stream)), "splitting_run")
    return u


def lattice_diagnostics_workspace_size(plan: Plan, prec: int, batch: int) -> int:
    n = _sz()
    _check(lib.lattice_diagnostics_workspace_size(plan.handle, prec, batch, ctypes.byref(n)),
           "lattice_diagnostics_workspace_size")
    return n.value


def lattice_diagnostics(plan: Plan, v, u, gamma: float, out=None, work=None, stream=None):
    """(norm^2, energy) of each state of u (device, (N,) or (batch, N)) under v
    (device float64, (N,) shared or (batch, N)): a (batch, 2) float64 tensor."""
    import torch
    N = plan.N
    prec = _prec_of(u)
    batch = u.numel() // N
    _check_dev(u, "u", numel=batch * N)
    _check_dev(v, "v", torch.float64)
    if v.numel() not in (N, batch * N):
        raise ValueError("v must hold N or batch*N values")
    if out is None:
        out = torch.empty((batch, 2), dtype=torch.float64, device=u.device)
    _check_dev(out, "out", torch.float64, 2 * batch)
    wb = 0
    if work is not None:
        _check_dev(work, "work")
        wb = work.numel() * work.element_size()
    _check(lib.lattice_diagnostics(plan.handle, prec, batch, _dev_ptr(v), 0 if v.numel() == N else N, _dev_ptr(u),
                                   float(gamma), _dev_ptr(out), _dev_ptr(work), wb, _stream(stream)),
           "lattice_diagnostics")
    return out


LT_KIND_COLUMN, LT_KIND_ROW, LT_KIND_RESIDENT = 0, 1, 2


def lt_timing_enable(on: bool) -> None:
    _check(lib.lt_timing_enable(int(bool(on))), "lt_timing_enable")


def lt_timing_summary(kind: int):
    """(launches, total_ms) of the recorded launches of one kernel class."""
    n, ms = _i64(), _f64()
    _check(lib.lt_timing_summary(kind, ctypes.byref(n), ctypes.byref(ms)), "lt_timing_summary")
    return n.value, ms.value


def lattice_plan_autotune(plan: Plan, prec: int, reps: int = 10, stream=None):
    """Time the kernel variants of the plan's passes on one state and on many
    states and keep the fastest of each; returns the single-state (column,
    row) choice (lattice_plan_get_kernels_batch reports the other)."""
    _check(lib.lattice_plan_autotune(plan.handle, prec, reps, _stream(stream)), "lattice_plan_autotune")
    return lattice_plan_get_kernels(plan, prec)


def lattice_plan_set_kernels(plan: Plan, prec: int, col_variant: int, row_variant: int) -> None:
    _check(lib.lattice_plan_set_kernels(plan.handle, prec, col_variant, row_variant),
           "lattice_plan_set_kernels")


def lattice_plan_get_kernels(plan: Plan, prec: int):
    cv, rv = _i32(), _i32()
    _check(lib.lattice_plan_get_kernels(plan.handle, prec, ctypes.byref(cv), ctypes.byref(rv)),
           "lattice_plan_get_kernels")
    return cv.value, rv.value


def lattice_plan_get_kernels_batch(plan: Plan, prec: int, batch: int):
    """(column, row) variants a launch of `batch` states takes."""
    cv, rv = _i32(), _i32()
    _check(lib.lattice_plan_get_kernels_batch(plan.handle, prec, batch, ctypes.byref(cv), ctypes.byref(rv)),
           "lattice_plan_get_kernels_batch")
    return cv.value, rv.value
