"""Thin ctypes binding of the C ABI in ``include/swr.h``.

Names mirror the C entry points (``swr_setup``, ``swr_solve``, ``swr_grad``,
``swr_apply_R``, ``swr_build_interface``, ``swr_interface_matvec``,
``swr_destroy``).  This module only marshals arguments: every step of the
solver runs in the HIP library ``_swr_hip.so``.  PyTorch supplies device memory
(complex128 / float64 CUDA tensors) and the current HIP stream.

Every array argument is checked before its pointer crosses the ABI: dtype
(float64 / complex128), device (the current GPU), contiguity and element
count against the context's sizes (``swr_sizes``).  The library itself cannot
see the extent of a raw pointer, so a wrong tensor would otherwise be read or
written past its end.

If the library is missing this module raises at import time; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_swr_hip.so")

SWR_OK, SWR_EINVAL, SWR_ENOMEM, SWR_EDEVICE, SWR_ENOCONV, SWR_ENAN = range(6)
SWR_ROBIN, SWR_S02, SWR_S03, SWR_S04, SWR_S12, SWR_S14, SWR_P22, SWR_P24 = 0, 1, 2, 3, 4, 5, 6, 7
SWR_V_STATIC, SWR_V_TIME, SWR_V_CUBIC = 0, 1, 2
SWR_SOLVER_FIXED, SWR_SOLVER_GMRES, SWR_SOLVER_CAUSAL, SWR_SOLVER_BICGSTAB = 0, 1, 2, 3


class SwrOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("restart", ctypes.c_int),
                ("solver", ctypes.c_int), ("precond", ctypes.c_int), ("batch", ctypes.c_int),
                ("v_per_problem", ctypes.c_int), ("checkpoint_K", ctypes.c_int),
                ("nl_max_iter", ctypes.c_int), ("nl_tol", ctypes.c_double),
                ("pipeline", ctypes.c_int), ("plain", ctypes.c_int),
                ("snapshot_stride", ctypes.c_int), ("tune_cache", ctypes.c_char_p),
                ("pade_m", ctypes.c_int), ("pade_theta", ctypes.c_double)]


class SwrInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("residual", ctypes.c_double),
                ("t_factor_ms", ctypes.c_double), ("t_build_ms", ctypes.c_double),
                ("t_iface_ms", ctypes.c_double), ("t_final_ms", ctypes.c_double),
                ("nl_worst", ctypes.c_int), ("t_total_ms", ctypes.c_double),
                ("t_sweep_ms", ctypes.c_double), ("n_sweep", ctypes.c_int),
                ("inner_iters", ctypes.c_int), ("history_ptr", ctypes.POINTER(ctypes.c_double)),
                ("history_len", ctypes.c_int)]

    @property
    def history(self):
        """Convergence measure after every interface iteration (a copy; the
        library's array is only valid until the next call on the context)."""
        n = int(self.history_len)
        if n <= 0 or not self.history_ptr:
            return np.zeros(0)
        return np.ctypeslib.as_array(self.history_ptr, shape=(n,)).copy()

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "history_ptr"}
        d["history"] = self.history.tolist()
        return d


class SwrSchedule(ctypes.Structure):
    _fields_ = [("pipeline", ctypes.c_int), ("help_max", ctypes.c_int), ("restart", ctypes.c_int),
                ("pair_from", ctypes.c_int), ("graph", ctypes.c_int), ("check", ctypes.c_int),
                ("group", ctypes.c_int), ("ms", ctypes.c_double),
                ("candidates", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# exported symbols of include/swr.h
EXPORTS = ("swr_default_opts", "swr_strerror", "swr_setup", "swr_solve", "swr_grad",
           "swr_apply_R", "swr_build_interface", "swr_interface_matvec", "swr_destroy",
           "swr_sizes", "swr_set_potential", "swr_tune", "swr_get_schedule", "swr_set_schedule",
           "swr_apply_R_noalloc")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
# PyTorch's HIP runtime first: the library then binds to the same runtime
# (one per process).  Loaded the other way round, the library's own copy of
# the runtime comes first and reports no device to the calls made through it.
import torch  # noqa: E402,F401
_L = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_I = ctypes.POINTER(ctypes.c_int)
_L.swr_default_opts.argtypes = [ctypes.POINTER(SwrOpts)]
_L.swr_default_opts.restype = None
_L.swr_strerror.argtypes = [ctypes.c_int]
_L.swr_strerror.restype = ctypes.c_char_p
_L.swr_setup.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, _P, ctypes.c_double,
                         ctypes.c_double, ctypes.c_int, _P, ctypes.c_int, ctypes.c_double,
                         ctypes.c_double, ctypes.POINTER(SwrOpts), _P, ctypes.POINTER(_P)]
_L.swr_setup.restype = ctypes.c_int
_L.swr_solve.argtypes = [_P, _P, _P, _P, _P, _P, ctypes.POINTER(SwrInfo)]
_L.swr_solve.restype = ctypes.c_int
_L.swr_grad.argtypes = [_P, _P, _P, _P, _P, ctypes.POINTER(SwrInfo)]
_L.swr_grad.restype = ctypes.c_int
_L.swr_apply_R.argtypes = [_P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_double)]
_L.swr_apply_R.restype = ctypes.c_int
_L.swr_apply_R_noalloc.argtypes = [_P, _P, _P, _P, _P, _P]
_L.swr_apply_R_noalloc.restype = ctypes.c_int
_L.swr_build_interface.argtypes = [_P, _P, _P, _P]
_L.swr_build_interface.restype = ctypes.c_int
_L.swr_interface_matvec.argtypes = [_P, _P, _P]
_L.swr_interface_matvec.restype = ctypes.c_int
_L.swr_destroy.argtypes = [_P]
_L.swr_destroy.restype = None
_L.swr_sizes.argtypes = [_P] + [_I] * 7
_L.swr_sizes.restype = ctypes.c_int
_L.swr_set_potential.argtypes = [_P, _P]
_L.swr_set_potential.restype = ctypes.c_int
_L.swr_tune.argtypes = [_P, _P, ctypes.c_double, ctypes.POINTER(SwrSchedule)]
_L.swr_tune.restype = ctypes.c_int
_L.swr_get_schedule.argtypes = [_P, ctypes.POINTER(SwrSchedule)]
_L.swr_get_schedule.restype = ctypes.c_int
_L.swr_set_schedule.argtypes = [_P, ctypes.POINTER(SwrSchedule)]
_L.swr_set_schedule.restype = ctypes.c_int


class SwrError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {swr_strerror(status)} (status {status})")


def swr_strerror(status: int) -> str:
    return _L.swr_strerror(int(status)).decode()


def swr_default_opts() -> SwrOpts:
    o = SwrOpts()
    _L.swr_default_opts(ctypes.byref(o))
    return o


def _arr(t, kind, count, name):
    """Pointer of a CUDA tensor after checking what the C ABI cannot: dtype
    (kind 'c' complex128, 'd' float64), device (the current GPU), contiguity
    and element count.  None passes through as NULL."""
    if t is None:
        return None
    import torch
    want = torch.complex128 if kind == "c" else torch.float64
    if t.dtype != want:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {want}")
    if not t.is_cuda:
        raise ValueError(f"{name}: tensor must live on the GPU")
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name}: tensor on {t.device}, the current device is "
                         f"cuda:{torch.cuda.current_device()}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if t.numel() != count:
        raise ValueError(f"{name}: {t.numel()} elements, expected {count}")
    return ctypes.c_void_p(t.data_ptr())


def _check(status, where, allow_noconv=False):
    if status == SWR_OK or (allow_noconv and status == SWR_ENOCONV):
        return status
    raise SwrError(status, where)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Sizes:
    nt: int
    nx: int
    B: int
    nv: int
    N: int
    vk: int
    S: int

    @property
    def ns(self):
        return 2 * self.N - 2

    @property
    def vec(self):
        return self.B * self.ns * self.nt

    def v_count(self):
        return self.nx * (self.nt + 1) if self.vk == SWR_V_TIME else self.nx * self.nv


def _sizes(ctx) -> Sizes:
    v = [ctypes.c_int(0) for _ in range(7)]
    _check(_L.swr_sizes(ctx, *[ctypes.byref(x) for x in v]), "swr_sizes")
    return Sizes(*(x.value for x in v))


def swr_setup(a0, b0, J, dt, T, vkind, V, trans, s=1 - 1j, opts: SwrOpts | None = None):
    """Create a context (see swr_setup in include/swr.h).  J: host int
    sequence; V: float64 CUDA tensor or None.  Returns the opaque handle."""
    Jarr = np.ascontiguousarray(np.asarray(J, dtype=np.int32))
    vp = None
    if V is not None:
        nx = int(Jarr.sum()) + 1
        nt = int(round(T / dt))
        B = opts.batch if opts is not None else 1
        if vkind == SWR_V_TIME:
            count = nx * (nt + 1)
        elif opts is not None and opts.v_per_problem:
            count = nx * B
        else:
            count = nx
        vp = _arr(V, "d", count, "V")
    out = _P()
    st = _L.swr_setup(float(a0), float(b0), int(len(Jarr)), Jarr.ctypes.data_as(_P), float(dt),
                      float(T), int(vkind), vp, int(trans), float(complex(s).real),
                      float(complex(s).imag), ctypes.byref(opts) if opts is not None else None,
                      _stream(), ctypes.byref(out))
    _check(st, "swr_setup")
    return out


def swr_destroy(ctx):
    if ctx:
        _L.swr_destroy(ctx)


def swr_solve(ctx, u0, uT, g=None, utrace=None, snaps=None):
    """Returns (status, info).  SWR_ENOCONV is returned, not raised (the
    outputs hold the last iterate); check the status.  snaps [B][S][nx] needs
    a context made with opts.snapshot_stride > 0."""
    z = _sizes(ctx)
    info = SwrInfo()
    S = z.S
    if snaps is not None and S == 0:
        raise ValueError("snaps: the context was made without opts.snapshot_stride")
    st = _L.swr_solve(ctx, _arr(u0, "c", z.B * z.nx, "u0"), _arr(uT, "c", z.B * z.nx, "uT"),
                      _arr(g, "c", z.vec, "g"), _arr(utrace, "c", z.B * z.N * 2 * (z.nt + 1), "utrace"),
                      _arr(snaps, "c", z.B * S * z.nx, "snaps") if snaps is not None else None,
                      ctypes.byref(info))
    _check(st, "swr_solve", allow_noconv=True)
    return st, info


def swr_grad(ctx, u0, gbar, dJdV, dJdu0):
    """Returns (status, info); SWR_ENOCONV is returned, not raised."""
    z = _sizes(ctx)
    n = z.B * z.nx
    info = SwrInfo()
    st = _L.swr_grad(ctx, _arr(u0, "c", n, "u0"), _arr(gbar, "c", n, "gbar"),
                     _arr(dJdV, "d", n, "dJdV"), _arr(dJdu0, "c", n, "dJdu0"), ctypes.byref(info))
    _check(st, "swr_grad", allow_noconv=True)
    return st, info


def swr_apply_R(ctx, u0, g_in, g_out, uT=None, want_maxdiff=False):
    z = _sizes(ctx)
    md = ctypes.c_double(0.0)
    st = _L.swr_apply_R(ctx, _arr(u0, "c", z.B * z.nx, "u0"), _arr(g_in, "c", z.vec, "g_in"),
                        _arr(g_out, "c", z.vec, "g_out"), _arr(uT, "c", z.B * z.nx, "uT"),
                        ctypes.byref(md) if want_maxdiff else None)
    _check(st, "swr_apply_R")
    return md.value


def swr_apply_R_noalloc(ctx, u0, g_in, g_out, uT=None, maxdiff=None):
    """swr_apply_R with the library's static scratch (no allocation, no
    synchronisation); maxdiff: a one-element float64 CUDA tensor or None."""
    z = _sizes(ctx)
    st = _L.swr_apply_R_noalloc(ctx, _arr(u0, "c", z.B * z.nx, "u0"), _arr(g_in, "c", z.vec, "g_in"),
                                _arr(g_out, "c", z.vec, "g_out"), _arr(uT, "c", z.B * z.nx, "uT"),
                                _arr(maxdiff, "d", 1, "maxdiff"))
    _check(st, "swr_apply_R_noalloc")


def swr_build_interface(ctx, u0, cols=None, d=None):
    z = _sizes(ctx)
    nvc = z.nv if z.vk == SWR_V_STATIC else 1
    _check(_L.swr_build_interface(ctx, _arr(u0, "c", z.B * z.nx, "u0"),
                                  _arr(cols, "c", nvc * z.N * 4 * z.nt, "cols"),
                                  _arr(d, "c", z.vec, "d")), "swr_build_interface")


def swr_interface_matvec(ctx, x, y):
    z = _sizes(ctx)
    _check(_L.swr_interface_matvec(ctx, _arr(x, "c", z.vec, "x"), _arr(y, "c", z.vec, "y")),
           "swr_interface_matvec")


def swr_set_potential(ctx, V):
    z = _sizes(ctx)
    _check(_L.swr_set_potential(ctx, _arr(V, "d", z.v_count(), "V")), "swr_set_potential")


def swr_tune(ctx, u0, budget_ms=2000.0):
    """Time candidate schedules on u0 and keep the fastest (see swr_tune in
    include/swr.h); returns the chosen SwrSchedule."""
    z = _sizes(ctx)
    out = SwrSchedule()
    _check(_L.swr_tune(ctx, _arr(u0, "c", z.B * z.nx, "u0"), float(budget_ms), ctypes.byref(out)),
           "swr_tune")
    return out


def swr_get_schedule(ctx):
    out = SwrSchedule()
    _check(_L.swr_get_schedule(ctx, ctypes.byref(out)), "swr_get_schedule")
    return out


def swr_set_schedule(ctx, pipeline=None, help_max=None, restart=None, pair_from=None, graph=None,
                     check=None, group=None):
    """Change some parameters of the context's schedule (the rest stay)."""
    cur = swr_get_schedule(ctx)
    for k, v in (("pipeline", pipeline), ("help_max", help_max), ("restart", restart),
                 ("pair_from", pair_from), ("graph", graph), ("check", check), ("group", group)):
        if v is not None:
            setattr(cur, k, int(v))
    _check(_L.swr_set_schedule(ctx, ctypes.byref(cur)), "swr_set_schedule")
    return cur


def swr_sizes(ctx):
    """(nt, nx, B, nv) of a context (swr_sizes also reports N and vk)."""
    z = _sizes(ctx)
    return z.nt, z.nx, z.B, z.nv


@dataclass
class Problem:
    """Convenience owner of one context (argument marshalling only)."""
    a0: float
    b0: float
    J: tuple
    dt: float
    T: float
    vkind: int
    trans: int
    s: complex = 1 - 1j
    opts: SwrOpts | None = None
    V: object = None

    def __post_init__(self):
        self.ctx = swr_setup(self.a0, self.b0, self.J, self.dt, self.T, self.vkind, self.V,
                             self.trans, self.s, self.opts)
        self.nt, self.nx, self.B, self.nv = swr_sizes(self.ctx)
        self.N = len(self.J)
        self.ns = 2 * self.N - 2

    def close(self):
        if getattr(self, "ctx", None):
            swr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
