"""Thin ctypes binding of the C ABI in ``include/swr.h``.

Names mirror the C entry points (``swr_setup``, ``swr_solve``, ``swr_grad``,
``swr_apply_R``, ``swr_build_interface``, ``swr_interface_matvec``,
``swr_destroy``).  This module only marshals arguments: every step of the
solver runs in the HIP library ``_swr_hip.so``.  PyTorch supplies device memory
(complex128 / float64 CUDA tensors) and the current HIP stream.

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
SWR_ROBIN, SWR_S02, SWR_S03, SWR_S04, SWR_S12, SWR_S14 = 0, 1, 2, 3, 4, 5
SWR_V_STATIC, SWR_V_TIME, SWR_V_CUBIC = 0, 1, 2
SWR_SOLVER_FIXED, SWR_SOLVER_GMRES, SWR_SOLVER_CAUSAL, SWR_SOLVER_BICGSTAB = 0, 1, 2, 3


class SwrOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("restart", ctypes.c_int),
                ("solver", ctypes.c_int), ("precond", ctypes.c_int), ("batch", ctypes.c_int),
                ("v_per_problem", ctypes.c_int), ("checkpoint_K", ctypes.c_int),
                ("nl_max_iter", ctypes.c_int), ("nl_tol", ctypes.c_double),
                ("pipeline", ctypes.c_int), ("plain", ctypes.c_int)]


class SwrInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("residual", ctypes.c_double),
                ("t_factor_ms", ctypes.c_double), ("t_build_ms", ctypes.c_double),
                ("t_iface_ms", ctypes.c_double), ("t_final_ms", ctypes.c_double),
                ("nl_worst", ctypes.c_int), ("t_total_ms", ctypes.c_double),
                ("t_sweep_ms", ctypes.c_double), ("n_sweep", ctypes.c_int),
                ("inner_iters", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# exported symbols of include/swr.h
EXPORTS = ("swr_default_opts", "swr_strerror", "swr_setup", "swr_solve", "swr_grad",
           "swr_apply_R", "swr_build_interface", "swr_interface_matvec", "swr_destroy",
           "swr_sizes", "swr_set_potential")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
_L = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_L.swr_default_opts.argtypes = [ctypes.POINTER(SwrOpts)]
_L.swr_default_opts.restype = None
_L.swr_strerror.argtypes = [ctypes.c_int]
_L.swr_strerror.restype = ctypes.c_char_p
_L.swr_setup.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, _P, ctypes.c_double,
                         ctypes.c_double, ctypes.c_int, _P, ctypes.c_int, ctypes.c_double,
                         ctypes.c_double, ctypes.POINTER(SwrOpts), _P, ctypes.POINTER(_P)]
_L.swr_setup.restype = ctypes.c_int
_L.swr_solve.argtypes = [_P, _P, _P, _P, _P, ctypes.POINTER(SwrInfo)]
_L.swr_solve.restype = ctypes.c_int
_L.swr_grad.argtypes = [_P, _P, _P, _P, _P, ctypes.POINTER(SwrInfo)]
_L.swr_grad.restype = ctypes.c_int
_L.swr_apply_R.argtypes = [_P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_double)]
_L.swr_apply_R.restype = ctypes.c_int
_L.swr_build_interface.argtypes = [_P, _P, _P, _P]
_L.swr_build_interface.restype = ctypes.c_int
_L.swr_interface_matvec.argtypes = [_P, _P, _P]
_L.swr_interface_matvec.restype = ctypes.c_int
_L.swr_destroy.argtypes = [_P]
_L.swr_destroy.restype = None
_L.swr_sizes.argtypes = [_P] + [ctypes.POINTER(ctypes.c_int)] * 4
_L.swr_sizes.restype = ctypes.c_int
_L.swr_set_potential.argtypes = [_P, _P]
_L.swr_set_potential.restype = ctypes.c_int


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


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _check(status, where, allow_noconv=False):
    if status == SWR_OK or (allow_noconv and status == SWR_ENOCONV):
        return status
    raise SwrError(status, where)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def swr_setup(a0, b0, J, dt, T, vkind, V, trans, s=1 - 1j, opts: SwrOpts | None = None):
    """Create a context (see swr_setup in include/swr.h).  J: host int
    sequence; V: float64 CUDA tensor or None.  Returns the opaque handle."""
    Jarr = np.ascontiguousarray(np.asarray(J, dtype=np.int32))
    out = _P()
    st = _L.swr_setup(float(a0), float(b0), int(len(Jarr)), Jarr.ctypes.data_as(_P), float(dt),
                      float(T), int(vkind), _ptr(V), int(trans), float(complex(s).real),
                      float(complex(s).imag), ctypes.byref(opts) if opts is not None else None,
                      _stream(), ctypes.byref(out))
    _check(st, "swr_setup")
    return out


def swr_destroy(ctx):
    if ctx:
        _L.swr_destroy(ctx)


def swr_solve(ctx, u0, uT, g=None, utrace=None):
    info = SwrInfo()
    st = _L.swr_solve(ctx, _ptr(u0), _ptr(uT), _ptr(g), _ptr(utrace), ctypes.byref(info))
    _check(st, "swr_solve", allow_noconv=True)
    return st, info


def swr_grad(ctx, u0, gbar, dJdV, dJdu0):
    info = SwrInfo()
    st = _L.swr_grad(ctx, _ptr(u0), _ptr(gbar), _ptr(dJdV), _ptr(dJdu0), ctypes.byref(info))
    _check(st, "swr_grad", allow_noconv=True)
    return st, info


def swr_apply_R(ctx, u0, g_in, g_out, uT=None, want_maxdiff=False):
    md = ctypes.c_double(0.0)
    st = _L.swr_apply_R(ctx, _ptr(u0), _ptr(g_in), _ptr(g_out), _ptr(uT),
                        ctypes.byref(md) if want_maxdiff else None)
    _check(st, "swr_apply_R")
    return md.value


def swr_build_interface(ctx, u0, cols=None, d=None):
    _check(_L.swr_build_interface(ctx, _ptr(u0), _ptr(cols), _ptr(d)), "swr_build_interface")


def swr_interface_matvec(ctx, x, y):
    _check(_L.swr_interface_matvec(ctx, _ptr(x), _ptr(y)), "swr_interface_matvec")


def swr_set_potential(ctx, V):
    _check(_L.swr_set_potential(ctx, _ptr(V)), "swr_set_potential")


def swr_sizes(ctx):
    v = [ctypes.c_int(0) for _ in range(4)]
    _check(_L.swr_sizes(ctx, *[ctypes.byref(x) for x in v]), "swr_sizes")
    return tuple(x.value for x in v)


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
