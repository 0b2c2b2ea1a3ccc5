"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/swr.h, and rejects invalid arguments before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swr.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(swr_[a-zA-Z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def swr():
    from paper_1503_02564_amd import build
    if not os.path.exists(build.LIB):
        build.build(force=True)
    from paper_1503_02564_amd import swr as m
    return m


def test_every_declared_symbol_is_exported(swr):
    lib = ctypes.CDLL(swr.LIB_PATH)
    names = _declared()
    assert "swr_setup" in names and "swr_solve" in names and "swr_grad" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(swr.EXPORTS)


def test_defaults_and_strerror(swr):
    o = swr.swr_default_opts()
    assert o.tol == 1e-10 and o.restart == 30 and o.batch == 1
    assert o.solver == swr.SWR_SOLVER_CAUSAL and o.checkpoint_K == 64
    assert o.pipeline == -1 and o.plain == 0 and o.nl_max_iter == 100
    assert o.pade_m == 20 and abs(o.pade_theta - np.pi / 4) < 1e-15
    for s in range(6):
        assert swr.swr_strerror(s)
    assert swr.swr_strerror(99) == "unknown status"


def _setup_raw(swr, a0=-1.0, b0=1.0, J=(4, 4), dt=0.1, T=1.0, vk=0, tr=1, s=(1.0, -1.0), opts=None):
    Jarr = np.asarray(J, dtype=np.int32)
    out = ctypes.c_void_p()
    return swr._L.swr_setup(a0, b0, len(Jarr), Jarr.ctypes.data_as(ctypes.c_void_p), dt, T, vk, None,
                            tr, s[0], s[1], ctypes.byref(opts) if opts else None, None,
                            ctypes.byref(out)), out


@pytest.mark.parametrize("kw", [
    dict(a0=1.0, b0=-1.0), dict(J=()), dict(J=(4, 0)), dict(dt=0.0), dict(T=-1.0),
    dict(dt=0.3, T=1.0), dict(vk=7), dict(tr=8), dict(tr=-1), dict(tr=0, s=(0.0, 0.0)),
    dict(tr=3, vk=2), dict(tr=5, vk=2), dict(tr=7, vk=2),
    dict(J=(600000,)), dict(J=(600,), tr=2), dict(vk=1), dict(dt=float("nan")),
])
def test_setup_rejects_invalid_arguments(swr, kw):
    if kw.get("J") == ():
        st, out = swr._L.swr_setup(-1.0, 1.0, 0, None, 0.1, 1.0, 0, None, 1, 0.0, 0.0, None, None,
                                   ctypes.byref(ctypes.c_void_p())), None
    else:
        st, out = _setup_raw(swr, **kw)
    assert st == swr.SWR_EINVAL


def test_setup_rejects_bad_opts(swr):
    for field, val in (("batch", 0), ("restart", 0), ("max_iter", 0), ("tol", 0.0),
                       ("pipeline", 100), ("pipeline", -64), ("nl_max_iter", 0)):
        o = swr.swr_default_opts()
        setattr(o, field, val)
        st, _ = _setup_raw(swr, opts=o)
        assert st == swr.SWR_EINVAL, field
    # Pade strategy: 1..128 auxiliary functions, branch rotation in (0, pi)
    for field, val in (("pade_m", 0), ("pade_m", 129), ("pade_theta", 0.0), ("pade_theta", np.pi),
                       ("pade_theta", float("nan"))):
        o = swr.swr_default_opts()
        setattr(o, field, val)
        st, _ = _setup_raw(swr, tr=swr.SWR_P22, opts=o)
        assert st == swr.SWR_EINVAL, field


def test_calls_reject_null_context(swr):
    assert swr._L.swr_solve(None, None, None, None, None, None, None) == swr.SWR_EINVAL
    assert swr._L.swr_apply_R(None, None, None, None, None, None) == swr.SWR_EINVAL
    assert swr._L.swr_grad(None, None, None, None, None, None) == swr.SWR_EINVAL
    swr._L.swr_destroy(None)
