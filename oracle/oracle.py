"""Python layer of the CPU oracle.  TEST INFRASTRUCTURE ONLY (see package doc).

The time stepping lives in ``swr_oracle.c`` (plain C99, FP64 complex); this
module marshals arrays and writes out the interface-level algorithms of the
paper in numpy, in the paper's order and notation:

* ``apply_R``          -- one SWR iteration g -> R g  (Sec. 3, eq. interfacepbR)
* ``classical``        -- fixed point on g           (Sec. 4, "Classical algorithm")
* ``impulse_columns``  -- first columns of the X blocks by impulse solves (Sec. 4.1)
* ``brute_L``          -- L column by column from R(e_i) (Props. 1-2), tiny sizes
* ``ltt_apply``        -- L g from first columns     (Props. 3-4: lower-triangular Toeplitz)
* ``gmres``            -- restarted GMRES (Saad, Alg. 6.9), plain MGS + Givens
* ``bicgstab``         -- BiCGStab (van der Vorst 1992), the paper's GPU solver
* ``causal_solve``     -- (I - L) g = d by forward substitution in time
* ``new_algorithm``    -- Sec. 4 "New algorithm": build L and d, solve, final sweep
* ``preconditioned``   -- Sec. 5: P = I - L_0 for V(t,x) and |u|^2
* ``mono`` / ``adjoint_mono`` -- monodomain CN and its discrete adjoint

Interface vector layout (Sec. 3): g = (r_1 | l_2, r_2 | ... | l_N), stored as
an array ``[2N-2, nt]``.  With 0-based subdomain k: l_k sits in slot 2k-1
(k >= 1), r_k in slot 2k (k <= N-2); subdomain k writes r_{k-1} (slot 2k-2)
and l_{k+1} (slot 2k+1).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import scipy.linalg

from paper_1503_02564_amd.workloads import (S02, S03, S04, S12, S14, V_CUBIC, V_STATIC,  # noqa: F401
                                            V_TIME,
                                            Workload, ROBIN)
from . import build as _build

__all__ = [
    "lib", "alpha", "beta", "c2_of", "assemble", "mass_apply", "thomas", "mono",
    "sweep", "slot_map", "apply_R", "apply_R0", "local_solution", "classical",
    "impulse_columns", "ltt_apply", "brute_L", "gmres", "bicgstab", "causal_solve",
    "interface_d", "new_algorithm", "preconditioned_time", "preconditioned_cubic",
    "adjoint_mono", "potential_of", "end_data", "sbar", "mono_ld", "pade_coef", "pade_eval",
    "pade_apply",
]

_LIB = None
_C = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double


def lib():
    """Load (building if stale) the oracle's C core."""
    global _LIB
    if _LIB is None:
        L = ctypes.CDLL(_build.build(force=False))
        L.orc_alpha.argtypes = [_I, _C]
        L.orc_beta.argtypes = [_I, _C]
        L.orc_assemble.argtypes = [_I, _D, _D, _D, _C, _C, _C]
        L.orc_mass_apply.argtypes = [_I, _D, _C, _C]
        L.orc_genmass_apply.argtypes = [_I, _D, _C, _C, _C]
        L.orc_thomas.argtypes = [_I, _C, _C, _C, _C]
        L.orc_thomas.restype = _I
        L.orc_mono_cn.argtypes = [_I, _D, _D, _I, _I, _C, _C, _C, _C, _C, _I, _D, _C]
        L.orc_mono_cn.restype = _I
        L.orc_sub_sweep.argtypes = [_I, _D, _D, _I, _I, _C, _I, _I, _I, _I, _I, _D, _D, _C,
                                    _C, _C, _C, _C, _C, _C, _C, _C, _C, _C, _I, _D, _C, _I, _D]
        L.orc_sub_sweep.restype = _I
        L.orc_mono_adjoint.argtypes = [_I, _D, _D, _I, _C, _C, _C, _C, _C]
        L.orc_mono_adjoint.restype = _I
        L.orc_end_data.argtypes = [_I, _C, _I, _I, _I, _D, _D, _I, _C, _C, _C]
        L.orc_mono_cn_ld.argtypes = [_I, _D, _D, _I, _I, _C, _C, _C, _I, _D, _C]
        L.orc_mono_cn_ld.restype = _I
        L.orc_sbar_apply.argtypes = [_I, _I, _D, _C, _C, _C, _C, _C, _C]
        L.orc_pade_coef.argtypes = [_I, _D, _C, _C]
        L.orc_pade_eval.argtypes = [_I, _D, _D, _D, _C]
        L.orc_pade_apply.argtypes = [_I, _I, _D, _I, _D, _C, _C, _C, _C, _C]
        L.orc_pade_apply.restype = _I
        _LIB = L
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(_C)


def _cvec(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if n is not None:
        assert a.shape == (n,), (a.shape, n)
    return a


# ---------------------------------------------------------------------------
# Sec. 2.2: convolution weights and the S0^2 constant
# ---------------------------------------------------------------------------

def alpha(n: int) -> np.ndarray:
    """alpha_0..alpha_{n-1} of the potential strategy (Sec. 2.2)."""
    out = np.zeros(n)
    lib().orc_alpha(n, _p(out))
    return out


def beta(n: int) -> np.ndarray:
    """beta_s = (-1)^s alpha_s (Sec. 2.2)."""
    out = np.zeros(n)
    lib().orc_beta(n, _p(out))
    return out


def c2_of(dt: float) -> complex:
    """c2 = e^{-i pi/4} sqrt(2/dt), the S0^2 prefactor (Sec. 2.2, Prop. 3)."""
    return complex(np.exp(-1j * np.pi / 4) * math.sqrt(2.0 / dt))


def end_data(wl: Workload, k: int, side: int, V=None):
    """(W_n, dn W_n, calW_n), n = 0..nt, at the left (side 0) or right
    (side 1) end of subdomain k: the potential data of the S0^3, S0^4, S1^2
    and S1^4 operators (Sec. 2.2; readings in swr_oracle.c)."""
    if V is None:
        V = potential_of(wl)
    Va = None if V is None else np.ascontiguousarray(V, np.float64)
    g = int(wl.offsets[k]) + (int(wl.J[k]) if side else 0)
    out = np.zeros((3, wl.nt + 1))
    lib().orc_end_data(wl.vkind, _p(Va), wl.nx, g, 1 if side else -1, wl.h, wl.dt, wl.nt,
                       _p(out[0]), _p(out[1]), _p(out[2]))
    return out[0].copy(), out[1].copy(), out[2].copy()


def sbar(kind: int, dt: float, v, W, dW, calW):
    """Sbar v_n, n = 0..len(v)-1, of the transmission operator `kind`
    (S02, S03, S04, S12, S14) on a given sequence v: returns (full, without
    the order-4 normal-derivative term)."""
    v = _cvec(v)
    nt = len(v) - 1
    W, dW, calW = (np.ascontiguousarray(a, np.float64) for a in (W, dW, calW))
    assert W.shape == dW.shape == calW.shape == (nt + 1,)
    out = np.zeros(nt + 1, np.complex128)
    out_s = np.zeros(nt + 1, np.complex128)
    lib().orc_sbar_apply(kind, nt, dt, _p(v), _p(W), _p(dW), _p(calW), _p(out), _p(out_s))
    return out, out_s


# ---------------------------------------------------------------------------
# P1 matrices and the tridiagonal solver (Sec. 2.2, eq. AvML)
# ---------------------------------------------------------------------------

def assemble(n: int, h: float, coef_m: complex, W=None):
    """Tridiagonal (diag, off) of coef_m*M - S + M_W on n nodes."""
    diag = np.zeros(n, np.complex128)
    off = np.zeros(max(n - 1, 1), np.complex128)
    Wa = None if W is None else np.ascontiguousarray(W, np.float64)
    lib().orc_assemble(n, h, complex(coef_m).real, complex(coef_m).imag, _p(Wa), _p(diag), _p(off))
    return diag, off[: n - 1]


def mass_apply(h: float, x) -> np.ndarray:
    x = _cvec(x)
    y = np.zeros_like(x)
    lib().orc_mass_apply(len(x), h, _p(x), _p(y))
    return y


def thomas(diag, off, rhs) -> np.ndarray:
    diag = _cvec(diag)
    n = len(diag)
    off = _cvec(off if n > 1 else np.zeros(1))
    rhs = _cvec(rhs, n)
    x = np.zeros(n, np.complex128)
    rc = lib().orc_thomas(n, _p(diag), _p(off), _p(rhs), _p(x))
    if rc:
        raise RuntimeError(f"thomas failed rc={rc}")
    return x


def potential_of(wl: Workload, b: int = 0):
    """The potential array of problem b (per-problem static V is [B][nx])."""
    if wl.V is None:
        return None
    if wl.vkind == V_STATIC and wl.V.ndim == 2:
        return np.ascontiguousarray(wl.V[b], np.float64)
    return np.ascontiguousarray(wl.V, np.float64)


# ---------------------------------------------------------------------------
# Monodomain reference: the plain definition SWR converges to
# ---------------------------------------------------------------------------

def mono(wl: Workload, u0, V=None, want_u=False, want_v=False, nl_maxit=100, nl_tol=1e-14):
    """Monodomain CN + P1 with Neumann walls (eq. Schequ, eq. CNS_L /
    eq. CNS_NL).  Returns uT, or (uT, u_all, v_all) when asked."""
    nx, nt = wl.nx, wl.nt
    u0 = _cvec(u0, nx)
    if V is None:
        V = potential_of(wl)
    Va = None if V is None else np.ascontiguousarray(V, np.float64)
    uT = np.zeros(nx, np.complex128)
    u_all = np.zeros((nt + 1, nx), np.complex128) if want_u else None
    v_all = np.zeros((nt, nx), np.complex128) if want_v else None
    worst = ctypes.c_int(0)
    rc = lib().orc_mono_cn(nx, wl.h, wl.dt, nt, wl.vkind, _p(Va), _p(u0), _p(uT), _p(u_all),
                           _p(v_all), nl_maxit, nl_tol, ctypes.byref(worst))
    if rc:
        raise RuntimeError(f"mono_cn failed rc={rc}")
    if want_u or want_v:
        return uT, u_all, v_all
    return uT


def mono_ld(wl: Workload, u0, V=None, nl_maxit=100, nl_tol=1e-17):
    """``mono`` computed in extended precision (80-bit long double, unit
    roundoff 5.4e-20), FP64 in and out: the monodomain reference on grids
    where one FP64 sweep over the whole domain loses accuracy (dt/h^2 large).
    The |u|^2 inner fixed point defaults to a tolerance of 1e-17."""
    nx, nt = wl.nx, wl.nt
    u0 = _cvec(u0, nx)
    if V is None:
        V = potential_of(wl)
    Va = None if V is None else np.ascontiguousarray(V, np.float64)
    uT = np.zeros(nx, np.complex128)
    worst = ctypes.c_int(0)
    rc = lib().orc_mono_cn_ld(nx, wl.h, wl.dt, nt, wl.vkind, _p(Va), _p(u0), _p(uT), nl_maxit,
                              nl_tol, ctypes.byref(worst))
    if rc:
        raise RuntimeError(f"mono_cn_ld failed rc={rc}")
    return uT


def pade_coef(m: int, theta: float):
    """(a[0..m], d[0..m]) of the Pade strategy: sqrt(z) ~ sum_s a_s -
    sum_{s>=1} a_s d_s / (z + d_s) (Sec. 2.2; reading in swr_oracle.c)."""
    a = np.zeros(m + 1, np.complex128)
    d = np.zeros(m + 1, np.complex128)
    lib().orc_pade_coef(m, theta, _p(a), _p(d))
    return a, d


def pade_eval(m: int, theta: float, z: complex) -> complex:
    """The rational approximation of sqrt(z) above at one point."""
    out = np.zeros(2)
    lib().orc_pade_eval(m, theta, float(np.real(z)), float(np.imag(z)), _p(out))
    return complex(out[0], out[1])


def pade_apply(order: int, m: int, theta: float, dt: float, v, W, dW):
    """Sbar v_n, n = 1..nt, of S2^{order,m} on a given sequence v (index 0 is
    returned as 0): returns (full, without the order-4 term)."""
    v = _cvec(v)
    nt = len(v) - 1
    W, dW = (np.ascontiguousarray(np.broadcast_to(x, (nt + 1,)), np.float64) for x in (W, dW))
    out = np.zeros(nt + 1, np.complex128)
    out_s = np.zeros(nt + 1, np.complex128)
    rc = lib().orc_pade_apply(order, m, theta, nt, dt, _p(v), _p(W), _p(dW), _p(out), _p(out_s))
    if rc:
        raise ValueError(f"pade_apply rc={rc}")
    return out, out_s


# ---------------------------------------------------------------------------
# One subdomain over the whole window (eq. AvML / AvMNL, eq. TransmissionCond_disc)
# ---------------------------------------------------------------------------

def sweep(wl: Workload, k: int, u0=None, l=None, r=None, hist0=None, V=None,
          want_v=False, nl_maxit=100, nl_tol=1e-14):
    """Solve subdomain k over all nt steps with incoming fluxes l, r
    (length nt, n = 1..nt; None = 0).  u0: global initial data (None = zero
    data).  hist0: the value used for v_0 at (left, right) end in the S0^2
    history (None = the initial data there, as in the paper)."""
    N, nt = wl.N, wl.nt
    o = int(wl.offsets[k])
    n = int(wl.J[k]) + 1
    if V is None:
        V = potential_of(wl)
    Va = None if V is None else np.ascontiguousarray(V, np.float64)
    u0l = None if u0 is None else _cvec(np.asarray(u0)[o:o + n])
    h0 = None if hist0 is None else _cvec(hist0, 2)
    la = None if l is None else _cvec(l, nt)
    ra = None if r is None else _cvec(r, nt)
    out = dict(rhoL=np.zeros(nt, np.complex128), rhoR=np.zeros(nt, np.complex128),
               uT=np.zeros(n, np.complex128), va=np.zeros(nt + 1, np.complex128),
               vb=np.zeros(nt + 1, np.complex128))
    out["v_all"] = np.zeros((nt, n), np.complex128) if want_v else None
    bt = beta(nt + 1)
    worst = ctypes.c_int(0)
    rc = lib().orc_sub_sweep(n, wl.h, wl.dt, nt, wl.vkind, _p(Va), wl.nx, o,
                             int(k > 0), int(k < N - 1), wl.trans,
                             wl.sigma.real, wl.sigma.imag, _p(bt), _p(u0l), _p(h0),
                             _p(la), _p(ra), _p(out["rhoL"]), _p(out["rhoR"]), _p(out["uT"]),
                             _p(out["va"]), _p(out["vb"]), _p(out["v_all"]),
                             nl_maxit, nl_tol, ctypes.byref(worst), int(wl.pade_m),
                             float(wl.pade_theta))
    if rc:
        raise RuntimeError(f"sub_sweep failed rc={rc}")
    out["nl_worst"] = worst.value
    return out


def slot_map(N: int, k: int):
    """(slot of l_k, slot of r_k, slot written by rhoL, slot written by rhoR);
    None where the end is a wall (Sec. 3, vector g)."""
    return (2 * k - 1 if k >= 1 else None, 2 * k if k <= N - 2 else None,
            2 * k - 2 if k >= 1 else None, 2 * k + 1 if k <= N - 2 else None)


def apply_R(wl: Workload, u0, g, V=None, hist0_zero=False, **kw):
    """One SWR iteration g -> R g (Sec. 3 eq. interfacepbR; exchange of
    eq. TransmisionCond).  u0 None = zero data (then R is linear: R = L)."""
    N, nt = wl.N, wl.nt
    g = np.asarray(g, np.complex128).reshape(max(2 * N - 2, 0), nt)
    gn = np.zeros_like(g)
    for k in range(N):
        sl, sr, ol, orr = slot_map(N, k)
        res = sweep(wl, k, u0, None if sl is None else g[sl], None if sr is None else g[sr],
                    hist0=np.zeros(2) if hist0_zero else None, V=V, **kw)
        if ol is not None:
            gn[ol] = res["rhoL"]
        if orr is not None:
            gn[orr] = res["rhoR"]
    return gn


def apply_R0(wl: Workload, x, V=None):
    """L x = R(x) - R(0) evaluated directly with zero data and zero v_0
    history (Prop. 1 linearity)."""
    return apply_R(wl, None, x, V=V, hist0_zero=True)


def local_solution(wl: Workload, u0, g, V=None):
    """Final sweep (Sec. 4 "New algorithm", step 3): solve every subdomain
    with the interface fluxes g and assemble u(T) on the global mesh; a node
    shared by two subdomains takes the average of the two values.  Also
    returns the outgoing fluxes R(g)."""
    N, nt = wl.N, wl.nt
    g = np.asarray(g, np.complex128).reshape(max(2 * N - 2, 0), nt)
    uT = np.zeros(wl.nx, np.complex128)
    cnt = np.zeros(wl.nx)
    Rg = np.zeros_like(g)
    for k in range(N):
        sl, sr, ol, orr = slot_map(N, k)
        res = sweep(wl, k, u0, None if sl is None else g[sl], None if sr is None else g[sr], V=V)
        o = int(wl.offsets[k])
        n = int(wl.J[k]) + 1
        uT[o:o + n] += res["uT"]
        cnt[o:o + n] += 1
        if ol is not None:
            Rg[ol] = res["rhoL"]
        if orr is not None:
            Rg[orr] = res["rhoR"]
    return uT / cnt, Rg


def classical(wl: Workload, u0, tol=1e-10, maxit=10000, g0=None, V=None):
    """Classical algorithm (Sec. 4): g^{k+1} = R g^k until
    max |g^{k+1} - g^k| < tol.  Returns (g, iterations, history)."""
    N, nt = wl.N, wl.nt
    g = np.zeros((max(2 * N - 2, 0), nt), np.complex128) if g0 is None else np.array(g0, np.complex128)
    hist = []
    for it in range(1, maxit + 1):
        gn = apply_R(wl, u0, g, V=V)
        ch = float(np.max(np.abs(gn - g))) if g.size else 0.0
        hist.append(ch)
        g = gn
        if ch < tol:
            return g, it, hist
    return g, -maxit, hist


# ---------------------------------------------------------------------------
# Sec. 4.1: explicit interface problem for time-independent V
# ---------------------------------------------------------------------------

def interface_d(wl: Workload, u0, V=None):
    """d = R . 0 (Sec. 4.1): one sweep per subdomain with zero fluxes."""
    N, nt = wl.N, wl.nt
    return apply_R(wl, u0, np.zeros((max(2 * N - 2, 0), nt)), V=V)


def impulse_columns(wl: Workload, V=None):
    """First columns of X^{k,1..4} (Sec. 4.1), returned as cols[N, 4, nt]:
    p = 0..3 <-> X^{k,1}, X^{k,2}, X^{k,3}, X^{k,4}.  Impulse l_{k,1} = 1
    gives X^{k,1} (rhoL) and X^{k,3} (rhoR); r_{k,1} = 1 gives X^{k,2} and
    X^{k,4}.  Computed with zero initial data and zero v_0 history, which
    yields "impulse response minus d" of the paper directly (Prop. 1)."""
    N, nt = wl.N, wl.nt
    cols = np.zeros((N, 4, nt), np.complex128)
    e1 = np.zeros(nt, np.complex128)
    e1[0] = 1.0
    for k in range(N):
        if k >= 1:
            res = sweep(wl, k, None, e1, None, hist0=np.zeros(2), V=V)
            cols[k, 0] = res["rhoL"]
            if k <= N - 2:
                cols[k, 2] = res["rhoR"]
        if k <= N - 2:
            res = sweep(wl, k, None, None, e1, hist0=np.zeros(2), V=V)
            if k >= 1:
                cols[k, 1] = res["rhoL"]
            cols[k, 3] = res["rhoR"]
    return cols


def _causal_conv(c, x):
    """y_n = sum_{s=0}^{n} c_{n-s} x_s: product of the lower-triangular
    Toeplitz matrix with first column c and the vector x."""
    nt = len(x)
    return np.convolve(c, x)[:nt]


def ltt_apply(wl: Workload, cols, g):
    """L g with every block lower-triangular Toeplitz (Props. 3-4, block
    layout eq. chp1_L_N)."""
    N, nt = wl.N, wl.nt
    g = np.asarray(g, np.complex128).reshape(max(2 * N - 2, 0), nt)
    y = np.zeros_like(g)
    for k in range(N):
        sl, sr, ol, orr = slot_map(N, k)
        if ol is not None:
            acc = np.zeros(nt, np.complex128)
            if sl is not None:
                acc += _causal_conv(cols[k, 0], g[sl])
            if sr is not None:
                acc += _causal_conv(cols[k, 1], g[sr])
            y[ol] = acc
        if orr is not None:
            acc = np.zeros(nt, np.complex128)
            if sl is not None:
                acc += _causal_conv(cols[k, 2], g[sl])
            if sr is not None:
                acc += _causal_conv(cols[k, 3], g[sr])
            y[orr] = acc
    return y


def brute_L(wl: Workload, V=None):
    """Dense L built column by column as R(e_i) - R(0) with zero data
    (Props. 1-2).  Size ((2N-2) nt)^2: tiny cases only."""
    N, nt = wl.N, wl.nt
    m = (2 * N - 2) * nt
    Lm = np.zeros((m, m), np.complex128)
    for i in range(m):
        e = np.zeros(m, np.complex128)
        e[i] = 1.0
        Lm[:, i] = apply_R0(wl, e.reshape(2 * N - 2, nt), V=V).ravel()
    return Lm


def gmres(matvec, b, x0=None, tol=1e-10, restart=30, maxit=5000):
    """Restarted GMRES(m) with modified Gram-Schmidt and Givens rotations
    (Saad, Iterative Methods for Sparse Linear Systems, Alg. 6.9/6.11), the
    Krylov method named in Sec. 4.  Stops on the relative residual
    ||b - A x||_2 <= tol ||b||_2 (recomputed at every restart).
    Returns (x, iterations, residual history)."""
    b = np.asarray(b, np.complex128).ravel()
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.complex128).ravel()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, [0.0]
    hist, its = [], 0
    while its < maxit:
        r = b - matvec(x)
        beta_ = np.linalg.norm(r)
        hist.append(beta_ / bn)
        if beta_ <= tol * bn:
            return x, its, hist
        m = restart
        Vb = np.zeros((m + 1, b.size), np.complex128)
        H = np.zeros((m + 1, m), np.complex128)
        cs = np.zeros(m, np.complex128)
        sn = np.zeros(m, np.complex128)
        e = np.zeros(m + 1, np.complex128)
        e[0] = beta_
        Vb[0] = r / beta_
        j_used = 0
        for j in range(m):
            w = matvec(Vb[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(Vb[i], w)
                w = w - H[i, j] * Vb[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                Vb[j + 1] = w / H[j + 1, j]
            # earlier rotations G_i = [[conj(c), conj(s)], [-s, c]], the same
            # unitary map that zeroed column i's subdiagonal and updated e
            for i in range(j):
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(abs(H[j, j]), abs(H[j + 1, j]))
            cs[j] = H[j, j] / den if den else 1.0
            sn[j] = H[j + 1, j] / den if den else 0.0
            H[j, j] = np.conj(cs[j]) * H[j, j] + np.conj(sn[j]) * H[j + 1, j]
            H[j + 1, j] = 0
            e[j + 1] = -sn[j] * e[j]
            e[j] = np.conj(cs[j]) * e[j]
            j_used = j + 1
            its += 1
            hist.append(abs(e[j + 1]) / bn)
            if abs(e[j + 1]) <= tol * bn or its >= maxit or H[j, j] == 0:
                break
        y = np.linalg.solve(np.triu(H[:j_used, :j_used]), e[:j_used])
        x = x + Vb[:j_used].T @ y
    r = b - matvec(x)
    return x, -its if np.linalg.norm(r) > tol * bn else its, hist


def bicgstab(matvec, b, x0=None, tol=1e-10, maxit=5000):
    """BiCGStab (van der Vorst, SIAM J. Sci. Stat. Comput. 13, 1992), the
    Krylov method of the paper's GPU runs (Sec. 6), unpreconditioned, for
    complex systems with the shadow residual r^_0 = r_0 and <u, w> =
    conj(u)^T w.  Stops when ||r||_2 <= tol ||b||_2 (checked on s after the
    half step and on r after the full step).  Returns (x, iterations,
    residual history); iterations are negative when maxit was reached."""
    b = np.asarray(b, np.complex128).ravel()
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.complex128).ravel()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, [0.0]
    r = b - matvec(x)
    rh = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    hist = [np.linalg.norm(r) / bn]
    if hist[0] <= tol:
        return x, 0, hist
    for it in range(1, maxit + 1):
        rho_new = np.vdot(rh, r)
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = matvec(p)
        alpha = rho_new / np.vdot(rh, v)
        s = r - alpha * v
        if np.linalg.norm(s) <= tol * bn:
            x = x + alpha * p
            hist.append(np.linalg.norm(s) / bn)
            return x, it, hist
        t = matvec(s)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        hist.append(np.linalg.norm(r) / bn)
        if hist[-1] <= tol:
            return x, it, hist
        rho = rho_new
    return x, -maxit, hist


def causal_solve(wl: Workload, cols, d):
    """Solve (I - L) g = d exactly for block lower-triangular-Toeplitz L by
    forward substitution in time.  With C_m the (2N-2)x(2N-2) matrix of the
    m-th Toeplitz coefficients of all blocks, time step n reads
    (I - C_0) g_n = d_n + sum_{s<n} C_{n-s} g_s  (Props. 3-4 make every
    block lower triangular in time)."""
    N, nt = wl.N, wl.nt
    ns = 2 * N - 2
    d = np.asarray(d, np.complex128).reshape(ns, nt)
    if ns == 0:
        return d.copy()
    # blocks: (out slot, in slot, column)
    blocks = []
    for k in range(N):
        sl, sr, ol, orr = slot_map(N, k)
        for out, p_l, p_r in ((ol, 0, 1), (orr, 2, 3)):
            if out is None:
                continue
            if sl is not None:
                blocks.append((out, sl, cols[k, p_l]))
            if sr is not None:
                blocks.append((out, sr, cols[k, p_r]))
    C0 = np.zeros((ns, ns), np.complex128)
    for out, inn, c in blocks:
        C0[out, inn] += c[0]
    Mat = np.eye(ns) - C0
    # (I - C_0) is the same at every step: one LU factorisation with partial
    # pivoting (what a dense solve does), then one triangular pair per step
    lu = scipy.linalg.lu_factor(Mat)
    g = np.zeros((ns, nt), np.complex128)
    for n in range(nt):
        rhs = d[:, n].copy()
        if n > 0:
            for out, inn, c in blocks:
                # sum_{s<n} c_{n-s} g_s
                rhs[out] += np.dot(c[n:0:-1], g[inn, :n])
        g[:, n] = scipy.linalg.lu_solve(lu, rhs)
    return g


def new_algorithm(wl: Workload, u0, solver="gmres", tol=1e-10, restart=30, maxit=5000, V=None):
    """Sec. 4 "New algorithm": (1) build L (impulse first columns) and d;
    (2) solve (I - L) g = d; (3) final sweep.  Returns (uT, g, info)."""
    cols = impulse_columns(wl, V=V)
    d = interface_d(wl, u0, V=V)
    ns = d.shape[0]
    if ns == 0:
        g = d
        its = 0
    elif solver == "causal":
        g = causal_solve(wl, cols, d)
        its = 1
    elif solver == "fixed":
        g = np.zeros_like(d)
        its = 0
        while True:
            gn = ltt_apply(wl, cols, g) + d
            its += 1
            ch = np.max(np.abs(gn - g))
            g = gn
            if ch < tol or its >= maxit:
                break
    elif solver == "bicgstab":
        mv = lambda x: x - ltt_apply(wl, cols, x.reshape(ns, -1)).ravel()  # noqa: E731
        gv, its, _ = bicgstab(mv, d.ravel(), tol=tol, maxit=maxit)
        g = gv.reshape(d.shape)
    else:
        mv = lambda x: x - ltt_apply(wl, cols, x.reshape(ns, -1)).ravel()  # noqa: E731
        gv, its, _ = gmres(mv, d.ravel(), tol=tol, restart=restart, maxit=maxit)
        g = gv.reshape(d.shape)
    uT, Rg = local_solution(wl, u0, g, V=V)
    res = np.linalg.norm(g - Rg) / max(np.linalg.norm(d), 1e-300)
    return uT, g, dict(iters=its, residual=res, cols=cols, d=d)


# ---------------------------------------------------------------------------
# Sec. 5: preconditioned algorithm, P = I - L_0
# ---------------------------------------------------------------------------

def _zero_potential(wl: Workload) -> Workload:
    import copy
    w0 = copy.copy(wl)
    w0.vkind = V_STATIC
    w0.V = np.zeros(wl.nx)
    return w0


def preconditioned_time(wl: Workload, u0, tol=1e-10, restart=30, maxit=2000, precond=True):
    """V(t,x): GMRES on (I - L) g = d with L x = R(x) - R(0) applied
    matrix-free by one full sweep (Sec. 4 "Classical algorithm, version 2"),
    right-preconditioned by P = I - L_0 (Sec. 5, eq. chp2_algopd_Lpf, P^{-1}
    applied exactly by ``causal_solve``).  Returns (uT, g, info)."""
    ns = 2 * wl.N - 2
    d = interface_d(wl, u0)
    cols0 = impulse_columns(_zero_potential(wl)) if precond else None
    Pinv = (lambda y: causal_solve(wl, cols0, y.reshape(ns, -1)).ravel()) if precond else (lambda y: y)
    A = lambda x: x - apply_R0(wl, x.reshape(ns, -1)).ravel()  # noqa: E731
    y, its, hist = gmres(lambda z: A(Pinv(z)), d.ravel(), tol=tol, restart=restart, maxit=maxit)
    g = Pinv(y).reshape(ns, -1)
    uT, Rg = local_solution(wl, u0, g)
    res = np.linalg.norm(g - Rg) / max(np.linalg.norm(d), 1e-300)
    return uT, g, dict(iters=its, residual=res, history=hist)


def preconditioned_cubic(wl: Workload, u0, tol=1e-10, maxit=2000, precond=True, g0=None):
    """|u|^2: preconditioned fixed point g^{k+1} = g^k - P^{-1}(g^k - R_nl g^k)
    (Sec. 5, eq. chp2_algopd_NL read as in the text around it), P = I - L_0
    applied exactly by ``causal_solve``; stops when max |g^{k+1}-g^k| < tol.
    Returns (uT, g, info)."""
    ns = 2 * wl.N - 2
    g = np.zeros((ns, wl.nt), np.complex128) if g0 is None else np.array(g0, np.complex128)
    cols0 = impulse_columns(_zero_potential(wl)) if precond else None
    hist = []
    its = 0
    while its < maxit:
        Rg = apply_R(wl, u0, g)
        y = g - Rg
        z = causal_solve(wl, cols0, y) if precond else y
        gn = g - z
        its += 1
        ch = float(np.max(np.abs(gn - g))) if g.size else 0.0
        hist.append(ch)
        g = gn
        if ch < tol:
            break
    uT, Rg = local_solution(wl, u0, g)
    return uT, g, dict(iters=its if its < maxit else -its, history=hist,
                       residual=float(np.max(np.abs(g - Rg))) if g.size else 0.0)


# ---------------------------------------------------------------------------
# Discrete adjoint (monodomain), for dJ/dV and dJ/du0
# ---------------------------------------------------------------------------

def adjoint_mono(wl: Workload, u0, gbar, V=None):
    """Gradient of a real objective J(u_nt) through the monodomain CN map
    with static real V: returns (dJ/dV [nx] real, dJ/du0 [nx] complex), both
    in the convention grad = dJ/dRe + i dJ/dIm for complex inputs."""
    if V is None:
        V = potential_of(wl)
    V = np.ascontiguousarray(V, np.float64)
    nx, nt = wl.nx, wl.nt
    _, _, v_all = mono(wl, u0, V=V, want_v=True)
    gb = _cvec(gbar, nx)
    dV = np.zeros(nx)
    du0 = np.zeros(nx, np.complex128)
    rc = lib().orc_mono_adjoint(nx, wl.h, wl.dt, nt, _p(V), _p(v_all), _p(gb), _p(dV), _p(du0))
    if rc:
        raise RuntimeError(f"mono_adjoint failed rc={rc}")
    return dV, du0
