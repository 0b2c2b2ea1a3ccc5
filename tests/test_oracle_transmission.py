"""Pins of the oracle's higher-order transmission operators (Sec. 2.2,
"Potential strategy" orders 2-4 and "Gauge change strategy" orders 2, 4).

The operators are pinned to facts fixed by the mathematics, not to their own
formulas:
* the continuous operators they discretise (half-order derivative and
  integral, integral) on t^2, to second order in dt;
* exact identities of the discrete convolution weights: the half integral
  applied twice is the integral (alpha * alpha = gamma), and the half
  derivative inverts the half integral (beta * alpha = delta);
* gauge covariance: for a static potential the gauge operators are the
  potential-strategy operators conjugated by e^{i calW_n};
* the normal derivative and gauge phase of the potential against closed forms;
* the converged SWR solution equals the monodomain solution for every
  operator (the exchange cancels the order-4 terms, which flip sign with the
  normal), for static and time-dependent potentials, and for the order-2 and
  order-3 operators with |u|^2.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1503_02564_amd import workloads as W

KINDS = [W.S02, W.S03, W.S04, W.S12, W.S14]
E_M = np.exp(-1j * np.pi / 4)
E_P = np.exp(1j * np.pi / 4)


def _ops(dt, v, w=0.0, dw=0.0, calw=None):
    n = len(v)
    Wn, dWn = np.full(n, w), np.full(n, dw)
    cW = np.zeros(n) if calw is None else calw
    return {k: O.sbar(k, dt, v, Wn, dWn, cW) for k in KINDS}


def test_operators_approach_the_continuous_ones_on_t_squared():
    """On h(t) = t^2 (h(0) = 0): S0^2 -> e^{-i pi/4} d^{1/2} h = e^{-i pi/4}
    2 t^{3/2}/Gamma(5/2); (S0^3 - S0^2) -> -e^{i pi/4}(W/2) I^{1/2} h with
    I^{1/2} t^2 = 2 t^{5/2}/Gamma(7/2); (S0^4 - S0^3) -> -i (dW/4) I h with
    I t^2 = t^3/3.  Errors at t = 1 fall like dt^2 (ratio ~4 per halving)."""
    w, dw = 1.7, -0.9
    errs = {k: [] for k in ("d12", "i12", "i1")}
    for nt in (40, 80, 160):
        dt = 1.0 / nt
        t = dt * np.arange(nt + 1)
        ops = _ops(dt, t * t + 0j, w, dw)
        d12 = ops[W.S02][0][-1]
        i12 = (ops[W.S03][0][-1] - ops[W.S02][0][-1]) / (-E_P * w / 2)
        i1 = (ops[W.S04][0][-1] - ops[W.S03][0][-1]) / (-1j * dw / 4)
        errs["d12"].append(abs(d12 - E_M * 2.0 / math.gamma(2.5)))
        errs["i12"].append(abs(i12 - 2.0 / math.gamma(3.5)))
        errs["i1"].append(abs(i1 - 1.0 / 3.0))
    for key, e in errs.items():
        assert e[-1] < 5e-4, (key, e)
        assert e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5, (key, e)


def test_half_integral_twice_is_the_integral_and_half_derivative_inverts_it():
    """alpha * alpha = gamma and beta * alpha = delta (generating functions
    ((1+z)/(1-z))^{1/2} squared and times ((1-z)/(1+z))^{1/2}): with K3 the
    order-3 term divided by its prefactor and K4 the order-4 term divided by
    its prefactor, K3 K3 v = K4 v and S0^2 K3 v = e^{-i pi/4} v exactly."""
    rng = np.random.default_rng(11)
    nt, dt, w, dw = 50, 0.013, 2.3, 0.7
    v = rng.standard_normal(nt + 1) + 1j * rng.standard_normal(nt + 1)
    ops = _ops(dt, v, w, dw)
    K3 = lambda x: (O.sbar(W.S03, dt, x, *_flat(nt, w, dw))[0]  # noqa: E731
                    - O.sbar(W.S02, dt, x, *_flat(nt, w, dw))[0]) / (-E_P * w / 2)
    k3v = K3(v)
    k4v = (ops[W.S04][0] - ops[W.S03][0]) / (-1j * dw / 4)
    assert np.max(abs(K3(k3v) - k4v)) < 1e-12 * np.max(abs(k4v))
    back = O.sbar(W.S02, dt, k3v, *_flat(nt, w, dw))[0] / E_M
    assert np.max(abs(back - v)) < 1e-12 * np.max(abs(v))


def _flat(nt, w, dw):
    return np.full(nt + 1, w), np.full(nt + 1, dw), np.zeros(nt + 1)


def test_gauge_operators_conjugate_the_potential_operators():
    """Static W: calW_n = (n - 1/2) dt W (calW_0 = 0), and for any x,
    S1^2[e^{i calW} x] = e^{i calW} S0^2[x] and
    (S1^4 - S1^2)[e^{i calW} x] = e^{i calW} (S0^4 - S0^3)[x]."""
    rng = np.random.default_rng(12)
    nt, dt, w, dw = 45, 0.02, -3.1, 1.3
    x = rng.standard_normal(nt + 1) + 1j * rng.standard_normal(nt + 1)
    calw = dt * w * (np.arange(nt + 1) - 0.5)
    calw[0] = 0.0
    ph = np.exp(1j * calw)
    Wn, dWn = np.full(nt + 1, w), np.full(nt + 1, dw)
    s12 = O.sbar(W.S12, dt, ph * x, Wn, dWn, calw)[0]
    s14 = O.sbar(W.S14, dt, ph * x, Wn, dWn, calw)[0]
    z = np.zeros(nt + 1)
    s02 = O.sbar(W.S02, dt, x, Wn, dWn, z)[0]
    s03 = O.sbar(W.S03, dt, x, Wn, dWn, z)[0]
    s04 = O.sbar(W.S04, dt, x, Wn, dWn, z)[0]
    assert np.max(abs(s12 - ph * s02)) < 1e-12 * np.max(abs(s02))
    assert np.max(abs((s14 - s12) - ph * (s04 - s03))) < 1e-12 * np.max(abs(s04 - s03))
    # the parts that cross the interface drop exactly the order-4 term
    assert np.array_equal(O.sbar(W.S14, dt, ph * x, Wn, dWn, calw)[1], s12)
    assert np.array_equal(O.sbar(W.S04, dt, x, Wn, dWn, z)[1], s03)


def test_potential_data_at_the_interfaces():
    """Linear static V = a x + b: dn W = -a at left ends, +a at right ends
    (the centred difference is exact); calW_n = (n - 1/2) dt V(x_e).
    V(t, x) = 5 x cos t: calW_n is the midpoint of calV = 5 x sin t at
    t_n, t_{n-1} up to the trapezoid error, O(dt^2)."""
    wl = W.small_case(N=3, nt=30, cells=8)
    x = wl.x()
    wl.V = 0.8 * x - 0.3
    for k, side in ((0, 1), (1, 0), (1, 1), (2, 0)):
        Wn, dWn, cW = O.end_data(wl, k, side)
        xe = x[int(wl.offsets[k]) + (int(wl.J[k]) if side else 0)]
        assert np.allclose(Wn, 0.8 * xe - 0.3, rtol=0, atol=1e-15)
        assert np.allclose(dWn, 0.8 if side else -0.8, rtol=0, atol=1e-12)
        ref = wl.dt * (np.arange(wl.nt + 1) - 0.5) * (0.8 * xe - 0.3)
        ref[0] = 0.0
        assert np.allclose(cW, ref, rtol=0, atol=1e-14)
    for nt in (30, 60):
        wt = W.small_case(N=3, nt=nt, cells=8, vkind=W.V_TIME)
        t = wt.dt * np.arange(nt + 1)
        g = int(wt.offsets[1])
        xe = wt.x()[g]
        Wn, dWn, cW = O.end_data(wt, 1, 0)
        calV = 5.0 * xe * np.sin(t)
        ref = np.concatenate([[0.0], 0.5 * (calV[1:] + calV[:-1])])
        assert np.max(abs(cW - ref)) < 5.0 * abs(xe) * wt.dt ** 2 * t[-1]
        assert np.allclose(dWn, -5.0 * 0.5 * (np.cos(t) + np.cos(np.concatenate([[0.0], t[:-1]]))),
                           rtol=0, atol=1e-12)


@pytest.mark.parametrize("vkind", [W.V_STATIC, W.V_TIME])
@pytest.mark.parametrize("trans", [W.S03, W.S04, W.S12, W.S14])
def test_classical_swr_converges_to_the_monodomain_solution(trans, vkind):
    """Every operator is a consistent transmission: the fixed point of the
    classical algorithm is the monodomain CN solution (Sec. 3), and with a
    static potential the interface problem is still block lower-triangular
    Toeplitz, so the new algorithm gives the same u(T)."""
    wl = W.small_case(N=3, nt=24, vkind=vkind, trans=trans, cells=8, seed=9)
    um = O.mono(wl, wl.u0[0])
    g, it, _ = O.classical(wl, wl.u0[0], tol=1e-12, maxit=400)
    assert it > 0
    uT, _ = O.local_solution(wl, wl.u0[0], g)
    assert np.max(abs(uT - um)) < 1e-11 * np.max(abs(um))
    if vkind == W.V_STATIC:
        u2 = O.new_algorithm(wl, wl.u0[0], solver="gmres", tol=1e-13)[0]
        assert np.max(abs(u2 - um)) < 1e-11 * np.max(abs(um))
        # Toeplitz: the impulse columns reproduce L applied by brute force
        Lb = O.brute_L(wl)
        cols = O.impulse_columns(wl)
        rng = np.random.default_rng(4)
        x = rng.standard_normal(Lb.shape[1]) + 1j * rng.standard_normal(Lb.shape[1])
        assert np.max(abs(O.ltt_apply(wl, cols, x).ravel() - Lb @ x)) < 1e-12 * np.max(abs(Lb @ x))


@pytest.mark.parametrize("trans", [W.S04, W.S14, W.P24])
def test_order_four_operators_with_the_cubic_potential_are_refused(trans):
    """The paper finds no discretisation of dn f(u) in the order-4 operators
    that keeps the interfaces continuous (Sec. 6): the oracle refuses them."""
    wl = W.small_case(N=2, nt=6, vkind=W.V_CUBIC, trans=trans, cells=6)
    with pytest.raises(RuntimeError):
        O.sweep(wl, 0, wl.u0[0])


@pytest.mark.parametrize("trans", [W.S03, W.S12, W.P22])
def test_order_two_and_three_operators_with_the_cubic_potential(trans):
    """With f(u) = |u|^2 the operators that carry W_n take it at the end node
    from the start of the step's inner fixed point, W_n = |v_{n-1}|^2: both
    sides of an interface see the same value once the iteration has
    converged, so the classical fixed point reaches the monodomain solution;
    and W_n really enters (the result differs from S0^2's iterates)."""
    wl = W.small_case(N=3, nt=24, vkind=W.V_CUBIC, trans=trans, cells=8, seed=9)
    wl.pade_m = 8
    u0 = 1.5 * wl.u0[0]
    um = O.mono(wl, u0)
    g, it, _ = O.classical(wl, u0, tol=1e-12, maxit=600)
    assert it > 0
    uT, _ = O.local_solution(wl, u0, g)
    assert np.max(abs(uT - um)) < 1e-11 * np.max(abs(um))
    # the first iterate from g = 0 differs from that of S0^2 (W_n is used)
    w2 = W.small_case(N=3, nt=24, vkind=W.V_CUBIC, trans=W.S02, cells=8, seed=9)
    z = np.zeros((2 * wl.N - 2, wl.nt), np.complex128)
    assert np.max(abs(O.apply_R(wl, u0, z) - O.apply_R(w2, u0, z))) > 1e-6
