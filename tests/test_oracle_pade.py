"""Pins of the oracle's Pade transmission operators S2^{2,m}, S2^{4,m}
(Sec. 2.1 "Pade approximation strategy", Sec. 2.2 discrete operators with
the auxiliary functions phi^s and psi).

The paper uses the coefficients a_s^m, d_s^m without stating them; the
oracle reads them as the partial fractions of the diagonal Pade approximant
of sqrt(1 + w) with the branch cut rotated by theta (swr_oracle.c).  Pinned to
facts fixed by the mathematics, not to the oracle's formulas:
* m = 1 by hand: the [1/1] approximant (4 + 3w)/(4 + w);
* every m: the closed form of the approximant,
  sqrt(1+w) (1 + rho^N)/(1 - rho^N), rho = (1 - q)/(1 + q), q = sqrt(1+w),
  N = 2m + 1, which never forms a partial fraction, and its exact relative
  error 2 rho^N / (1 - rho^N) against the square root;
* the discrete operator on a geometric sequence v_n = zeta^n (|zeta| > 1):
  once the start-up transient has decayed, Sbar v_n / v_n is the symbol
  -i R(z_d + W) (+ (dW/4)/(z_d + W) at order 4) with z_d = (2i/dt)
  (zeta - 1)/(zeta + 1), the Crank-Nicolson symbol of i d_t -- this checks
  the coefficients, the auxiliary recursions and the assembly of Sbar
  together against the closed form;
* W = 0: as m grows the Pade operator tends to the potential strategy's
  S0^2 (both discretise -i sqrt(i d_t) with the same CN symbol);
* the converged SWR solution is the monodomain solution (consistency), for
  both orders and static and time-dependent potentials.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1503_02564_amd import workloads as W

THETA = np.pi / 4


def _closed(m, z, theta=THETA):
    """e^{i theta/2} R_m(e^{-i theta} z - 1) from the closed form."""
    q = np.sqrt(np.exp(-1j * theta) * z + 0j)
    rho = (1 - q) / (1 + q)
    N = 2 * m + 1
    return np.exp(1j * theta / 2) * q * (1 + rho ** N) / (1 - rho ** N)


def test_first_order_approximant_by_hand():
    """m = 1, theta = 0: R_1(w) = (4 + 3w)/(4 + w), so the form at z = 1 + w
    is (1 + 3z)/(3 + z) = 1/3 + (8/3) z/(z + 3): a_0 = 1/3, a_1 = 8/3, d_1 = 3."""
    a, d = O.pade_coef(1, 0.0)
    assert np.allclose(a, [1 / 3, 8 / 3], rtol=0, atol=1e-14)
    assert np.allclose(d, [0, 3], rtol=0, atol=1e-14)
    for z in (0.3, 1.0, 2.5 - 1j, 40j):
        assert abs(O.pade_eval(1, 0.0, z) - (1 + 3 * z) / (3 + z)) < 1e-14 * abs((1 + 3 * z) / (3 + z))


@pytest.mark.parametrize("m", [1, 2, 5, 20, 50, 100])
def test_coefficients_equal_the_closed_form_and_its_error(m):
    """The partial fractions equal the closed form of the approximant, and
    their error against sqrt(z) is the closed form's exact relative error
    2 rho^N/(1 - rho^N); on the arguments 2i/dt + W of the paper's grids
    (dt = 1e-3) the approximation is coarse for small m and tightens with m
    (the paper's iteration counts fall with m)."""
    for z in (1.0, 0.5 - 0.1j, 3 + 2000j, -30 + 2000j, 100 + 1e4j, 7 + 200j):
        r = O.pade_eval(m, THETA, z)
        c = _closed(m, z)
        assert abs(r - c) < 1e-11 * abs(c), (m, z)
        q = np.sqrt(np.exp(-1j * THETA) * z + 0j)
        rho = (1 - q) / (1 + q)
        err = 2 * rho ** (2 * m + 1) / (1 - rho ** (2 * m + 1))
        sq = np.exp(1j * THETA / 2) * q         # the principal sqrt(z) for these z
        assert abs(sq - np.sqrt(z + 0j)) < 1e-12 * abs(sq)
        assert abs((r - sq) / sq - err) < 1e-11 * max(1.0, abs(err)), (m, z)
    e = [abs(O.pade_eval(mm, THETA, 2000j) / np.sqrt(2000j) - 1) for mm in (20, 50, 100)]
    assert e[0] > e[1] > e[2] and e[2] < 1e-3


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("m", [1, 5, 20, 100])
def test_discrete_operator_has_the_crank_nicolson_symbol(order, m):
    dt, nt, w, dw = 0.01, 3000, 3.0, -2.5
    zeta = 1.01 * np.exp(0.3j)
    v = zeta ** np.arange(nt + 1)
    zd = (2j / dt) * (zeta - 1) / (zeta + 1)
    out, out_s = O.pade_apply(order, m, THETA, dt, v, w, dw)
    sym_s = -1j * _closed(m, zd + w)
    sym = sym_s + ((dw / 4) / (zd + w) if order == 4 else 0)
    assert abs(out[-1] / v[-1] - sym) < 1e-11 * abs(sym)
    # the exchanged part drops the order-4 term
    assert abs(out_s[-1] / v[-1] - sym_s) < 1e-11 * abs(sym_s)


def test_large_m_tends_to_the_potential_strategy_operator():
    """W = 0, v_0 = 0, a smooth sequence on the paper's dt: the distance to
    Sbar_0^2 falls steadily with m."""
    dt, nt = 1e-3, 2000
    t = dt * np.arange(nt + 1)
    v = np.sin(3 * t) ** 2 * np.exp(5j * t)
    z = np.zeros(nt + 1)
    s02, _ = O.sbar(W.S02, dt, v, z, z, z)
    dist = []
    for m in (20, 50, 100, 200):
        p, _ = O.pade_apply(2, m, THETA, dt, v, 0.0, 0.0)
        dist.append(np.max(abs(p[1:] - s02[1:])) / np.max(abs(s02)))
    assert all(a > 4 * b for a, b in zip(dist, dist[1:])), dist
    assert dist[-1] < 1e-6, dist


@pytest.mark.parametrize("vkind", [W.V_STATIC, W.V_TIME])
@pytest.mark.parametrize("trans", [W.P22, W.P24])
def test_swr_with_pade_converges_to_the_monodomain_solution(trans, vkind):
    """Consistency: the classical algorithm's fixed point and, for a static
    potential, the new algorithm (block lower-triangular Toeplitz interface
    problem) give the monodomain CN solution."""
    wl = W.small_case(N=3, nt=24, vkind=vkind, trans=trans, cells=8, seed=9)
    wl.pade_m = 8
    um = O.mono(wl, wl.u0[0])
    g, it, _ = O.classical(wl, wl.u0[0], tol=1e-12, maxit=600)
    assert it > 0
    uT, _ = O.local_solution(wl, wl.u0[0], g)
    assert np.max(abs(uT - um)) < 1e-11 * np.max(abs(um))
    if vkind == W.V_STATIC:
        u2 = O.new_algorithm(wl, wl.u0[0], solver="gmres", tol=1e-13)[0]
        assert np.max(abs(u2 - um)) < 1e-11 * np.max(abs(um))
        Lb = O.brute_L(wl)
        cols = O.impulse_columns(wl)
        rng = np.random.default_rng(4)
        x = rng.standard_normal(Lb.shape[1]) + 1j * rng.standard_normal(Lb.shape[1])
        assert np.max(abs(O.ltt_apply(wl, cols, x).ravel() - Lb @ x)) < 1e-12 * np.max(abs(Lb @ x))


def test_order_four_pade_with_the_cubic_potential_is_refused():
    """S2^{4,m} carries dn f(u) (refused with |u|^2, as S0^4 and S1^4); S2^{2,m}
    with |u|^2 is pinned with the other order-2 operators in
    test_oracle_transmission.py."""
    wl = W.small_case(N=2, nt=6, vkind=W.V_CUBIC, trans=W.P24, cells=6)
    with pytest.raises(RuntimeError):
        O.sweep(wl, 0, wl.u0[0])
