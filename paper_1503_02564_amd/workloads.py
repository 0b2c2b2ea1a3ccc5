"""Seeded synthetic inputs for the SWR solver (mesh, potential, initial data).

This module only *generates inputs*: it evaluates the analytic potentials and
initial wave packets that the paper's experiments are built from (Sec. 6:
harmonic potential, linear time-dependent potential, Gaussian packets) at the
nodes of a uniform mesh, with seeded random parameters.  It contains none of the
method's arithmetic and is imported by both the GPU path and the CPU oracle.

Conventions
-----------
* Mesh: uniform, ``nc = sum(J)`` cells on ``(a0, b0)``, nodes
  ``x_i = a0 + i*h``, ``i = 0..nc``.  Subdomain ``k`` owns nodes
  ``o_k .. o_k + J_k`` (``o_0 = 0``, ``o_{k+1} = o_k + J_k``).
* Potential kinds: ``V_STATIC`` (``V[nx]``), ``V_TIME`` (``V[nt+1][nx]``,
  row ``n`` at ``t_n = n*dt``), ``V_CUBIC`` (``|u|^2``, no array).
* Transmission: ``ROBIN`` (``dn u + sigma u``, complex ``sigma``), ``S02``,
  ``S03``, ``S04`` (potential strategy of order 2, 3, 4), ``S12``, ``S14``
  (gauge change strategy of order 2, 4) or ``P22``, ``P24`` (Pade strategy of
  order 2, 4 with ``pade_m`` auxiliary functions and branch rotation
  ``pade_theta``).
* Complex arrays are ``complex128`` (interleaved re/im doubles).
* Random numbers: ``numpy.random.default_rng(seed)``, fixed draw order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

V_STATIC, V_TIME, V_CUBIC = 0, 1, 2
ROBIN, S02, S03, S04, S12, S14, P22, P24 = 0, 1, 2, 3, 4, 5, 6, 7


@dataclass
class Workload:
    """One SWR problem instance (or a batch sharing mesh, potential kind and
    transmission)."""
    name: str
    a0: float
    b0: float
    J: np.ndarray            # int32 cells per subdomain
    dt: float
    nt: int
    vkind: int
    V: Optional[np.ndarray]  # [nx] | [nt+1][nx] | [B][nx] (per-problem static) | None
    trans: int
    sigma: complex           # Robin coefficient of dn + sigma (unused for S02)
    u0: np.ndarray           # [B][nx] complex128
    tol: float = 1e-10
    seed: int = 0
    extras: dict = field(default_factory=dict)
    pade_m: int = 20                 # Pade strategy: auxiliary functions per end
    pade_theta: float = np.pi / 4    # and the rotation of the square root's branch cut

    @property
    def N(self) -> int:
        return int(len(self.J))

    @property
    def nc(self) -> int:
        return int(np.sum(self.J))

    @property
    def nx(self) -> int:
        return self.nc + 1

    @property
    def h(self) -> float:
        return (self.b0 - self.a0) / self.nc

    @property
    def B(self) -> int:
        return int(self.u0.shape[0])

    @property
    def offsets(self) -> np.ndarray:
        o = np.zeros(self.N, dtype=np.int64)
        o[1:] = np.cumsum(self.J)[:-1]
        return o

    def x(self) -> np.ndarray:
        return mesh_nodes(self.a0, self.b0, self.nc)

    def pt_steps(self) -> int:
        """Grid-point x time-step count of one solve of the whole batch."""
        return self.nx * self.nt * self.B


def mesh_nodes(a0: float, b0: float, nc: int) -> np.ndarray:
    h = (b0 - a0) / nc
    return a0 + h * np.arange(nc + 1, dtype=np.float64)


def gaussian_packet(x: np.ndarray, x0: float, k0: float) -> np.ndarray:
    """exp(-(x-x0)^2 + i k0 (x-x0)): unit-width packet centred at x0 with
    momentum k0 (the initial-data family of Sec. 6)."""
    d = x - x0
    return np.exp(-d * d + 1j * k0 * d)


def bumpy_harmonic(x: np.ndarray, amps, centres, curvature=-0.05) -> np.ndarray:
    """curvature*x^2 plus unit-width Gaussian bumps A_k exp(-(x-c_k)^2)."""
    v = curvature * x * x
    for a, c in zip(amps, centres):
        v = v + a * np.exp(-(x - c) ** 2)
    return v


# ---------------------------------------------------------------------------
# The workloads of the measurements and the full-size tests.  ``scale`` shrinks them for tests
# (fewer cells per subdomain and fewer steps, same structure).
# ---------------------------------------------------------------------------

def robin_window() -> Workload:
    """Plain SWR: (-10,10), 400 cells, 4 equal subdomains, V=0,
    u0 = exp(-x^2 + 2ix), dt=1e-3, 500 steps, Robin dn u + (1-i) u,
    classical fixed point to max trace change < 1e-10."""
    J = np.full(4, 100, dtype=np.int32)
    x = mesh_nodes(-10.0, 10.0, int(J.sum()))
    u0 = gaussian_packet(x, 0.0, 2.0)[None, :]
    return Workload("robin_window", -10.0, 10.0, J, 1e-3, 500, V_STATIC,
                    np.zeros_like(x), ROBIN, 1.0 - 1.0j, u0, tol=1e-10, seed=1)


def static_packet(N: int = 64, cells: int = 256, nt: int = 2000, seed: int = 2) -> Workload:
    """Time-independent potential, preprocessed interface algorithm:
    (-40,40), N x cells cells, V = -0.05x^2 + 8 seeded Gaussian bumps
    (A ~ U(-5,5), c ~ U(-30,30)), packet with x0, k0 ~ U(-5,5),
    dt = 5e-4 (scaled so T = 1 stays fixed when nt changes), S0^2, GMRES."""
    rng = np.random.default_rng(seed)
    amps = rng.uniform(-5.0, 5.0, 8)
    centres = rng.uniform(-30.0, 30.0, 8)
    x0, k0 = rng.uniform(-5.0, 5.0, 2)
    J = np.full(N, cells, dtype=np.int32)
    x = mesh_nodes(-40.0, 40.0, int(J.sum()))
    V = bumpy_harmonic(x, amps, centres)
    u0 = gaussian_packet(x, x0, k0)[None, :]
    dt = 1.0 / nt
    return Workload("static_packet", -40.0, 40.0, J, dt, nt, V_STATIC, V,
                    S02, 0j, u0, tol=1e-10, seed=seed,
                    extras=dict(amps=amps, centres=centres, x0=x0, k0=k0))


def batched_uneven(N: int = 500, lo: int = 40, hi: int = 400, B: int = 32, nt: int = 2000,
            seed: int = 3) -> Workload:
    """Batched uneven decomposition: (-100,100), N subdomains with seeded
    sizes U{lo..hi} cells, V = V2(0.4 x) (the static-packet form stretched to the
    domain), B seeded packets (x0 ~ U(-12.5,12.5), k0 ~ U(-5,5)),
    dt = 5e-4 at nt=2000, S0^2."""
    rng = np.random.default_rng(seed)
    J = rng.integers(lo, hi + 1, N).astype(np.int32)
    amps = rng.uniform(-5.0, 5.0, 8)
    centres = rng.uniform(-30.0, 30.0, 8)
    pk = rng.uniform(size=(B, 2))
    x = mesh_nodes(-100.0, 100.0, int(J.sum()))
    V = bumpy_harmonic(0.4 * x, amps, centres)
    u0 = np.stack([gaussian_packet(x, -12.5 + 25.0 * a, -5.0 + 10.0 * b) for a, b in pk])
    return Workload("batched_uneven", -100.0, 100.0, J, 1.0 / nt, nt, V_STATIC, V,
                    S02, 0j, u0, tol=1e-10, seed=seed)


def _four_packets(x, rng):
    p = rng.uniform(-5.0, 5.0, (4, 2))
    return sum(gaussian_packet(x, a, b) for a, b in p)


def time_dependent(N: int = 128, cells: int = 256, nt: int = 4000, seed: int = 4) -> Workload:
    """Time-dependent potential V(t,x) = 5 x cos t on (-40,40), N x cells
    cells, seeded sum of 4 packets, dt = 2.5e-4 at nt = 4000, S0^2,
    preconditioned by the zero-potential interface operator."""
    rng = np.random.default_rng(seed)
    J = np.full(N, cells, dtype=np.int32)
    x = mesh_nodes(-40.0, 40.0, int(J.sum()))
    u0 = _four_packets(x, rng)[None, :]
    dt = 1.0 / nt
    t = dt * np.arange(nt + 1)
    V = 5.0 * np.cos(t)[:, None] * x[None, :]
    return Workload("time_dependent", -40.0, 40.0, J, dt, nt, V_TIME, V,
                    S02, 0j, u0, tol=1e-10, seed=seed)


def cubic_packets(N: int = 128, cells: int = 256, nt: int = 4000, seed: int = 4) -> Workload:
    """Cubic nonlinearity V = |u|^2 with the same mesh, data and step as 4a."""
    rng = np.random.default_rng(seed)
    J = np.full(N, cells, dtype=np.int32)
    x = mesh_nodes(-40.0, 40.0, int(J.sum()))
    u0 = _four_packets(x, rng)[None, :]
    return Workload("cubic_packets", -40.0, 40.0, J, 1.0 / nt, nt, V_CUBIC, None,
                    S02, 0j, u0, tol=1e-10, seed=seed)


def adjoint_batch(N: int = 256, cells: int = 64, nt: int = 2000, B: int = 16, seed: int = 5) -> Workload:
    """Differentiation: (-40,40), N x cells cells, B seeded potentials of the
    static-packet form plus one seeded reference potential, one seeded packet,
    dt = 5e-4 at nt = 2000, S0^2, adjoint checkpoint interval 64.
    V is [B][nx]; extras['V_ref'] is the reference potential."""
    rng = np.random.default_rng(seed)
    J = np.full(N, cells, dtype=np.int32)
    x = mesh_nodes(-40.0, 40.0, int(J.sum()))
    Vs = []
    for _ in range(B + 1):
        amps = rng.uniform(-5.0, 5.0, 8)
        centres = rng.uniform(-30.0, 30.0, 8)
        Vs.append(bumpy_harmonic(x, amps, centres))
    x0, k0 = rng.uniform(-5.0, 5.0, 2)
    u0 = np.repeat(gaussian_packet(x, x0, k0)[None, :], B, axis=0)
    return Workload("adjoint_batch", -40.0, 40.0, J, 1.0 / nt, nt, V_STATIC,
                    np.stack(Vs[:B]), S02, 0j, u0, tol=1e-10, seed=seed,
                    extras=dict(V_ref=Vs[B], checkpoint_K=64))


def paper_case(kind: str, N: int = 1000, dx: float = 1e-4, nt: int = 500) -> Workload:
    """The workloads of the paper's numerical section (Sec. 6): (-21, 21)
    in N equal subdomains of mesh size dx, T = 0.5, dt = T/nt (1e-3), S0^2.
    kind 'harmonic': V = -x^2; 'linear_t': V(t, x) = 5 t x (both with
    u0 = exp(-(x+10)^2 + 20 i (x+10))); 'cubic': |u|^2 with
    u0 = 2 sech(sqrt(2)(x+10)) exp(20 i (x+10)).  The paper's grids are
    dx = 1e-5 and 1e-4 with N up to 1000; no random numbers are drawn."""
    a0, b0, T = -21.0, 21.0, 0.5
    nc = int(round((b0 - a0) / dx))
    if nc % N:
        raise ValueError("N must divide the number of cells")
    J = np.full(N, nc // N, dtype=np.int32)
    x = mesh_nodes(a0, b0, nc)
    dt = T / nt
    y = x + 10.0
    if kind == "cubic":
        u0 = (2.0 / np.cosh(np.sqrt(2.0) * y)) * np.exp(20j * y)
    else:
        u0 = np.exp(-y * y + 20j * y)
    if kind == "harmonic":
        vk, V = V_STATIC, -x * x
    elif kind == "linear_t":
        t = dt * np.arange(nt + 1)
        vk, V = V_TIME, 5.0 * t[:, None] * x[None, :]
    elif kind == "cubic":
        vk, V = V_CUBIC, None
    else:
        raise ValueError(kind)
    return Workload(f"paper_{kind}", a0, b0, J, dt, nt, vk, V, S02, 0j, u0[None, :], tol=1e-10)


def small_case(N=3, J=None, nt=12, a0=-6.0, b0=6.0, vkind=V_STATIC, trans=S02,
               sigma=1.0 - 1.0j, B=1, seed=7, cells=8) -> Workload:
    """Tiny seeded case for brute-force checks (a few dozen nodes)."""
    rng = np.random.default_rng(seed)
    if J is None:
        J = np.full(N, cells, dtype=np.int32)
    J = np.asarray(J, dtype=np.int32)
    x = mesh_nodes(a0, b0, int(J.sum()))
    dt = 0.5 / nt
    if vkind == V_STATIC:
        V = bumpy_harmonic(x, rng.uniform(-5, 5, 3), rng.uniform(a0, b0, 3))
    elif vkind == V_TIME:
        t = dt * np.arange(nt + 1)
        V = 5.0 * np.cos(t)[:, None] * x[None, :]
    else:
        V = None
    pk = rng.uniform(size=(B, 2))
    u0 = np.stack([gaussian_packet(x, a0 / 3 + (b0 - a0) / 3 * a, -3 + 6 * b) for a, b in pk])
    return Workload("small", a0, b0, J, dt, nt, vkind, V, trans, sigma, u0, seed=seed)
