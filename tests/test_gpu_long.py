"""GPU parity of the long-chunk sweep: subdomains of more than 64 * 8 nodes
(the paper's finest grid, Sec. 6, has 4201-node subdomains at N = 1000),
alone and mixed with register-sweep subdomains, for Robin and S0^2 with a
static, a time-dependent and the |u|^2 potential, against the CPU oracle
through the C ABI.  One sweep: 1e-11 -- the per-lane Thomas elimination runs
over up to 66 nodes instead of at most 8, which adds rounding against the
oracle's single Thomas sweep (measured up to 1.1e-12 with the packet on an
interface); converged solves 1e-10 against the monodomain solution."""
import numpy as np
import pytest

import oracle as O
from paper_1503_02564_amd import workloads as W
from tests.gpu_util import make_problem, rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu

# 4201 nodes: 66 per lane; 530 / 601 / 2001: 9, 10, 32 per lane; 300: register sweep
MIXED = [600, 4200, 300, 2000, 530]

SWEEP_CASES = [
    ("static-s02", W.V_STATIC, W.S02, 0j, 1e-11),
    ("static-robin", W.V_STATIC, W.ROBIN, 2 - 3j, 1e-11),
    ("time-s02", W.V_TIME, W.S02, 0j, 1e-11),
    ("cubic-s02", W.V_CUBIC, W.S02, 0j, 1e-11),
]


def _case(J, nt, vk, trans, sigma, seed=5):
    """A packet on the interface between the first two subdomains (so that
    the interface data d is of the solution's size, not a far tail)."""
    wl = W.small_case(J=J, nt=nt, vkind=vk, trans=trans, sigma=sigma, seed=seed, a0=-12.0, b0=12.0)
    x = wl.x()
    wl.u0 = W.gaussian_packet(x, x[int(wl.offsets[1])], 2.0)[None, :].astype(np.complex128)
    if vk == W.V_CUBIC:
        wl.u0 = 1.5 * wl.u0
    return wl


@pytest.mark.parametrize("label,vk,trans,sigma,bar", SWEEP_CASES)
def test_one_sweep_matches_oracle(dev, label, vk, trans, sigma, bar):
    import torch
    from paper_1503_02564_amd import swr
    wl = _case(MIXED, 130, vk, trans, sigma)
    say("long one_sweep", label)
    pb = make_problem(wl)
    rng = np.random.default_rng(13)
    g = 0.3 * (rng.standard_normal((pb.ns, wl.nt)) + 1j * rng.standard_normal((pb.ns, wl.nt)))
    g_out = torch.zeros((1, pb.ns, wl.nt), dtype=torch.complex128, device=dev)
    uT = torch.zeros((1, wl.nx), dtype=torch.complex128, device=dev)
    swr.swr_apply_R(pb.ctx, to_dev(wl.u0), to_dev(g[None]), g_out, uT)
    torch.cuda.synchronize()
    eg = rel(to_np(g_out)[0], O.apply_R(wl, wl.u0[0], g))
    eu = rel(to_np(uT)[0], O.local_solution(wl, wl.u0[0], g)[0])
    say("long one_sweep", label, "g", eg, "uT", eu)
    assert eg < bar and eu < bar
    pb.close()


def test_impulse_columns_match_oracle(dev):
    import torch
    from paper_1503_02564_amd import swr
    wl = _case(MIXED, 130, W.V_STATIC, W.S02, 0j)
    say("long build_interface")
    pb = make_problem(wl)
    cols = torch.zeros((1, wl.N, 4, wl.nt), dtype=torch.complex128, device=dev)
    d = torch.zeros((1, pb.ns, wl.nt), dtype=torch.complex128, device=dev)
    swr.swr_build_interface(pb.ctx, to_dev(wl.u0), cols, d)
    torch.cuda.synchronize()
    ec = rel(to_np(cols)[0], O.impulse_columns(wl))
    ed = rel(to_np(d)[0], O.interface_d(wl, wl.u0[0]))
    say("long build_interface", "cols", ec, "d", ed)
    assert ec < 1e-11 and ed < 1e-11
    pb.close()


SOLVE_CASES = [
    ("static-s02-causal", W.V_STATIC, W.S02, 0j, "causal"),
    ("static-s02-gmres", W.V_STATIC, W.S02, 0j, "gmres"),
    ("static-robin-fixed", W.V_STATIC, W.ROBIN, 2 - 3j, "fixed"),
    ("time-s02", W.V_TIME, W.S02, 0j, "default"),
    ("cubic-s02", W.V_CUBIC, W.S02, 0j, "default"),
]


@pytest.mark.parametrize("label,vk,trans,sigma,solver", SOLVE_CASES)
def test_solve_matches_monodomain(dev, label, vk, trans, sigma, solver):
    import torch
    from paper_1503_02564_amd import swr
    wl = _case(MIXED, 100, vk, trans, sigma)
    sv = dict(causal=swr.SWR_SOLVER_CAUSAL, gmres=swr.SWR_SOLVER_GMRES, fixed=swr.SWR_SOLVER_FIXED,
              default=None)[solver]
    say("long solve", label)
    tol = 1e-12 if solver == "fixed" else 1e-13
    pb = make_problem(wl, solver=sv, tol=tol, restart=60, max_iter=3000)
    uT = torch.zeros((1, wl.nx), dtype=torch.complex128, device=dev)
    st, info = swr.swr_solve(pb.ctx, to_dev(wl.u0), uT)
    torch.cuda.synchronize()
    say("long solve", label, info.iters, info.residual)
    assert st == swr.SWR_OK
    assert rel(to_np(uT)[0], O.mono(wl, wl.u0[0])) < 1e-10
    pb.close()


def test_gradient_refuses_long_subdomains(dev):
    import torch
    from paper_1503_02564_amd import swr
    wl = _case([600, 300], 64, W.V_STATIC, W.S02, 0j)
    pb = make_problem(wl)
    u0 = to_dev(wl.u0)
    dV = torch.zeros((1, wl.nx), dtype=torch.float64, device=dev)
    with pytest.raises(swr.SwrError) as e:
        swr.swr_grad(pb.ctx, u0, torch.zeros_like(u0), dV, torch.zeros_like(u0))
    assert e.value.status == swr.SWR_EINVAL
    pb.close()
