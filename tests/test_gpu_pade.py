"""GPU parity of the Pade strategy's transmissions S2^{2,m}, S2^{4,m}
(Sec. 2.1 "Pade approximation strategy", Sec. 2.2 auxiliary functions phi^s,
psi) against the CPU oracle, through the C ABI; coefficients as the oracle
reads them (diagonal Pade approximant of sqrt(1 + w), branch cut rotated by
theta).

One sweep / one interface build: 1e-12 relative (rounding order only: the GPU
sums the m auxiliary terms of each step as a 64-lane tree, the oracle in
order).  Converged solves: 1e-10 against the monodomain solution.  The
pipelined solve carries the auxiliary functions across its chunk launches and
equals the staged solve bit for bit.
"""
import numpy as np
import pytest

import oracle as O
from paper_1503_02564_amd import workloads as W
from tests.gpu_util import make_problem, rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu

KINDS = [("p22", W.P22), ("p24", W.P24)]
RAGGED = [40, 63, 64, 100, 127, 128, 200, 255, 256, 300]


def _case(J, nt, trans, m, B=1, seed=3, theta=np.pi / 4):
    wl = W.small_case(J=J, nt=nt, trans=trans, sigma=0j, B=B, seed=seed, a0=-12.0, b0=12.0)
    wl.pade_m = m
    wl.pade_theta = theta
    return wl


@pytest.mark.parametrize("name,trans", KINDS)
@pytest.mark.parametrize("m", [1, 20, 65, 128])
@pytest.mark.parametrize("with_data", [True, False])
def test_one_sweep_matches_oracle(dev, name, trans, m, with_data):
    import torch
    from paper_1503_02564_amd import swr
    wl = _case(RAGGED, 150, trans, m)
    say("pade one_sweep", name, "m", m, "data" if with_data else "zero-data")
    pb = make_problem(wl)
    rng = np.random.default_rng(11)
    g = rng.standard_normal((pb.ns, wl.nt)) + 1j * rng.standard_normal((pb.ns, wl.nt))
    u0 = wl.u0[0] if with_data else None
    g_out = torch.zeros((1, pb.ns, wl.nt), dtype=torch.complex128, device=dev)
    uT = torch.zeros((1, wl.nx), dtype=torch.complex128, device=dev)
    swr.swr_apply_R(pb.ctx, to_dev(wl.u0) if with_data else None, to_dev(g[None]), g_out, uT)
    torch.cuda.synchronize()
    want = O.apply_R(wl, u0, g, hist0_zero=not with_data)
    assert rel(to_np(g_out)[0], want) < 1e-12
    if with_data:
        assert rel(to_np(uT)[0], O.local_solution(wl, u0, g)[0]) < 1e-12
    pb.close()


@pytest.mark.parametrize("name,trans", KINDS)
def test_impulse_columns_and_d_match_oracle(dev, name, trans):
    import torch
    from paper_1503_02564_amd import swr
    wl = _case(RAGGED, 150, trans, 50, theta=0.6)
    say("pade build_interface", name)
    pb = make_problem(wl)
    cols = torch.zeros((1, wl.N, 4, wl.nt), dtype=torch.complex128, device=dev)
    d = torch.zeros((1, pb.ns, wl.nt), dtype=torch.complex128, device=dev)
    swr.swr_build_interface(pb.ctx, to_dev(wl.u0), cols, d)
    torch.cuda.synchronize()
    assert rel(to_np(cols)[0], O.impulse_columns(wl)) < 1e-12
    assert rel(to_np(d)[0], O.interface_d(wl, wl.u0[0])) < 1e-12
    pb.close()


@pytest.mark.parametrize("name,trans", KINDS)
@pytest.mark.parametrize("solver", ["causal", "gmres", "bicgstab", "fixed"])
def test_solve_matches_monodomain(dev, name, trans, solver):
    import torch
    from paper_1503_02564_amd import swr
    wl = _case([40, 63, 64, 100, 127, 200, 31], 130, trans, 20)
    sv = dict(causal=swr.SWR_SOLVER_CAUSAL, gmres=swr.SWR_SOLVER_GMRES,
              bicgstab=swr.SWR_SOLVER_BICGSTAB, fixed=swr.SWR_SOLVER_FIXED)[solver]
    say("pade solve", name, solver)
    tol = 1e-12 if solver == "fixed" else 1e-13
    pb = make_problem(wl, solver=sv, tol=tol, restart=60, max_iter=3000)
    uT = torch.zeros((1, wl.nx), dtype=torch.complex128, device=dev)
    g = torch.zeros((1, pb.ns, wl.nt), dtype=torch.complex128, device=dev)
    st, info = swr.swr_solve(pb.ctx, to_dev(wl.u0), uT, g)
    torch.cuda.synchronize()
    assert st == swr.SWR_OK
    um = O.mono(wl, wl.u0[0])
    assert rel(to_np(uT)[0], um) < 1e-10
    if solver == "fixed":
        _, it, _ = O.classical(wl, wl.u0[0], tol=tol, maxit=3000)
        assert abs(info.iters - it) <= 1
    else:
        assert info.residual < 1e-11
        gw = O.causal_solve(wl, O.impulse_columns(wl), O.interface_d(wl, wl.u0[0]))
        assert rel(to_np(g)[0], gw) < 1e-10
    pb.close()


@pytest.mark.parametrize("name,trans", KINDS)
def test_pipelined_solve_equals_staged_solve(dev, name, trans):
    """Chunk launches restore the auxiliary functions they saved: the
    pipelined solve equals the staged one bit for bit, batched."""
    import torch
    from paper_1503_02564_amd import swr
    wl = _case([40, 63, 64, 100, 127, 200, 31], 450, trans, 100, B=3)
    out = []
    for ch in (0, 64):
        say("pade pipeline", name, "chunk", ch)
        pb = make_problem(wl, pipeline=ch)
        uT = torch.zeros((3, wl.nx), dtype=torch.complex128, device=dev)
        g = torch.zeros((3, pb.ns, wl.nt), dtype=torch.complex128, device=dev)
        st, info = swr.swr_solve(pb.ctx, to_dev(wl.u0), uT, g)
        torch.cuda.synchronize()
        assert st == swr.SWR_OK and info.residual < 1e-11
        out.append((to_np(uT), to_np(g)))
        pb.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    for b in range(3):
        assert rel(out[1][0][b], O.mono(wl, wl.u0[b])) < 1e-10


def test_gradient_refuses_pade(dev):
    import torch
    from paper_1503_02564_amd import swr
    wl = _case([40, 50], 64, W.P22, 8)
    say("pade grad refuses")
    pb = make_problem(wl)
    u0 = to_dev(wl.u0)
    dV = torch.zeros((1, wl.nx), dtype=torch.float64, device=dev)
    with pytest.raises(swr.SwrError) as e:
        swr.swr_grad(pb.ctx, u0, torch.zeros_like(u0), dV, torch.zeros_like(u0))
    assert e.value.status == swr.SWR_EINVAL
    pb.close()
