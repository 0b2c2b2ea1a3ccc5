"""The C-ABI outputs beyond u(T): snapshots of u(t_n, x) from the final sweep,
the per-iteration convergence history in swr_info, the size query, and the
binding's argument checks (dtype, device, element count) before a pointer
reaches the library.

Snapshots are compared element by element with the oracle's monodomain
u_n at the same steps (1e-10 relative, the method's target; the solves
iterate to 1e-13), in the pipelined (chunked final sweep), staged and GMRES
launch forms, with a stride that does not divide the number of steps and with
a ragged last pipeline chunk."""
import numpy as np
import pytest

import oracle as O
from paper_1503_02564_amd import workloads as W
from tests.gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _problem(wl, **kw):
    from paper_1503_02564_amd import swr
    o = swr.swr_default_opts()
    o.batch = wl.B
    o.tol = 1e-13
    for k, v in kw.items():
        setattr(o, k, v)
    V = None if wl.V is None else to_dev(np.asarray(wl.V, np.float64))
    return swr.Problem(wl.a0, wl.b0, tuple(int(j) for j in wl.J), wl.dt, wl.dt * wl.nt, wl.vkind,
                       wl.trans, wl.sigma, o, V)


@pytest.mark.parametrize("form", ["pipelined", "staged", "gmres"])
def test_snapshots_equal_monodomain_steps(dev, form):
    import torch
    from paper_1503_02564_amd import swr
    wl = W.small_case(J=[60, 90, 75, 128, 47], nt=200, B=2, seed=11, a0=-10.0, b0=10.0)
    stride = 7
    kw = dict(snapshot_stride=stride)
    if form == "pipelined":
        kw["pipeline"] = 64          # 200 steps: chunks 64, 64, 64, 8
    elif form == "staged":
        kw["pipeline"] = 0
    else:
        kw.update(solver=swr.SWR_SOLVER_GMRES, restart=60, max_iter=2000)
    say("snapshots", form, "stride", stride, "nt", wl.nt, "B", wl.B)
    pb = _problem(wl, **kw)
    z = swr._sizes(pb.ctx)
    S = wl.nt // stride + 1
    assert z.S == S and z.N == wl.N and z.vk == wl.vkind
    uT = torch.zeros((wl.B, wl.nx), dtype=torch.complex128, device=dev)
    snaps = torch.zeros((wl.B, S, wl.nx), dtype=torch.complex128, device=dev)
    st, info = swr.swr_solve(pb.ctx, to_dev(wl.u0), uT, snaps=snaps)
    torch.cuda.synchronize()
    assert st == swr.SWR_OK, st
    got = to_np(snaps)
    for b in range(wl.B):
        _, u_all, _ = O.mono(wl, wl.u0[b], want_u=True)
        want = u_all[::stride]
        assert want.shape == got[b].shape
        err = rel(got[b], want)
        say("snapshots", form, "member", b, "rel err", err)
        assert err < 1e-10
        assert np.array_equal(got[b][0], wl.u0[b])        # step 0 is the data itself
    # the last snapshot step (196) is not nt (200): u(T) is not a snapshot
    assert rel(to_np(uT), np.stack([O.mono(wl, wl.u0[b]) for b in range(wl.B)])) < 1e-10
    pb.close()


def test_snapshots_need_a_stride(dev):
    import torch
    from paper_1503_02564_amd import swr
    wl = W.small_case(J=[20, 20], nt=10, seed=3)
    pb = _problem(wl)
    uT = torch.zeros((1, wl.nx), dtype=torch.complex128, device=dev)
    snaps = torch.zeros((1, 2, wl.nx), dtype=torch.complex128, device=dev)
    with pytest.raises(ValueError):
        swr.swr_solve(pb.ctx, to_dev(wl.u0), uT, snaps=snaps)
    # the library itself refuses a snapshot buffer without a stride
    st = swr._L.swr_solve(pb.ctx, swr._arr(to_dev(wl.u0), "c", wl.nx, "u0"),
                          swr._arr(uT, "c", wl.nx, "uT"), None, None,
                          swr._arr(snaps, "c", 2 * wl.nx, "snaps"), None)
    assert st == swr.SWR_EINVAL
    pb.close()


def test_history_of_each_solver(dev):
    """GMRES and BiCGStab record one relative residual estimate per
    iteration, decreasing to the tolerance; the fixed point its max trace
    changes; the causal solve (one pass) its certified residual."""
    import torch
    from paper_1503_02564_amd import swr
    wl = W.small_case(J=[40, 52, 40, 33], nt=96, seed=5, a0=-8.0, b0=8.0)
    uT = torch.zeros((1, wl.nx), dtype=torch.complex128, device=dev)
    for name, solver in (("gmres", swr.SWR_SOLVER_GMRES), ("bicgstab", swr.SWR_SOLVER_BICGSTAB),
                         ("fixed", swr.SWR_SOLVER_FIXED), ("causal", swr.SWR_SOLVER_CAUSAL)):
        pb = _problem(wl, solver=solver, tol=1e-11, max_iter=3000, restart=40)
        st, info = swr.swr_solve(pb.ctx, to_dev(wl.u0), uT)
        torch.cuda.synchronize()
        h = info.history
        say("history", name, "iters", info.iters, "len", len(h), "first", h[:2], "last", h[-1:])
        assert st == swr.SWR_OK
        if name == "causal":
            assert len(h) == 1 and h[0] == info.residual
        else:
            assert len(h) == info.iters
            assert h[-1] < 1e-11 and h[0] > h[-1]
            assert np.all(np.isfinite(h))
        assert rel(to_np(uT)[0], O.mono(wl, wl.u0[0])) < 1e-9
        pb.close()


def test_binding_checks_arguments_before_the_abi(dev):
    import torch
    from paper_1503_02564_amd import swr
    wl = W.small_case(J=[20, 24], nt=8, B=2, seed=4)
    pb = _problem(wl)
    u0 = to_dev(wl.u0)
    uT = torch.zeros((2, wl.nx), dtype=torch.complex128, device=dev)
    bad = [
        (u0.to(torch.complex64), uT),                                       # dtype
        (u0[:1].contiguous(), uT),                                          # element count
        (u0, torch.zeros((2, wl.nx + 1), dtype=torch.complex128, device=dev)),
        (u0.cpu(), uT),                                                     # device
        (u0.t(), uT),                                                       # not contiguous
    ]
    for a, b in bad:
        with pytest.raises(ValueError):
            swr.swr_solve(pb.ctx, a, b)
    with pytest.raises(ValueError):
        swr.swr_set_potential(pb.ctx, to_dev(np.asarray(wl.V, np.float32)))
    with pytest.raises(ValueError):
        swr.swr_set_potential(pb.ctx, to_dev(np.zeros(wl.nx - 1)))
    g = torch.zeros((2, 2, wl.nt), dtype=torch.complex128, device=dev)
    with pytest.raises(ValueError):
        swr.swr_apply_R(pb.ctx, u0, g, g[:1].contiguous())
    st, _ = swr.swr_solve(pb.ctx, u0, uT, g)
    assert st == swr.SWR_OK
    pb.close()


def test_autograd_raises_when_the_interface_solve_does_not_converge(dev):
    """SWRFunction reports a non-converged forward solve instead of returning
    its last iterate as u(T)."""
    import torch
    from paper_1503_02564_amd import swr
    from paper_1503_02564_amd.autograd import SWRFunction
    wl = W.small_case(J=[30, 30, 30], nt=40, seed=6)
    pb = _problem(wl, solver=swr.SWR_SOLVER_GMRES, max_iter=2, restart=2, tol=1e-14)
    V = to_dev(np.asarray(wl.V, np.float64)).requires_grad_(True)
    with pytest.raises(swr.SwrError):
        SWRFunction.apply(V, to_dev(wl.u0), pb)
    pb.close()
