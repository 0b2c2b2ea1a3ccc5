"""The static causal solve replayed as one HIP graph (schedule option graph)
equals the solve launched kernel by kernel bit for bit, on every replay:
u(T), the interface fluxes g, the end-node traces, the snapshots and the
certified residual.  The replays read their inputs live (a new u0 written
into the same buffer), a new output pointer re-captures, and a new potential
goes back to an uncaptured solve first."""
import numpy as np
import pytest

from paper_1503_02564_amd import workloads as W
from tests.gpu_util import say, to_dev, to_np

pytestmark = pytest.mark.gpu

GRAPH_CASES = [
    # (label, J, nt, trans, sigma, B, pipeline)
    ("s02-pipelined", [60, 90, 75, 128, 200, 47, 250], 300, W.S02, 0j, 4, 64),
    ("robin-staged", [50, 70, 300, 33], 200, W.ROBIN, 1 - 1j, 3, 0),
    ("s02-staged-wide", [40] * 70, 160, W.S02, 0j, 2, 0),       # 69 interfaces: workgroup PCR
    # two finished 256-step super-blocks of the causal solve's far history
    ("s02-pipelined-long", [60, 90, 75, 128, 47], 600, W.S02, 0j, 2, 256),
]


def _problem(wl, pipeline):
    from paper_1503_02564_amd import swr
    o = swr.swr_default_opts()
    o.batch = wl.B
    o.pipeline = pipeline
    o.snapshot_stride = 50
    return swr.Problem(wl.a0, wl.b0, tuple(int(j) for j in wl.J), wl.dt, wl.dt * wl.nt, wl.vkind,
                       wl.trans, wl.sigma, o, to_dev(np.asarray(wl.V, np.float64)))


class _Outs:
    def __init__(self, pb, wl, dev):
        import torch
        B, nt = wl.B, wl.nt
        self.uT = torch.zeros((B, wl.nx), dtype=torch.complex128, device=dev)
        self.g = torch.zeros((B, pb.ns, nt), dtype=torch.complex128, device=dev)
        self.tr = torch.zeros((B, wl.N, 2, nt + 1), dtype=torch.complex128, device=dev)
        self.sn = torch.zeros((B, nt // 50 + 1, wl.nx), dtype=torch.complex128, device=dev)

    def solve(self, pb, u0):
        import torch
        from paper_1503_02564_amd import swr
        for x in (self.uT, self.g, self.tr, self.sn):
            x.fill_(float("nan"))
        st, info = swr.swr_solve(pb.ctx, u0, self.uT, self.g, self.tr, self.sn)
        assert st == swr.SWR_OK
        torch.cuda.synchronize()
        return [to_np(x) for x in (self.uT, self.g, self.tr, self.sn)], info.residual


@pytest.mark.parametrize("label,J,nt,trans,sigma,B,pipeline", GRAPH_CASES)
def test_graph_replays_equal_the_uncaptured_solve(dev, label, J, nt, trans, sigma, B, pipeline):
    import torch
    from paper_1503_02564_amd import swr
    wl = W.small_case(J=J, nt=nt, trans=trans, sigma=sigma, B=B, seed=41, a0=-12.0, b0=12.0)
    wl2 = W.small_case(J=J, nt=nt, trans=trans, sigma=sigma, B=B, seed=42, a0=-12.0, b0=12.0)
    eager = _problem(wl, pipeline)
    graph = _problem(wl, pipeline)
    swr.swr_set_schedule(graph.ctx, graph=1)
    assert swr.swr_get_schedule(graph.ctx).graph == 1
    assert swr.swr_get_schedule(eager.ctx).graph == 0
    oe, og = _Outs(eager, wl, dev), _Outs(graph, wl, dev)
    u0e, u0g = to_dev(wl.u0), to_dev(wl.u0)
    # call 1 uncaptured, call 2 captures and replays, calls 3-4 replay; the
    # input buffer of call 4 holds another initial condition
    for call in range(4):
        if call == 3:
            u0e.copy_(to_dev(wl2.u0))
            u0g.copy_(to_dev(wl2.u0))
        say("graph", label, "call", call)
        ref, res_e = oe.solve(eager, u0e)
        got, res_g = og.solve(graph, u0g)
        # the program's own eager work between replays
        torch.cuda.synchronize()
        _ = (u0g * 2).sum().item()
        for x, y in zip(ref, got):
            assert np.array_equal(x, y), (label, call)
        assert res_e == res_g and res_g < 1e-10
    # new output pointers: a new capture, same results
    og2 = _Outs(graph, wl, dev)
    for call in range(3):
        got, _ = og2.solve(graph, u0g)
        for x, y in zip(ref, got):
            assert np.array_equal(x, y), (label, "new pointers", call)
    # a new potential: an uncaptured solve (new causal set-up), then replays
    V2 = np.asarray(wl.V, np.float64) * 0.5
    for pb in (eager, graph):
        swr.swr_set_potential(pb.ctx, to_dev(V2))
    for call in range(3):
        ref, res_e = oe.solve(eager, u0e)
        got, res_g = og.solve(graph, u0g)
        for x, y in zip(ref, got):
            assert np.array_equal(x, y), (label, "new potential", call)
        assert res_e == res_g
    eager.close()
    graph.close()
