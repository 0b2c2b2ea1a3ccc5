"""The autotuner (swr_tune) and its cache.  Schedules change how the work is
launched, never the arithmetic of a result: the solve with the tuned
schedule equals the default one bit for bit (pipeline chunk, helper-wave
bound).  The cache written by swr_tune is read back by a later swr_setup of
the same problem shape and ignored by another shape."""
import numpy as np
import pytest

from paper_1503_02564_amd import workloads as W
from tests.gpu_util import say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _problem(wl, cache=None, **kw):
    from paper_1503_02564_amd import swr
    o = swr.swr_default_opts()
    o.batch = wl.B
    if cache is not None:
        o.tune_cache = cache.encode()
    for k, v in kw.items():
        setattr(o, k, v)
    return swr.Problem(wl.a0, wl.b0, tuple(int(j) for j in wl.J), wl.dt, wl.dt * wl.nt, wl.vkind,
                       wl.trans, wl.sigma, o, to_dev(np.asarray(wl.V, np.float64)))


def test_tuned_schedule_gives_the_same_result_and_is_cached(dev, tmp_path):
    import torch
    from paper_1503_02564_amd import swr
    wl = W.static_packet(N=16, cells=96, nt=600)
    cache = str(tmp_path / "swr_schedules.txt")
    pb = _problem(wl, cache)
    default = swr.swr_get_schedule(pb.ctx).as_dict()
    say("tune", "default schedule", default)
    assert default["pipeline"] == 256            # 46 build tasks: the pipelined form
    u0 = to_dev(wl.u0)
    u_def = torch.zeros_like(u0)
    st, _ = swr.swr_solve(pb.ctx, u0, u_def)
    assert st == swr.SWR_OK
    chosen = swr.swr_tune(pb.ctx, u0, budget_ms=3000.0)
    say("tune", "chosen", chosen.as_dict())
    assert chosen.candidates >= 2 and np.isfinite(chosen.ms)
    assert chosen.pipeline in (0, 128, 256, 512) and chosen.help_max >= 0
    assert swr.swr_get_schedule(pb.ctx).as_dict()["pipeline"] == chosen.pipeline
    u_tuned = torch.zeros_like(u0)
    st, _ = swr.swr_solve(pb.ctx, u0, u_tuned)
    assert st == swr.SWR_OK
    assert np.array_equal(to_np(u_def), to_np(u_tuned))
    pb.close()
    text = open(cache).read()
    assert text.count("\n") == 1
    # a later setup of the same shape starts from the cached schedule ...
    pb2 = _problem(wl, cache)
    s2 = swr.swr_get_schedule(pb2.ctx)
    assert (s2.pipeline, s2.help_max, s2.restart) == (chosen.pipeline, chosen.help_max, chosen.restart)
    pb2.close()
    # ... another shape does not
    other = W.static_packet(N=12, cells=96, nt=600)
    pb3 = _problem(other, cache)
    assert swr.swr_get_schedule(pb3.ctx).as_dict() == swr.swr_get_schedule(
        _problem(other).ctx).as_dict()
    pb3.close()


def test_default_schedule_pipelines_filled_batches(dev):
    from paper_1503_02564_amd import swr
    wl = W.batched_uneven(N=100, B=48, nt=128)   # 100 * 48 + 198 build tasks: sweeps fill the GPU
    pb = _problem(wl)
    assert swr.swr_get_schedule(pb.ctx).pipeline == 256
    pb.close()


PAIR_CASES = [
    # (label, J, nt, trans, sigma, B, pipeline): odd batches leave single tasks
    ("s02-staged", [60, 90, 75, 128, 200, 47, 250], 300, W.S02, 0j, 3, 0),
    ("s02-pipelined", [60, 90, 75, 128, 200, 47, 250], 300, W.S02, 0j, 4, 64),
    ("robin-staged", [50, 70, 300, 33], 200, W.ROBIN, 1 - 1j, 3, 0),
]


@pytest.mark.parametrize("label,J,nt,trans,sigma,B,pipeline", PAIR_CASES)
def test_two_task_waves_equal_one_task_waves(dev, label, J, nt, trans, sigma, B, pipeline):
    """Sweeps that run two tasks of one subdomain per wave (forced here for
    every width and launch size) perform each task's arithmetic exactly as
    the one-task waves: u(T), g, end-node traces, snapshots and the adjoint's
    gradients are bitwise equal; u(T) matches the monodomain oracle."""
    import torch
    import oracle as O
    from paper_1503_02564_amd import swr
    from tests.gpu_util import rel
    wl = W.small_case(J=J, nt=nt, trans=trans, sigma=sigma, B=B, seed=29, a0=-12.0, b0=12.0)
    out = {}
    for pair in (False, True):
        say("two-task waves", label, "pairs", pair)
        pb = _problem(wl, pipeline=pipeline, snapshot_stride=50)
        if pair:
            swr.swr_set_schedule(pb.ctx, help_max=0, pair_from=1)
        else:
            swr.swr_set_schedule(pb.ctx, pair_from=9)
        u0 = to_dev(wl.u0)
        uT = torch.zeros_like(u0)
        g = torch.zeros((B, pb.ns, nt), dtype=torch.complex128, device=dev)
        tr = torch.zeros((B, wl.N, 2, nt + 1), dtype=torch.complex128, device=dev)
        sn = torch.zeros((B, nt // 50 + 1, wl.nx), dtype=torch.complex128, device=dev)
        st, info = swr.swr_solve(pb.ctx, u0, uT, g, tr, sn)
        assert st == swr.SWR_OK and info.residual < 1e-10
        dV = torch.zeros((B, wl.nx), dtype=torch.float64, device=dev)
        du0 = torch.zeros_like(u0)
        st2, _ = swr.swr_grad(pb.ctx, u0, (2.0 * uT).contiguous(), dV, du0)
        assert st2 == swr.SWR_OK
        torch.cuda.synchronize()
        out[pair] = [to_np(x) for x in (uT, g, tr, sn, dV, du0)]
        pb.close()
    for x, y in zip(out[False], out[True]):
        assert np.array_equal(x, y)
    for b in range(B):
        assert rel(out[True][0][b], O.mono(wl, wl.u0[b])) < 1e-10


GROUP_CASES = [
    # (label, J, nt, trans, sigma, B, pipeline, v_per_problem): a record's
    # tasks (2 impulse + B d tasks in the build list, B in the final list)
    # cut into ragged groups; widths 1 to 8
    ("s02-staged", [60, 90, 75, 128, 200, 47, 250, 480], 300, W.S02, 0j, 3, 0, False),
    ("s02-pipelined", [60, 90, 75, 128, 200, 47, 250], 300, W.S02, 0j, 5, 64, False),
    ("robin-staged", [50, 70, 300, 33, 500], 200, W.ROBIN, 1 - 1j, 3, 0, False),
    ("s02-v-per-problem", [60, 90, 200, 47], 200, W.S02, 0j, 3, 0, True),
]


@pytest.mark.parametrize("label,J,nt,trans,sigma,B,pipeline,vpp", GROUP_CASES)
def test_shared_factor_groups_equal_one_task_waves(dev, label, J, nt, trans, sigma, B, pipeline, vpp):
    """Sweeps that run the tasks of one factor record as the waves of one
    workgroup reading an LDS copy of the record (forced here for every width
    and launch size, group sizes 2, 3 and 8) perform each task's arithmetic
    exactly as one-task workgroups: u(T), g, end-node traces, snapshots and
    the adjoint's gradients are bitwise equal; u(T) matches the monodomain
    oracle."""
    import torch
    import oracle as O
    from paper_1503_02564_amd import swr
    from tests.gpu_util import rel
    wl = W.small_case(J=J, nt=nt, trans=trans, sigma=sigma, B=B, seed=31, a0=-12.0, b0=12.0)
    Vs = None
    if vpp:
        # one potential per problem: every record has its problem's task only
        # (and the two impulse tasks of each interface in the build list)
        Vs = np.stack([(1.0 + 0.25 * b) * np.asarray(wl.V) for b in range(B)])
        wl = W.Workload("pp", wl.a0, wl.b0, wl.J, wl.dt, wl.nt, W.V_STATIC, Vs, trans, sigma, wl.u0)
    out = {}
    for grp in (1, 2, 3, 8):
        say("shared-factor groups", label, "group", grp)
        pb = _problem(wl, pipeline=pipeline, snapshot_stride=50, v_per_problem=int(vpp))
        swr.swr_set_schedule(pb.ctx, help_max=0, group=grp)
        assert swr.swr_get_schedule(pb.ctx).group == grp
        u0 = to_dev(wl.u0)
        uT = torch.zeros_like(u0)
        g = torch.zeros((B, pb.ns, nt), dtype=torch.complex128, device=dev)
        tr = torch.zeros((B, wl.N, 2, nt + 1), dtype=torch.complex128, device=dev)
        sn = torch.zeros((B, nt // 50 + 1, wl.nx), dtype=torch.complex128, device=dev)
        st, info = swr.swr_solve(pb.ctx, u0, uT, g, tr, sn)
        assert st == swr.SWR_OK and info.residual < 1e-10
        dV = torch.zeros((B, wl.nx), dtype=torch.float64, device=dev)
        du0 = torch.zeros_like(u0)
        st2, _ = swr.swr_grad(pb.ctx, u0, (2.0 * uT).contiguous(), dV, du0)
        assert st2 == swr.SWR_OK
        torch.cuda.synchronize()
        out[grp] = [to_np(x) for x in (uT, g, tr, sn, dV, du0)]
        pb.close()
    names = ("uT", "g", "traces", "snapshots", "dJ/dV", "dJ/du0")
    for grp in (1, 2, 3, 8):
        for nm, x in zip(names, out[grp]):
            assert np.isfinite(x).all(), (nm, grp, np.argwhere(~np.isfinite(x))[:4].tolist())
    for grp in (2, 3, 8):
        for nm, x, y in zip(names, out[1], out[grp]):
            assert np.array_equal(x, y), (nm, grp)
    for b in range(B):
        ref = O.mono(wl, wl.u0[b], V=Vs[b]) if vpp else O.mono(wl, wl.u0[b])
        assert rel(out[8][0][b], ref) < 1e-10


def test_group_schedule_is_validated(dev):
    from paper_1503_02564_amd import swr
    wl = W.small_case(J=[60, 90], nt=64, B=2, seed=3)
    pb = _problem(wl)
    assert swr.swr_get_schedule(pb.ctx).group == 4
    for bad in (0, 9, -1):
        with pytest.raises(swr.SwrError):
            swr.swr_set_schedule(pb.ctx, group=bad)
    assert swr.swr_get_schedule(pb.ctx).group == 4
    pb.close()


@pytest.mark.parametrize("vkind", [W.V_STATIC, W.V_TIME])
def test_gmres_readback_period_changes_nothing(dev, vkind):
    """GMRES reads its residual estimates back every `check` inner steps:
    u(T), g, the iteration count and the residual history are bitwise those of
    a read-back after every step (static GMRES and the V(t,x) iteration)."""
    import torch
    from paper_1503_02564_amd import swr
    wl = W.small_case(J=[60, 90, 75, 128, 200, 47, 250], nt=200, vkind=vkind, trans=W.S02, sigma=0j,
                      B=3, seed=17, a0=-12.0, b0=12.0)
    out = {}
    for chk in (1, 3, 16):
        say("gmres check", vkind, chk)
        kw = dict(solver=swr.SWR_SOLVER_GMRES) if vkind == W.V_STATIC else {}
        pb = _problem(wl, tol=1e-12, **kw)
        swr.swr_set_schedule(pb.ctx, check=chk, restart=9)
        assert swr.swr_get_schedule(pb.ctx).check == chk
        u0 = to_dev(wl.u0)
        uT = torch.zeros_like(u0)
        g = torch.zeros((wl.B, pb.ns, wl.nt), dtype=torch.complex128, device=dev)
        st, info = swr.swr_solve(pb.ctx, u0, uT, g)
        assert st == swr.SWR_OK
        torch.cuda.synchronize()
        out[chk] = (to_np(uT), to_np(g), info.iters, info.history)
        pb.close()
    for chk in (3, 16):
        assert np.array_equal(out[1][0], out[chk][0]) and np.array_equal(out[1][1], out[chk][1])
        assert out[1][2] == out[chk][2] and np.array_equal(out[1][3], out[chk][3])
    assert out[1][2] > 9      # more than one restart cycle
