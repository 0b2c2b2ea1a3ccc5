"""swr_apply_R_noalloc (the entry point for callers that cannot allocate)
against swr_apply_R, through the C ABI: two calls in a row on two contexts,
the second with a smaller problem (fewer subdomains, fewer steps, fewer
problems) so that it reuses the library's static scratch after a larger
call; g_out, u(T) and the max change must equal swr_apply_R's bit for bit
(same kernels, same order of operations).  Also: a problem whose scratch
would exceed the fixed size is refused with SWR_EINVAL."""
import numpy as np
import pytest

from paper_1503_02564_amd import workloads as W
from tests.gpu_util import say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _ctx(wl, trans):
    from paper_1503_02564_amd import swr
    o = swr.swr_default_opts()
    o.batch = wl.B
    return swr.Problem(wl.a0, wl.b0, tuple(int(j) for j in wl.J), wl.dt, wl.dt * wl.nt, wl.vkind,
                       trans, wl.sigma, o, to_dev(np.asarray(wl.V, np.float64)))


@pytest.mark.parametrize("trans", [1, 0])   # S0^2 (history in the scratch), Robin
def test_noalloc_equals_apply_R_twice_shrinking(dev, trans):
    import torch
    from paper_1503_02564_amd import swr
    cases = [W.small_case(J=[60, 90, 75, 128, 47, 100], nt=300, B=3, seed=21, a0=-10.0, b0=10.0),
             W.small_case(J=[33, 41, 29], nt=70, B=2, seed=22, a0=-5.0, b0=5.0)]
    for ci, wl in enumerate(cases):
        say("noalloc", "trans", trans, "case", ci, "N", wl.N, "nt", wl.nt, "B", wl.B)
        pb = _ctx(wl, trans)
        rng = np.random.default_rng(100 + ci)
        gin = rng.standard_normal((wl.B, pb.ns, wl.nt)) + 1j * rng.standard_normal((wl.B, pb.ns, wl.nt))
        g_in = to_dev(gin)
        u0 = to_dev(wl.u0)
        out = {}
        for name in ("ref", "noalloc"):
            g_out = torch.full_like(g_in, complex(np.nan, np.nan))
            uT = torch.full_like(u0, complex(np.nan, np.nan))
            if name == "ref":
                md = swr.swr_apply_R(pb.ctx, u0, g_in, g_out, uT, want_maxdiff=True)
            else:
                mdt = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
                swr.swr_apply_R_noalloc(pb.ctx, u0, g_in, g_out, uT, mdt)
                torch.cuda.synchronize()
                md = float(mdt.item())
            out[name] = (to_np(g_out), to_np(uT), md)
        a, b = out["ref"], out["noalloc"]
        assert np.all(np.isfinite(b[0])) and np.all(np.isfinite(b[1]))
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2], ci
        pb.close()


def test_noalloc_refuses_problems_beyond_its_scratch(dev):
    import torch
    from paper_1503_02564_amd import swr
    # 40 x 8 problems of 2001 steps: 2 * 320 * 2002 * 16 B = 20.5 MB of history > 16 MiB
    wl = W.small_case(J=[20] * 40, nt=2000, B=8, seed=23, a0=-10.0, b0=10.0)
    pb = _ctx(wl, 1)
    g = torch.zeros((wl.B, pb.ns, wl.nt), dtype=torch.complex128, device=dev)
    with pytest.raises(swr.SwrError) as e:
        swr.swr_apply_R_noalloc(pb.ctx, to_dev(wl.u0), g, torch.zeros_like(g))
    assert e.value.status == swr.SWR_EINVAL
    pb.close()
