"""The paper's own workloads (Sec. 6) at its largest decomposition: (-21, 21),
T = 0.5, dt = 1e-3 (500 steps), N = 1000 subdomains, S0^2; V = -x^2 (new
algorithm), V = 5 t x (preconditioned GMRES) and |u|^2 with the sech soliton
(preconditioned fixed point), on the paper's two grids: mesh size 1e-4
(420000 cells, subdomains of 420 cells: the register sweep) and 1e-5 (4.2
million cells, subdomains of 4200 cells: the long-chunk sweep, 66 nodes per
lane).  999 interfaces: the causal solve runs in its 1024-thread workgroup
form (the per-step block system is block diagonally dominant at these
subdomain widths), for the static system and as P^{-1}.

Reference: the monodomain Crank-Nicolson solution in extended precision,
sampled every 200 (2000) nodes (tests/golden/paper_scale_*.txt, written by
make_paper_scale.py from the oracle).  At these grids (dt/h^2 = 1e5 and 1e7)
FP64 time stepping itself loses accuracy: the plain FP64 monodomain sweep of
the oracle is off by the amount recorded in each fixture.  The bar
is max(1e-10, 10 x that recorded error): a decomposed FP64 solve may carry up
to ten times the rounding of the plain sweep it replaces, no more, so a
kernel regression of ten times fails.
Iteration counts at the paper's tolerance 1e-10, and those of BiCGStab on the
static system, are printed beside the paper's (context only: its counts are
for its own grids and initial vectors).
"""
import time

import numpy as np
import pytest

from paper_1503_02564_amd import workloads as W
from tests.golden.make_paper_scale import read_fixture
from tests.gpu_util import make_problem, say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _run(dev, wl, **kw):
    import torch
    from paper_1503_02564_amd import swr
    pb = make_problem(wl, **kw)
    uT = torch.zeros((1, wl.nx), dtype=torch.complex128, device=dev)
    u0 = to_dev(wl.u0)
    t0 = time.perf_counter()
    st, info = swr.swr_solve(pb.ctx, u0, uT)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0)
    pb.close()
    return st, info, to_np(uT)[0], ms


GRIDS = [pytest.param(1e-4, id="dx1e-4"), pytest.param(1e-5, id="dx1e-5")]


def _check(kind, wl, uT, dx):
    idx, ref, scale, err64 = read_fixture(kind, dx)
    err = float(np.max(np.abs(uT[idx] - ref)) / scale)
    bar = max(1e-10, 10.0 * err64)
    say("paper-scale", kind, "rel err vs extended-precision monodomain", err,
        "FP64 monodomain oracle's own error", err64, "bar", bar)
    assert abs(np.max(np.abs(uT)) - scale) <= bar * scale
    assert err <= bar


@pytest.mark.parametrize("dx", GRIDS)
def test_paper_harmonic_potential_new_algorithm(dev, dx):
    from paper_1503_02564_amd import swr
    wl = W.paper_case("harmonic", dx=dx)
    say("paper-scale", "harmonic", "N", wl.N, "nx", wl.nx)
    st, info, uT, ms = _run(dev, wl, tol=1e-10)
    say("paper-scale", "harmonic", "causal: status", st, "iterations", info.iters,
        "residual", info.residual, "ms", ms)
    assert st == swr.SWR_OK and info.iters == 1
    assert info.residual < 1e-11
    _check("harmonic", wl, uT, dx)
    st, info, _, ms = _run(dev, wl, solver=swr.SWR_SOLVER_BICGSTAB, tol=1e-10, max_iter=5000)
    say("paper-scale", "harmonic", "BiCGStab tol 1e-10: status", st, "iterations", info.iters,
        "ms", ms)
    assert st == swr.SWR_OK


@pytest.mark.parametrize("dx", GRIDS)
def test_paper_linear_time_potential_preconditioned(dev, dx):
    from paper_1503_02564_amd import swr
    wl = W.paper_case("linear_t", dx=dx)
    say("paper-scale", "5tx", "N", wl.N)
    st, info, _, ms = _run(dev, wl, tol=1e-10, restart=100, max_iter=400)
    say("paper-scale", "5tx", "tol 1e-10: status", st, "GMRES iterations", info.iters,
        "(paper: 25 at this N and grid)", "ms", ms)
    st, info, uT, ms = _run(dev, wl, tol=1e-12, restart=100, max_iter=400)
    say("paper-scale", "5tx", "tol 1e-12: status", st, "iterations", info.iters,
        "residual", info.residual, "ms", ms)
    assert st == swr.SWR_OK
    _check("linear_t", wl, uT, dx)


@pytest.mark.parametrize("dx", GRIDS)
def test_paper_cubic_soliton_preconditioned(dev, dx):
    from paper_1503_02564_amd import swr
    wl = W.paper_case("cubic", dx=dx)
    say("paper-scale", "cubic", "N", wl.N)
    st, info, _, ms = _run(dev, wl, tol=1e-10, max_iter=300)
    say("paper-scale", "cubic", "tol 1e-10: status", st, "fixed-point iterations", info.iters,
        "(paper: 26 at this N on its finer grid)", "worst inner", info.nl_worst, "ms", ms)
    st, info, uT, ms = _run(dev, wl, tol=1e-12, max_iter=300)
    say("paper-scale", "cubic", "tol 1e-12: status", st, "iterations", info.iters, "ms", ms)
    assert st == swr.SWR_OK
    _check("cubic", wl, uT, dx)
