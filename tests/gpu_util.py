"""Helpers shared by the GPU parity tests: move seeded numpy inputs to the
device, build a context for a workload, compare against the oracle."""
import sys

import numpy as np


def say(*a):
    """Name the case before a GPU step (flushed, so a failing run shows it)."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def to_dev(x, dtype=None):
    import torch
    x = np.ascontiguousarray(x)
    t = torch.from_numpy(x)
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_np(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    b = np.asarray(b)
    return float(np.max(np.abs(np.asarray(a) - b)) / max(np.max(np.abs(b)), 1e-300))


def make_problem(wl, solver=None, tol=None, restart=None, max_iter=None, v_per_problem=False,
                 batch=None, precond=None, pipeline=None):
    from paper_1503_02564_amd import swr
    o = swr.swr_default_opts()
    o.batch = wl.B if batch is None else batch
    if solver is not None:
        o.solver = solver
    if tol is not None:
        o.tol = tol
    if restart is not None:
        o.restart = restart
    if max_iter is not None:
        o.max_iter = max_iter
    o.v_per_problem = int(v_per_problem)
    if precond is not None:
        o.precond = int(precond)
    if pipeline is not None:
        o.pipeline = int(pipeline)
    o.pade_m = int(wl.pade_m)
    o.pade_theta = float(wl.pade_theta)
    V = None if wl.V is None else to_dev(np.asarray(wl.V, np.float64))
    return swr.Problem(wl.a0, wl.b0, tuple(int(j) for j in wl.J), wl.dt, wl.dt * wl.nt, wl.vkind,
                       wl.trans, wl.sigma, o, V)
