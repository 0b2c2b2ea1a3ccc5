"""Benchmark: grid-point x time-step throughput of one SWR solve to interface
residual 1e-10 on one MI355X.

Workload (default): a time-independent potential on (-40, 40), 16384 cells in
64 equal subdomains, 2000 Crank-Nicolson steps (dt = 5e-4), S0^2 transmission,
seeded potential (-0.05 x^2 + 8 Gaussian bumps) and packet.  One "step" is one
full solve of the paper's new algorithm (Sec. 4): assembly + factorisation,
all impulse sweeps and the d sweeps (one launch per time chunk), the causal
interface solve and the final sweep -> u(T), the three stages overlapped
chunk by chunk (--pipeline 0 runs them one after the other).  Inputs are
resident in HBM before the timed region.

Second figure of the metric: the adjoint/forward cost ratio on the
differentiation workload ((-40,40), 256 subdomains of 64 cells, 2000 steps,
16 seeded potentials, one per problem, J = ||u(T) - u*||^2 with u* from a
seeded reference potential): T(swr_grad) - T(swr_solve) over T(swr_solve),
both to interface residual 1e-10.

Output: one JSON line (see the keys below).  The roofline object describes the
dominant kernel (the subdomain sweep); the cpu_baseline object times the CPU
oracle on the host on the same workload.

``--calibrate-copy MIB`` only runs a plain device-to-device copy of MIB MiB
five times (the reference kernel that scales the HBM byte counters).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 peak of the MI355X vector ALUs (published): 78.6 TFLOP/s
PEAK_FP64_TFLOPS = 78.6


def sweep_flops_per_pt_step(wl) -> float:
    """Algorithmic FP64 flops of one grid point advanced one step in a
    subdomain sweep: c M u_{n-1} (8), Thomas forward (14) and backward (8)
    with precomputed factors, u_n = 2 v_n - u_{n-1} (4).  The S0^2 history
    adds 2 ends x n real-by-complex MACs at step n, i.e. 4 (nt+1)/(J+1) per
    point-step on average."""
    base = 34.0
    if wl.trans == 1:
        base += 4.0 * (wl.nt + 1) / (float(np.mean(wl.J)) + 1.0)
    return base


SWEEP_SOURCES = ("paper_1503_02564_amd/csrc/swr_sweep_kernel.h", "paper_1503_02564_amd/csrc/swr_lane.h",
                 "paper_1503_02564_amd/csrc/swr_sweep_static.hip", "paper_1503_02564_amd/csrc/swr_sweep_static_s02.hip",
                 "paper_1503_02564_amd/csrc/swr_sweep.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_kernel_static_64x256_hbm.txt")


def sweep_source_hash() -> str:
    """sha256 over the sources of the static sweep kernel: a traffic figure
    measured on other sources is not reported."""
    import hashlib
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(pipeline):
    """HBM bytes per sweep launch from the committed counter summary (two
    rocprofv3 --pmc passes, FETCH_SIZE and WRITE_SIZE, each scaled by what the
    counter reads for a plain copy of known size), or None when the summary
    is missing, was taken with another pipeline chunk, or the kernel sources
    changed since."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith(("#", " ", "|")):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_sha256") != sweep_source_hash() or int(kv.get("pipeline", -1)) != pipeline:
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(wl, budget_s=30.0):
    """Time the oracle (as it stands) on the host for the same workload: the
    new algorithm with the causal interface solve, single thread."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    import oracle as O
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    runs, t_all = 0, 0.0
    try:
        while runs == 0 or t_all < 0.5 * budget_s:
            t0 = time.perf_counter()
            uT, g, info = O.new_algorithm(wl, wl.u0[0], solver="causal")
            t_all += time.perf_counter() - t0
            runs += 1
    finally:
        if ctx is not None:
            ctx.unregister() if hasattr(ctx, "unregister") else None
    dt = t_all / runs
    pts = wl.nx * wl.nt
    return dict(value=pts / dt, unit="pt-steps/s", cores=1, kind="oracle",
                sample=f"{runs} full solve(s) of the same workload (batch member 0) by the "
                       f"oracle (impulse columns, d, causal interface solve, final sweep), "
                       f"{dt:.2f} s each, single-threaded", residual=float(info["residual"])), uT


def adjoint_ratio(steps, warmup):
    """Adjoint/forward cost ratio on the differentiation workload (16
    potentials, one per problem, 256 subdomains).  Forward = swr_solve;
    backward = swr_grad minus the forward it contains (swr_grad re-runs the
    forward with checkpoints).  Wall clock around synchronised calls."""
    import torch
    from paper_1503_02564_amd import swr
    from paper_1503_02564_amd import workloads as W
    wl = W.adjoint_batch()
    dev = torch.device("cuda:0")

    def opts(B, per_problem):
        o = swr.swr_default_opts()
        o.tol = wl.tol
        o.batch = B
        o.v_per_problem = int(per_problem)
        o.checkpoint_K = 64
        return o

    J = tuple(int(j) for j in wl.J)
    T = wl.dt * wl.nt
    u0 = torch.from_numpy(np.ascontiguousarray(wl.u0)).to(dev)
    # target state from the reference potential (outside the timed region)
    Vr = torch.from_numpy(np.ascontiguousarray(wl.extras["V_ref"])).to(dev)
    ref = swr.Problem(wl.a0, wl.b0, J, wl.dt, T, wl.vkind, wl.trans, wl.sigma, opts(1, False), Vr)
    u_star = torch.zeros_like(u0[:1])
    swr.swr_solve(ref.ctx, u0[:1].contiguous(), u_star)
    ref.close()
    V = torch.from_numpy(np.ascontiguousarray(wl.V)).to(dev)
    pb = swr.Problem(wl.a0, wl.b0, J, wl.dt, T, wl.vkind, wl.trans, wl.sigma, opts(wl.B, True), V)
    uT = torch.zeros_like(u0)
    swr.swr_solve(pb.ctx, u0, uT)
    gbar = (2.0 * (uT - u_star)).contiguous()
    dV = torch.zeros_like(V)
    du0 = torch.zeros_like(u0)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = [fn() for _ in range(steps)]
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / steps, out

    t_fwd, fi = timed(lambda: swr.swr_solve(pb.ctx, u0, uT)[1].as_dict())
    t_grad, gi = timed(lambda: swr.swr_grad(pb.ctx, u0, gbar, dV, du0)[1].as_dict())
    ph = {k: float(np.mean([i[k] for i in gi])) for k in
          ("t_factor_ms", "t_build_ms", "t_iface_ms", "t_final_ms")}
    bwd_events = ph["t_build_ms"] + ph["t_iface_ms"] + ph["t_final_ms"]
    res = dict(
        workload="(-40,40), 256 x 64 cells, 2000 steps dt=5e-4, S0^2, 16 seeded potentials "
                 "(one per problem), J = ||u(T)-u*||^2, checkpoints every 64 steps",
        fwd_ms=t_fwd, grad_ms=t_grad,
        ratio_bwd_over_fwd=(t_grad - t_fwd) / t_fwd,
        ratio_fwd_plus_bwd_over_fwd=t_grad / t_fwd,
        ratio_events_bwd_over_fwd=bwd_events / ph["t_factor_ms"],
        grad_phases_ms=ph,
        fwd_residual=max(i["residual"] for i in fi),
        adj_residual=max(i["residual"] for i in gi),
        fwd_pt_steps_per_s=wl.pt_steps() / (1e-3 * t_fwd))
    pb.close()
    return res


# the paper's own figures for these workloads (Sec. 6 tables; 1000 MPI
# processes on its CPU cluster): context, not a target
PAPER_CONTEXT = {
    "harmonic": "new algorithm, N = 1000, dx = 1e-5: 7.12 s (BiCGStab), 8.17 s (GMRES)",
    "linear_t": "preconditioned, N = 1000, dx = 1e-4: 25 iterations, 54.5 s",
    "cubic": "preconditioned, N = 1000, dx = 1e-5: 26 iterations, 83.8 s",
}


def paper_workloads(reps=3):
    """The paper's Sec. 6 workloads on its dx = 1e-4 grid at N = 1000
    (420001 nodes, 500 steps): wall time per solve (median of reps after one
    warm-up), iterations at interface tolerance 1e-10."""
    import torch
    from paper_1503_02564_amd import swr
    from paper_1503_02564_amd import workloads as W
    out = {}
    for kind in ("harmonic", "linear_t", "cubic"):
        wl = W.paper_case(kind)
        o = swr.swr_default_opts()
        o.tol = 1e-10
        o.restart = 100
        o.max_iter = 400
        dev = torch.device("cuda:0")
        V = None if wl.V is None else torch.from_numpy(np.ascontiguousarray(wl.V)).to(dev)
        pb = swr.Problem(wl.a0, wl.b0, tuple(int(j) for j in wl.J), wl.dt, wl.dt * wl.nt, wl.vkind,
                         wl.trans, wl.sigma, o, V)
        u0 = torch.from_numpy(np.ascontiguousarray(wl.u0)).to(dev)
        uT = torch.zeros_like(u0)
        swr.swr_solve(pb.ctx, u0, uT)
        torch.cuda.synchronize()
        ts, info = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            st, info = swr.swr_solve(pb.ctx, u0, uT)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ms = 1e3 * float(np.median(ts))
        out[kind] = {"ms_per_solve": ms, "iterations": info.iters, "status": st,
                     "pt_steps_per_s": wl.pt_steps() / (ms * 1e-3),
                     "interface_residual": info.residual, "paper": PAPER_CONTEXT[kind]}
        pb.close()
        del V
    out["workload"] = ("(-21,21), dx = 1e-4 (420001 nodes), dt = 1e-3, 500 steps, N = 1000 x 420 "
                       "cells, S0^2; V = -x^2 (causal interface solve), V = 5tx (GMRES preconditioned "
                       "by I - L_0), |u|^2 sech soliton (preconditioned fixed point)")
    return out


def filled_roofline(reps=3):
    """The sweep kernel where its launches fill the GPU: the batched-uneven
    workload ((-100,100), 500 subdomains of U{40..400} cells, 32 problems,
    2000 steps, S0^2; 16998 build tasks and 16000 final-sweep tasks per
    solve).  Algorithmic flops per task: 34 per point-step plus the S0^2
    history, 4 nt (nt + 1) per task; time: the library's HIP-event sum over
    the sweep launches (median solve of reps after one warm-up)."""
    import torch
    from paper_1503_02564_amd import swr
    from paper_1503_02564_amd import workloads as W
    wl = W.batched_uneven()
    dev = torch.device("cuda:0")
    o = swr.swr_default_opts()
    o.batch = wl.B
    o.tol = wl.tol
    V = torch.from_numpy(np.ascontiguousarray(wl.V)).to(dev)
    pb = swr.Problem(wl.a0, wl.b0, tuple(int(j) for j in wl.J), wl.dt, wl.dt * wl.nt, wl.vkind,
                     wl.trans, wl.sigma, o, V)
    u0 = torch.from_numpy(np.ascontiguousarray(wl.u0)).to(dev)
    uT = torch.zeros_like(u0)
    swr.swr_solve(pb.ctx, u0, uT)
    torch.cuda.synchronize()
    infos, walls = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        st, info = swr.swr_solve(pb.ctx, u0, uT)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        infos.append(info.as_dict())
    pb.close()
    i = int(np.argsort([x["t_sweep_ms"] for x in infos])[len(infos) // 2])
    info = infos[i]
    N, nt, B = wl.N, wl.nt, wl.B
    flops = 0.0
    for k in range(N):
        ntask = int(k > 0) + int(k < N - 1) + 2 * B
        flops += ntask * (34.0 * (int(wl.J[k]) + 1) * nt + 4.0 * nt * (nt + 1))
    achieved = flops / (1e-3 * info["t_sweep_ms"]) / 1e12
    return {"workload": "batched_uneven: (-100,100), 500 subdomains U{40..400} cells, 32 problems, "
                        "2000 steps, S0^2, causal interface solve",
            "bound": "alu", "kernel": "sweep_kernel", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
            "sweep_ms_per_solve": info["t_sweep_ms"], "launches_per_solve": info["n_sweep"],
            "ms_per_solve": 1e3 * float(np.median(walls)),
            "pt_steps_per_s": wl.pt_steps() / float(np.median(walls)), "status": st}


def batched_vs_plain(batched_ms):
    """The same benchmark solve with every sweep task launched on its own
    (one subdomain of one problem per launch, one stream, staged), against
    the batched and pipelined form: same kernels, same interface solve, same
    certified residual."""
    import torch
    from paper_1503_02564_amd import swr
    from paper_1503_02564_amd import workloads as W
    wl = W.static_packet()
    dev = torch.device("cuda:0")
    o = swr.swr_default_opts()
    o.tol = wl.tol
    o.plain = 1
    V = torch.from_numpy(np.ascontiguousarray(wl.V)).to(dev)
    u0 = torch.from_numpy(np.ascontiguousarray(wl.u0)).to(dev)
    uT = torch.zeros_like(u0)
    pb = swr.Problem(wl.a0, wl.b0, tuple(int(j) for j in wl.J), wl.dt, wl.dt * wl.nt, wl.vkind,
                     wl.trans, wl.sigma, o, V)
    swr.swr_solve(pb.ctx, u0, uT)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, info = swr.swr_solve(pb.ctx, u0, uT)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0)
    pb.close()
    return dict(plain_ms_per_solve=ms, batched_ms_per_solve=batched_ms,
                speedup_batched_over_plain=ms / batched_ms, plain_residual=info.residual,
                launches_plain=int(2 * wl.N * wl.B + 2 * wl.N - 2))


def calibrate_copy(mib):
    """A plain copy of a known size, for scaling the HBM byte counters."""
    import torch
    n = int(mib) * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_read": 8 * n, "calibrate_copy_bytes_written": 8 * n,
                      "launches": 5}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--solver", default="causal", choices=["causal", "gmres", "bicgstab", "fixed"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--pipeline", type=int, default=256,
                    help="steps per pipeline chunk of the causal solve (0 = staged)")
    ap.add_argument("--workload", default="static_packet", choices=["static_packet"])
    ap.add_argument("--no-paper", dest="paper", action="store_false",
                    help="skip the paper's Sec. 6 workloads at N = 1000 and the filled-GPU roofline point")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward ratio on the differentiation workload")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain MIB-MiB device copy (counter calibration)")
    ap.add_argument("--no-plain", dest="plain", action="store_false",
                    help="skip the one-launch-per-subdomain comparison")
    ap.add_argument("--source-hash", action="store_true",
                    help="print the sweep kernel source hash and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "only --gpus 1 is supported: the solver runs on one GPU "
                                   "and has no multi-GPU sharding", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.source_hash:
        print(sweep_source_hash())
        return
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return

    import torch
    from paper_1503_02564_amd import swr
    from paper_1503_02564_amd import workloads as W

    wl = W.static_packet()
    dev = torch.device("cuda:0")
    o = swr.swr_default_opts()
    o.solver = dict(causal=swr.SWR_SOLVER_CAUSAL, gmres=swr.SWR_SOLVER_GMRES,
                    bicgstab=swr.SWR_SOLVER_BICGSTAB, fixed=swr.SWR_SOLVER_FIXED)[args.solver]
    o.tol = wl.tol
    o.pipeline = args.pipeline
    V = torch.from_numpy(np.ascontiguousarray(wl.V)).to(dev)
    u0 = torch.from_numpy(np.ascontiguousarray(wl.u0)).to(dev)
    uT = torch.zeros_like(u0)
    pb = swr.Problem(wl.a0, wl.b0, tuple(int(j) for j in wl.J), wl.dt, wl.dt * wl.nt, wl.vkind,
                     wl.trans, wl.sigma, o, V)
    for _ in range(args.warmup):
        swr.swr_solve(pb.ctx, u0, uT)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, info = swr.swr_solve(pb.ctx, u0, uT)
        infos.append(info.as_dict())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = 1e3 * wall / args.steps
    pts = wl.pt_steps()
    value = pts / (wall / args.steps)
    ph = {k: float(np.mean([i[k] for i in infos])) for k in
          ("t_factor_ms", "t_build_ms", "t_iface_ms", "t_final_ms", "t_total_ms")}
    resid = max(i["residual"] for i in infos)

    # dominant kernel: the subdomain sweep.  The library brackets every sweep
    # launch (impulse/d sweeps and final sweep, per pipeline chunk) with HIP
    # events on the stream it runs on and reports their summed duration.
    fpp = sweep_flops_per_pt_step(wl)
    n_build = (2 * wl.N - 2) + wl.N * wl.B        # impulse sweeps + d sweeps
    n_final = wl.N * wl.B
    pts_per_sweep = float(np.mean(wl.J + 1)) * wl.nt
    flops = fpp * pts_per_sweep * (n_build + n_final)   # per solve
    n_launch = float(np.mean([i["n_sweep"] for i in infos]))
    t_sweep_ms = float(np.mean([i["t_sweep_ms"] for i in infos]))
    achieved = flops / (1e-3 * t_sweep_ms) / 1e12
    roof = {"bound": "alu", "kernel": "sweep_kernel",
            "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": measured_traffic(args.pipeline if args.solver == "causal" else 0),
            "avg_launch_ms": t_sweep_ms / n_launch, "launches_per_solve": n_launch,
            "flops_per_launch": flops / n_launch, "flops_per_pt_step": fpp}

    plain = None
    if args.plain:
        plain = batched_vs_plain(ms)

    paper = paper_workloads() if args.paper else None
    filled = filled_roofline() if args.paper else None

    adj = None
    if not args.no_adjoint:
        adj = adjoint_ratio(max(1, min(args.steps, 5)), 1)

    cpu = None
    if not args.no_cpu:
        cpu, u_cpu = cpu_baseline(wl)
        got = uT.cpu().numpy()[0]
        cpu["max_rel_diff_gpu_vs_oracle"] = float(np.max(np.abs(got - u_cpu)) / np.max(np.abs(u_cpu)))

    out = {
        "metric": "grid-point*time-steps/s to interface residual 1e-10; adjoint/forward cost ratio",
        "value": value, "unit": "pt-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "static_packet: (-40,40), 64x256 cells, 2000 steps dt=5e-4, S0^2, "
                               "seeded bumpy harmonic V and packet, new algorithm, "
                               f"{args.solver} interface solve",
                   "nx": wl.nx, "nt": wl.nt, "N": wl.N, "B": wl.B, "solver": args.solver,
                   "pipeline": args.pipeline if args.solver == "causal" else 0},
        "interface_residual": resid, "phases_ms": ph,
        "batched_vs_plain": plain,
        "adjoint_forward_cost_ratio": None if adj is None else adj["ratio_bwd_over_fwd"],
        "adjoint": adj,
        "paper_workloads": paper,
        "roofline_filled": filled,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    pb.close()


if __name__ == "__main__":
    main()
