"""Benchmark: grid-point x time-step throughput of SWR solves to interface
residual 1e-10 on one MI355X.

Headline workload (default): the batched uneven decomposition -- (-100, 100),
500 subdomains of seeded sizes U{40..400} cells (109113 nodes), time-
independent potential, 32 independent seeded packets solved in one batch,
2000 Crank-Nicolson steps (dt = 5e-4), S0^2 transmission.  One "step" is one
full solve of the paper's new algorithm (Sec. 4) for the whole batch:
assembly + factorisation, every impulse sweep and d sweep, the causal
interface solve and the final sweep -> u(T), the three stages overlapped
chunk by chunk.  Inputs are resident in HBM before the timed region.

value = 32 x 109113 x 2000 grid-point x time-steps per solve / seconds per
solve.  In the same JSON line:
* roofline: the dominant kernel (the subdomain sweep) on the headline run:
  algorithmic flops per launch / average launch duration (HIP events the
  library records around every sweep launch, on the stream it runs on);
  traffic from the committed counter summary while the kernel sources hash
  the same;
* secondary: the static-packet workload ((-40,40), 64 x 256 cells, one
  problem) with the causal, GMRES and BiCGStab interface solvers; the
  time-dependent (V = 5 x cos t, preconditioned GMRES) and cubic (|u|^2,
  preconditioned fixed point) workloads on 128 x 256 cells over 4000 steps;
  the adjoint/forward cost ratio on the differentiation workload; the
  batched form against one launch per subdomain; the paper's Sec. 6
  workloads at N = 1000;
* cpu_baseline: the oracle's monodomain Crank-Nicolson solve (the paper's
  T_ref analogue) of headline batch member 0 over its first 500 steps on one
  pinned host core.

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
# the oracle's CPU sample: whole monodomain solves of batch members 0, 1, ...
# until at least CPU_MIN_S seconds of CPU work
CPU_MIN_S = 10.0


FAR_SUPER = 256   # super-chunk of the S0^2 far history (kFarSuper in the library)


def far_terms(nt):
    """S0^2 history terms per end of one task: all of them (output step n
    adds n terms, n = 1..nt), and the old parts that the library's batched
    product computes per super-chunk (output n in the 64-step block n0 of
    the super-chunk C = n0 - n0 % 256 takes q <= C - 65 from it)."""
    n = np.arange(1, nt + 1)
    n0 = 64 * ((n - 1) // 64)
    C = n0 - n0 % FAR_SUPER
    return float(n.sum()), float(np.maximum(0, C - 64).sum())


def sweep_task_flops(J_cells, nt, trans):
    """Algorithmic FP64 flops of one sweep task (one subdomain of one
    problem over nt steps): c M u_{n-1} (8), Thomas forward (14) and backward
    (8) with precomputed factors, u_n = 2 v_n - u_{n-1} (4) per point-step,
    plus the S0^2 history: at step n, 2 ends x n real-by-complex MACs (4
    flops each), i.e. 4 nt (nt + 1) per task -- summed partly by the sweep
    kernel, partly (the super-chunks' old parts) by far_old_kernel between
    its launches."""
    f = 34.0 * (float(J_cells) + 1.0) * nt
    if trans == 1:
        f += 4.0 * nt * (nt + 1.0)
    return f


def far_old_flops(wl):
    """Algorithmic flops of the old far-history parts of one solve (the
    batched Toeplitz products on the matrix cores): every task of the
    impulse, d and final lists, 2 ends x 4 flops per term."""
    if wl.trans != 1:
        return 0.0
    N, B = wl.N, wl.B
    ntask = sum(int(k > 0) + int(k < N - 1) + 2 * B for k in range(N))
    return 8.0 * far_terms(wl.nt)[1] * ntask


def solve_sweep_pt_steps(wl):
    """Point-steps swept in one solve (impulse, d and final sweeps)."""
    N, B = wl.N, wl.B
    return float(sum((int(k > 0) + int(k < N - 1) + 2 * B) * (int(wl.J[k]) + 1) * wl.nt
                     for k in range(N)))


def solve_flops(wl):
    """Sweep flops of one solve of the new algorithm: every impulse sweep
    (2 per interface), and per problem one d sweep and one final sweep of
    every subdomain."""
    N, B = wl.N, wl.B
    tot = 0.0
    for k in range(N):
        ntask = int(k > 0) + int(k < N - 1) + 2 * B
        tot += ntask * sweep_task_flops(wl.J[k], wl.nt, wl.trans)
    return tot


SWEEP_SOURCES = ("paper_1503_02564_amd/csrc/swr_sweep_kernel.h", "paper_1503_02564_amd/csrc/swr_lane.h",
                 "paper_1503_02564_amd/csrc/swr_sweep_static.hip",
                 "paper_1503_02564_amd/csrc/swr_sweep_static_s02.hip",
                 "paper_1503_02564_amd/csrc/swr_sweep_group.hip",
                 "paper_1503_02564_amd/csrc/swr_sweep.hip",
                 "paper_1503_02564_amd/csrc/swr_common.h",
                 "paper_1503_02564_amd/csrc/swr_host.hip",
                 "paper_1503_02564_amd/build.py")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_kernel_batched_uneven_hbm.txt")


def sweep_source_hash() -> str:
    """sha256 over the sources and build flags of the static sweep kernel and
    the far-history product between its launches, and the host code that
    cuts the launches: a traffic figure measured on other code is not
    reported."""
    import hashlib
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per sweep launch from the committed counter summary (two
    rocprofv3 --pmc passes, FETCH_SIZE and WRITE_SIZE, each scaled by what the
    counter reads for a plain copy of known size), or None when the summary
    is missing or the kernel sources changed since."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith(("#", " ", "|")):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_sha256") != sweep_source_hash():
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def make_problem(wl, **kw):
    import torch
    from paper_1503_02564_amd import swr
    o = swr.swr_default_opts()
    o.batch = wl.B
    o.tol = wl.tol
    for k, v in kw.items():
        setattr(o, k, v)
    V = None if wl.V is None else torch.from_numpy(np.ascontiguousarray(wl.V)).cuda()
    return swr.Problem(wl.a0, wl.b0, tuple(int(j) for j in wl.J), wl.dt, wl.dt * wl.nt, wl.vkind,
                       wl.trans, wl.sigma, o, V)


def timed_solves(wl, steps, warmup, tune_ms=0.0, sched=None, **kw):
    """Wall time per solve (synchronised around `steps` solves after
    `warmup`), the infos of the timed solves, the last u(T) and status.  With
    tune_ms > 0 the library's autotuner first picks the schedule (outside the
    timed region); sched (a dict) receives the schedule the solves ran with."""
    import torch
    from paper_1503_02564_amd import swr
    pb = make_problem(wl, **kw)
    u0 = torch.from_numpy(np.ascontiguousarray(wl.u0)).cuda()
    uT = torch.zeros_like(u0)
    if tune_ms > 0:
        swr.swr_tune(pb.ctx, u0, tune_ms)
    if sched is not None:
        sched.update(swr.swr_get_schedule(pb.ctx).as_dict())
    st = None
    for _ in range(warmup):
        st, _ = swr.swr_solve(pb.ctx, u0, uT)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        st, info = swr.swr_solve(pb.ctx, u0, uT)
        infos.append(info.as_dict())
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / max(steps, 1)
    pb.close()
    return ms, infos, uT.cpu().numpy(), st


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(wl):
    """The oracle as it stands: its monodomain Crank-Nicolson solve (the
    definition every decomposed solve converges to; the paper's T_ref, Sec. 6)
    of batch members 0, 1, ... over all steps, one member after the other
    until at least CPU_MIN_S seconds have passed, single-threaded on one
    pinned host core (the C core is single-threaded)."""
    import oracle as O
    try:
        os.sched_setaffinity(0, {sorted(os.sched_getaffinity(0))[0]})
    except (AttributeError, OSError):
        pass
    members = 0
    t0 = time.perf_counter()
    while members < wl.B and (members == 0 or time.perf_counter() - t0 < CPU_MIN_S):
        O.mono(wl, wl.u0[members])
        members += 1
    dt = time.perf_counter() - t0
    model, ncpu = cpu_info()
    return dict(value=wl.nx * wl.nt * members / dt, unit="pt-steps/s", cores=1, kind="oracle",
                sample=f"monodomain Crank-Nicolson (the paper's T_ref) of batch members "
                       f"0..{members - 1}, all {wl.nt} steps each ({wl.nx} nodes), {dt:.2f} s, "
                       f"one pinned core",
                cpu_model=model, nproc=ncpu)


def static_packet_solvers(steps):
    """The static-packet workload with each interface solver: ms per solve,
    iterations, certified residual; the causal run also gives the sweep
    kernel's roofline point on a single problem."""
    from paper_1503_02564_amd import swr
    from paper_1503_02564_amd import workloads as W
    wl = W.static_packet()
    out = {"workload": "static_packet: (-40,40), 64x256 cells, 2000 steps dt=5e-4, S0^2, one "
                       "problem, new algorithm"}
    for name, solver, reps in (("causal", swr.SWR_SOLVER_CAUSAL, steps),
                               ("bicgstab", swr.SWR_SOLVER_BICGSTAB, 2),
                               ("gmres", swr.SWR_SOLVER_GMRES, 2)):
        ms, infos, _, st = timed_solves(wl, reps, 1, solver=solver)
        out[name] = {"ms_per_solve": ms, "iterations": infos[-1]["iters"],
                     "interface_residual": infos[-1]["residual"], "status": st,
                     "pt_steps_per_s": wl.pt_steps() / (1e-3 * ms)}
        if name == "causal":
            t_sweep = float(np.mean([i["t_sweep_ms"] for i in infos]))
            n_sweep = float(np.mean([i["n_sweep"] for i in infos]))
            fl = solve_flops(wl)
            out[name]["sweep_roofline"] = {
                "achieved_tflops": fl / (1e-3 * t_sweep) / 1e12,
                "frac": fl / (1e-3 * t_sweep) / 1e12 / PEAK_FP64_TFLOPS,
                "avg_launch_ms": t_sweep / n_sweep, "launches_per_solve": n_sweep}
            out[name]["phases_ms"] = {k: float(np.mean([i[k] for i in infos])) for k in
                                      ("t_build_ms", "t_iface_ms", "t_final_ms", "t_total_ms")}
    return out


def long_window_workloads():
    """Time-dependent V = 5 x cos t (GMRES(200) preconditioned by I - L_0)
    and |u|^2 (preconditioned fixed point) on 128 x 256 cells, 4000 steps:
    one solve each after a warm-up, to interface tolerance 1e-10."""
    from paper_1503_02564_amd import workloads as W
    out = {}
    for name, wl, kw in (("time_dependent", W.time_dependent(), dict(restart=200, max_iter=1500)),
                         ("cubic_packets", W.cubic_packets(), dict(max_iter=500))):
        ms, infos, _, st = timed_solves(wl, 1, 1, **kw)
        out[name] = {"ms_per_solve": ms, "iterations": infos[-1]["iters"], "status": st,
                     "residual": infos[-1]["residual"], "nl_worst": infos[-1]["nl_worst"],
                     "pt_steps_per_s": wl.pt_steps() / (1e-3 * ms)}
    out["workload"] = ("(-40,40), 128 x 256 cells, 4000 steps dt=2.5e-4, S0^2, sum of 4 packets; "
                       "time_dependent: V = 5 x cos t, GMRES(200) preconditioned by I - L_0; "
                       "cubic_packets: |u|^2, preconditioned fixed point")
    return out


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
    u0 = torch.from_numpy(np.ascontiguousarray(wl.u0)).to(dev)
    # target state from the reference potential (outside the timed region)
    import copy
    wr = copy.copy(wl)
    wr.V = wl.extras["V_ref"]
    wr.u0 = wl.u0[:1]
    ref = make_problem(wr, checkpoint_K=64)
    u_star = torch.zeros_like(u0[:1])
    swr.swr_solve(ref.ctx, u0[:1].contiguous(), u_star)
    ref.close()
    pb = make_problem(wl, v_per_problem=1, checkpoint_K=64)
    uT = torch.zeros_like(u0)
    swr.swr_solve(pb.ctx, u0, uT)
    gbar = (2.0 * (uT - u_star)).contiguous()
    dV = torch.zeros((wl.B, wl.nx), dtype=torch.float64, device=dev)
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
    from paper_1503_02564_amd import workloads as W
    out = {}
    for kind in ("harmonic", "linear_t", "cubic"):
        wl = W.paper_case(kind)
        ms, infos, _, st = timed_solves(wl, reps, 1, tol=1e-10, restart=100, max_iter=400)
        out[kind] = {"ms_per_solve": ms, "iterations": infos[-1]["iters"], "status": st,
                     "pt_steps_per_s": wl.pt_steps() / (ms * 1e-3),
                     "interface_residual": infos[-1]["residual"], "paper": PAPER_CONTEXT[kind]}
    out["workload"] = ("(-21,21), dx = 1e-4 (420001 nodes), dt = 1e-3, 500 steps, N = 1000 x 420 "
                       "cells, S0^2; V = -x^2 (causal interface solve), V = 5tx (GMRES preconditioned "
                       "by I - L_0), |u|^2 sech soliton (preconditioned fixed point)")
    return out


def batched_vs_plain(batched_ms):
    """The static-packet solve with every sweep task launched on its own (one
    subdomain of one problem per launch, one stream, staged) against the
    batched and pipelined form: same kernels, same interface solve, same
    certified residual."""
    from paper_1503_02564_amd import workloads as W
    wl = W.static_packet()
    ms, infos, _, st = timed_solves(wl, 1, 1, plain=1)
    return dict(workload="static_packet", plain_ms_per_solve=ms, batched_ms_per_solve=batched_ms,
                speedup_batched_over_plain=ms / batched_ms, plain_residual=infos[-1]["residual"],
                launches_plain=int(2 * wl.N * wl.B + 2 * wl.N - 2))


def fixture_error(uT):
    """Largest relative difference of the headline u(T) of members 0 and 31
    from the oracle's fixtures (sampled every 37 nodes and at every interface
    node; written by tests/golden/make_full_size.py)."""
    try:
        from tests.golden.make_full_size import read_fixture
    except ImportError:
        return None
    err = 0.0
    for m in (0, 31):
        idx, ref, scale = read_fixture("batched_uneven", m)
        err = max(err, float(np.max(np.abs(uT[m][idx] - ref)) / scale))
    return err


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
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--tune-ms", type=float, default=4000.0,
                    help="autotuner budget for the 'autotune' key, run after the headline on a "
                         "context of its own (0 = skip)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline solves (profiling runs)")
    ap.add_argument("--no-paper", dest="paper", action="store_false",
                    help="skip the paper's Sec. 6 workloads at N = 1000")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward ratio on the differentiation workload")
    ap.add_argument("--no-plain", dest="plain", action="store_false",
                    help="skip the one-launch-per-subdomain comparison")
    ap.add_argument("--no-long", dest="long", action="store_false",
                    help="skip the 4000-step time-dependent and cubic workloads")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain MIB-MiB device copy (counter calibration)")
    ap.add_argument("--source-hash", action="store_true",
                    help="print the sweep kernel source hash and exit")
    ap.add_argument("--profile", choices=["static_packet", "adjoint_batch"],
                    help="only timed solves of this workload (profiling runs): static_packet with "
                         "--solver, adjoint_batch forward solve and gradient")
    ap.add_argument("--solver", choices=["causal", "gmres", "bicgstab"], default="causal")
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
    if args.profile:
        from paper_1503_02564_amd import swr
        from paper_1503_02564_amd import workloads as W
        if args.profile == "static_packet":
            sv = dict(causal=swr.SWR_SOLVER_CAUSAL, gmres=swr.SWR_SOLVER_GMRES,
                      bicgstab=swr.SWR_SOLVER_BICGSTAB)[args.solver]
            sched = {}
            ms, infos, _, st = timed_solves(W.static_packet(), args.steps, args.warmup, sched=sched,
                                            solver=sv)
            print(json.dumps({"profile": "static_packet", "solver": args.solver, "ms_per_solve": ms,
                              "iterations": infos[-1]["iters"], "status": st, "schedule": sched}))
        else:
            print(json.dumps({"profile": "adjoint_batch", **adjoint_ratio(args.steps, args.warmup)}))
        return

    from paper_1503_02564_amd import workloads as W
    wl = W.batched_uneven()
    sched = {}
    ms, infos, uT, st = timed_solves(wl, args.steps, args.warmup, sched=sched)
    value = wl.pt_steps() / (1e-3 * ms)
    ph = {k: float(np.mean([i[k] for i in infos])) for k in
          ("t_factor_ms", "t_build_ms", "t_iface_ms", "t_final_ms", "t_total_ms")}
    resid = max(i["residual"] for i in infos)
    # dominant kernel: the subdomain sweep.  The library brackets every sweep
    # launch (impulse/d sweeps and final sweep, per pipeline chunk) with HIP
    # events on the stream it runs on and reports their summed duration; the
    # brackets also hold the S0^2 old far-history products (far_old_kernel)
    # launched between the sweep pieces, whose work is part of the sweep's
    # algorithmic count (the history terms), so both sides cover the same.
    flops = solve_flops(wl)
    n_launch = float(np.mean([i["n_sweep"] for i in infos]))
    t_sweep_ms = float(np.mean([i["t_sweep_ms"] for i in infos]))
    achieved = flops / (1e-3 * t_sweep_ms) / 1e12
    roof = {"bound": "alu", "kernel": "sweep_kernel (with the far_old_kernel products between its launches)",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": measured_traffic(), "avg_launch_ms": t_sweep_ms / n_launch,
            "launches_per_solve": n_launch, "flops_per_launch": flops / n_launch,
            "flops_per_pt_step": flops / solve_sweep_pt_steps(wl),
            "sweep_ms_per_solve": t_sweep_ms,
            "far_old_flops_share": far_old_flops(wl) / flops}
    out = {
        "metric": "grid-point*time-steps/s to interface residual 1e-10; adjoint/forward cost ratio",
        "value": value, "unit": "pt-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batched_uneven: (-100,100), 500 subdomains of U{40..400} cells "
                               "(109113 nodes), 32 seeded packets in one batch, 2000 steps "
                               "dt=5e-4, S0^2, seeded bumpy harmonic V, new algorithm, causal "
                               "interface solve",
                   "nx": wl.nx, "nt": wl.nt, "N": wl.N, "B": wl.B, "solver": "causal",
                   "schedule": {k: sched[k] for k in ("pipeline", "help_max", "restart", "pair_from", "group",
                                                      "graph", "check")}},
        "status": st, "interface_residual": resid, "phases_ms": ph,
        "max_rel_diff_vs_oracle_fixture": fixture_error(uT),
    }
    if not args.headline_only:
        # the same kernel with the GPU to itself: the staged schedule (build
        # sweeps, interface solve, final sweep one after the other), so that
        # no launch shares the GPU with the interface solve's kernels
        sms, sinfos, _, sst = timed_solves(wl, args.steps, args.warmup, pipeline=0)
        s_sweep = float(np.mean([i["t_sweep_ms"] for i in sinfos]))
        s_launch = float(np.mean([i["n_sweep"] for i in sinfos]))
        s_ach = flops / (1e-3 * s_sweep) / 1e12
        out["roofline_staged"] = {"bound": "alu", "kernel": "sweep_kernel", "achieved": s_ach,
                                  "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                  "frac": s_ach / PEAK_FP64_TFLOPS, "avg_launch_ms": s_sweep / s_launch,
                                  "launches_per_solve": s_launch, "sweep_ms_per_solve": s_sweep,
                                  "ms_per_solve": sms, "status": sst}
    if not args.headline_only and args.tune_ms > 0:
        # the autotuner on the headline workload (a context of its own, after
        # the timed region): the schedule it picks and the time it measured
        tuned = {}
        tms, _, _, _ = timed_solves(wl, 2, 0, tune_ms=args.tune_ms, sched=tuned)
        out["autotune"] = {"budget_ms": args.tune_ms, "chosen": tuned, "ms_per_solve": tms,
                           "default_schedule_ms": ms}
    if not args.headline_only:
        sp = static_packet_solvers(args.steps)
        out["static_packet"] = sp
        if args.plain:
            out["batched_vs_plain"] = batched_vs_plain(sp["causal"]["ms_per_solve"])
        if args.long:
            out["long_window"] = long_window_workloads()
        if not args.no_adjoint:
            adj = adjoint_ratio(max(1, min(args.steps, 5)), 1)
            out["adjoint_forward_cost_ratio"] = adj["ratio_bwd_over_fwd"]
            out["adjoint"] = adj
        if args.paper:
            out["paper_workloads"] = paper_workloads()
    out["roofline"] = roof
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
