"""Write reference solutions of the paper's numerical-section workloads
(Sec. 6: (-21, 21), T = 0.5, dt = 1e-3, mesh size 1e-4 or 1e-5, S0^2 for the
decomposed solvers) as sampled text fixtures for the paper-scale GPU tests.
Calls the oracle only.

    python tests/golden/make_paper_scale.py [--dx 1e-5] [harmonic] [linear_t] [cubic]

The reference is the monodomain Crank-Nicolson solution (the plain definition
the decomposed solvers converge to, Sec. 3), computed in extended precision
(oracle.mono_ld): on this grid (dt/h^2 = 1e5, 420001 nodes) one FP64 sweep
over the whole domain is itself off by ~1e-9, far more than the decomposed
solution.  Each file holds u(T) at every STRIDE-th node, the maximum of
|u(T)| over all nodes (the scale of the relative comparison), and the error
of the FP64 monodomain oracle (oracle.mono) against it over all nodes: the
accuracy FP64 arithmetic of the plain definition reaches on this grid.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_1503_02564_amd import workloads as W  # noqa: E402

STRIDE = {1e-4: 200, 1e-5: 2000}   # about 2100 sampled nodes per fixture


def fixture_path(kind, dx=1e-4):
    tag = "" if dx == 1e-4 else f"_dx{dx:.0e}"
    return os.path.join(HERE, f"paper_scale_{kind}{tag}.txt")


def read_fixture(kind, dx=1e-4):
    """(node indices, u(T) there, max |u(T)| over all nodes, relative error
    of the FP64 monodomain oracle)."""
    scale = err64 = None
    with open(fixture_path(kind, dx)) as f:
        for line in f:
            if line.startswith("# max_abs_u"):
                scale = float(line.split()[2])
            if line.startswith("# fp64_monodomain_rel_err"):
                err64 = float(line.split()[2])
    dat = np.loadtxt(fixture_path(kind, dx))
    return dat[:, 0].astype(np.int64), dat[:, 1] + 1j * dat[:, 2], scale, err64


def main(kinds, dx=1e-4):
    for kind in kinds:
        wl = W.paper_case(kind, dx=dx)
        t0 = time.time()
        uT = O.mono_ld(wl, wl.u0[0], nl_tol=1e-16, nl_maxit=200)
        err64 = np.max(np.abs(O.mono(wl, wl.u0[0]) - uT)) / np.max(np.abs(uT))
        stride = STRIDE[dx]
        idx = np.arange(0, wl.nx, stride)
        with open(fixture_path(kind, dx), "w") as f:
            f.write(f"# u(T) of the paper's Sec. 6 workload '{kind}' (nx = {wl.nx}, nt = {wl.nt}, "
                    f"dt = {wl.dt}, h = {wl.h}): monodomain Crank-Nicolson in extended precision "
                    f"(oracle.mono_ld).\n")
            f.write("# written by tests/golden/make_paper_scale.py (oracle only)\n")
            f.write(f"# max_abs_u {np.max(np.abs(uT)):.17e}\n")
            f.write(f"# fp64_monodomain_rel_err {err64:.6e}\n")
            f.write(f"# stride {stride}\n")
            f.write("# columns: node re im\n")
            for i in idx:
                f.write(f"{i} {uT[i].real:.17e} {uT[i].imag:.17e}\n")
        print(kind, "written in", round(time.time() - t0, 1), "s", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    dx = 1e-4
    if args[:1] == ["--dx"]:
        dx = float(args[1])
        args = args[2:]
    main(args or ["harmonic", "linear_t", "cubic"], dx)
