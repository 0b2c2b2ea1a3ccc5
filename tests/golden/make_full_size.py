"""Write reference solutions of the full-length batched-uneven and
cubic-packets workloads as sampled text fixtures for the full-size GPU tests.
Calls the oracle only.

    python tests/golden/make_full_size.py [batched_uneven] [cubic_packets]

The reference is the monodomain Crank-Nicolson solution (oracle.mono, FP64;
for |u|^2 with the inner fixed point of the paper's nonlinear scheme), the
plain definition a converged decomposed solve reproduces (Sec. 3):
* batched_uneven: (-100, 100), 500 subdomains of U{40..400} cells (~109k
  nodes), 2000 steps, members 0 and 31 of the 32-problem batch;
* cubic_packets: (-40, 40), 128 x 256 cells, |u|^2, 4000 steps.
Each file holds u(T) at every STRIDE-th node and at every node shared by two
subdomains (where the decomposed solve averages its two sides), plus max |u(T)|
over all nodes (the scale of the relative comparison).  At these grids
(dt/h^2 <= 150) FP64 time stepping is accurate to ~1e-13, so the FP64 oracle
is the reference itself.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_1503_02564_amd import workloads as W  # noqa: E402

STRIDE = 37
CASES = {
    "batched_uneven": (W.batched_uneven, (0, 31)),
    "cubic_packets": (W.cubic_packets, (0,)),
}


def fixture_path(kind, member):
    return os.path.join(HERE, f"full_{kind}_m{member}.txt")


def sample_nodes(wl):
    """Every STRIDE-th node, both walls and every interface node."""
    idx = set(range(0, wl.nx, STRIDE)) | {wl.nx - 1} | set(int(o) for o in wl.offsets[1:])
    return np.array(sorted(idx), dtype=np.int64)


def read_fixture(kind, member):
    """(node indices, u(T) there, max |u(T)| over all nodes)."""
    scale = None
    with open(fixture_path(kind, member)) as f:
        for line in f:
            if line.startswith("# max_abs_u"):
                scale = float(line.split()[2])
    dat = np.loadtxt(fixture_path(kind, member))
    return dat[:, 0].astype(np.int64), dat[:, 1] + 1j * dat[:, 2], scale


def main(kinds):
    for kind in kinds:
        make, members = CASES[kind]
        wl = make()
        for m in members:
            t0 = time.time()
            uT = O.mono(wl, wl.u0[m])
            idx = sample_nodes(wl)
            with open(fixture_path(kind, m), "w") as f:
                f.write(f"# u(T) of the '{kind}' workload, batch member {m} (nx = {wl.nx}, "
                        f"nt = {wl.nt}, dt = {wl.dt}, h = {wl.h}, N = {wl.N}): monodomain "
                        f"Crank-Nicolson, FP64 (oracle.mono).\n")
                f.write("# written by tests/golden/make_full_size.py (oracle only)\n")
                f.write(f"# max_abs_u {np.max(np.abs(uT)):.17e}\n")
                f.write(f"# stride {STRIDE} plus walls and interface nodes\n")
                f.write("# columns: node re im\n")
                for i in idx:
                    f.write(f"{i} {uT[i].real:.17e} {uT[i].imag:.17e}\n")
            print(kind, m, "written in", round(time.time() - t0, 1), "s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
