"""Writes c2_reactions.txt: the reaction totals of the two pin sets of the 256 x 256 x 16
compact-tension plate (the C2 workload of workloads.c2_compact_tension), from the FP64 CPU
oracle's run of Algorithm 1 to a relative equilibrium residual of 1e-9 (eq 5).  The reactions
are the Lagrange multipliers of the strong constraints, -2^-b p at the constrained DOFs,
summed per set (Section 4.1).  Calls only oracle/ and the seeded workload generator.

    python tests/golden/make_c2_reactions.py        # about 10-20 minutes on 8 host cores
"""
import os
import sys
import time

import numpy as np
import scipy.fft

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.solver import Solver  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_reactions.txt")
TOL = 1e-9


def main():
    prob = W.c2_compact_tension()
    t0 = time.time()
    with scipy.fft.set_workers(os.cpu_count() or 1):
        s = Solver.from_problem(prob)
        out = s.solve(tol=TOL, max_iter=20000)
    dt = time.time() - t0
    if not out["converged"]:
        raise SystemExit(f"oracle did not converge: residual {out['residual']:.3e} after {out['iterations']}")
    tot = np.asarray(out["totals"])
    with open(OUT, "w") as f:
        f.write("# C2 compact-tension plate 256x256x16 (workloads.c2_compact_tension), FP64 oracle,\n")
        f.write(f"# Algorithm 1 with ACV_P depth 4 period 2, relative residual < {TOL:g} (eq 5).\n")
        f.write("# Written by tests/golden/make_c2_reactions.py; reaction totals per set, x y z.\n")
        f.write(f"iterations: {out['iterations']}\n")
        f.write(f"residual: {out['residual']:.17e}\n")
        for k in range(tot.shape[0]):
            f.write(f"set{k}: " + " ".join(f"{v:.17e}" for v in tot[k]) + "\n")
        f.write(f"# oracle wall time {dt:.0f} s\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()
