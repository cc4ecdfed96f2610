"""Writes the oracle's solution of the 3D recipe at 16^3 cells (degree 1, w = 20, mu ~ U[1,2] per
cell from seed 3, plane wave on x = 0, impedance elsewhere; 104,544 DoFs) for the GPU parity test
of that size: the oracle's global sparse LU (nested-dissection order, iterative refinement), with
its relative residual checked <= 1e-13.  Too slow to recompute inside a test (about ten minutes
and 10 GB of host memory).  Calls only oracle/ and the seeded input generator.

Usage: python tests/golden/make_c3_reference.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import system  # noqa: E402
from oracle.system import Problem  # noqa: E402

OUT = os.path.join(HERE, "c3_m16_oracle_E.npy")


def main():
    d = dict(workloads.c3(16), subdomains=(1, 1, 1))
    t0 = time.time()
    s = system.assemble(Problem(**d))
    E = system.solve_lu(s)
    res = system.relative_residual(s, E)
    print(f"{s.n} DoFs, global relative residual {res:.3e}, {time.time() - t0:.1f}s", flush=True)
    assert res <= 1e-13, res
    np.save(OUT, E)


if __name__ == "__main__":
    main()
