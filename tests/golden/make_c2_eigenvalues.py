"""Writes c2_eigenvalues.txt: the 128 lowest eigenvalues of the C2 workload (72^3 grid,
23,847 plane waves, Gamma, 64 atoms x 4 projectors, seed 2) from the oracle's block
Davidson to a residual of 1e-10 Ry, the reference the GPU Davidson's 1e-8 eigenvalues
are compared with. Calls only the oracle and the input generator:

    python tests/golden/make_c2_eigenvalues.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2501_08697_amd import workload as W  # noqa: E402


def main():
    p = W.make_problem("C2")
    eig, _, res, its = oracle.davidson(p, tol=1e-10, max_iter=400)
    assert np.max(res) < 1e-10, np.max(res)
    with open(os.path.join(HERE, "c2_eigenvalues.txt"), "w") as f:
        f.write("# 128 lowest eigenvalues (Ry) of the C2 workload (72^3, 23,847 PW, Gamma, seed 2), written by\n")
        f.write(f"# tests/golden/make_c2_eigenvalues.py: oracle block Davidson, max residual {np.max(res):.2e} Ry, "
                f"{int(its[0])} iterations\n")
        for e in eig[0]:
            f.write(f"{e:.15f}\n")


if __name__ == "__main__":
    main()
