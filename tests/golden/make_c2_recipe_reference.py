"""Writes the oracle's u(T) for the benchmark recipe at n = 4095.

The benchmark runs n = 65535, M = 2048 (alpha 1.5, gamma 0.4, r 4, kappa seed
3, f seed 4); the direct oracle (dense LU per level, full L1 history) cannot
run there, so its FP64 answer is computed once at n = 4095 with the same M,
orders, grading and seeds (the seeded fields evaluated on the coarse grid).
GPU tests compare every solver form against this file.

Usage (from the repository root; about 10 minutes on 8 cores):
    python tests/golden/make_c2_recipe_reference.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2002_11978_amd import workloads as W  # noqa: E402

N, M = 4095, 2048
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_recipe_n4095_M2048_uT.txt")


def main():
    pb = W.seeded(1.5, 0.4, N, M, r=4.0, kappa_seed=3, f_seed=4)
    U = oracle.dids_solve(pb.alpha, pb.gamma, pb.n, pb.M, pb.r, pb.kappa, pb.f, pb.phi)
    header = (f"oracle (direct scheme, dense LU, full L1 history) u^M at n={N}, M={M}, alpha=1.5, gamma=0.4, "
              f"r=4, kappa seed 3, f seed 4, phi=(1-x^2)^(alpha/2); written by make_c2_recipe_reference.py")
    np.savetxt(OUT, U[-1], fmt="%.17e", header=header)
    print("wrote", OUT, "max |u^M| =", float(np.abs(U[-1]).max()))


if __name__ == "__main__":
    main()
