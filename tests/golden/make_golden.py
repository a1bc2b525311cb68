"""Write the oracle's reference values for the fixed workloads.

Calls only ``oracle`` and ``datagen``.  Output: one text file per workload,
``oracle_<name>.txt``, holding the t dominant generalised eigenvalues of
exp(S_B) x = lam exp(S_W) x (exact reduction route), the head of the reduced
spectrum, and the attainable-accuracy report (u lam_1 / lam_i per pair and
u lam_1 / gap for the span).  Usage: python tests/golden/make_golden.py C1 C2
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import datagen  # noqa: E402
import oracle as O  # noqa: E402
from tests.golden.reader import read  # noqa: E402,F401


def write(name: str) -> str:
    p = datagen.config(name)
    H_W, H_B = O.scatter_factors(p.X, p.counts)
    red = O.eda_reduced(H_W, H_B, p.t)
    fl = O.accuracy_floor(red.lam_all, p.t)
    sB = np.linalg.svd(H_B, compute_uv=False) ** 2
    sW = np.linalg.svd(H_W, compute_uv=False) ** 2
    path = os.path.join(HERE, f"oracle_{name}.txt")
    with open(path, "w") as f:
        f.write(f"# oracle reference values for workload {name}: d={p.d} k={p.k} "
                f"n={p.n} t={p.t} r={p.r} seed={p.seed}\n")
        f.write("# written by tests/golden/make_golden.py (oracle.eda_reduced, float64)\n")
        f.write(f"sigma2_B_max {sB[0]:.17e}\nsigma2_B_min_nonzero {sB[p.k - 2]:.17e}\n")
        f.write(f"nu_1 {sW[0]:.17e}\n")
        f.write(f"span_floor {fl['span']:.6e}\ngap {fl['gap']:.17e}\n")
        f.write("# i lam_i log_lam_i pair_floor_i\n")
        for i in range(p.t):
            f.write(f"{i} {red.lam[i]:.17e} {red.log_lam[i]:.17e} {fl['pair'][i]:.6e}\n")
        f.write("# reduced spectrum head (lam_{t+1} ...)\n")
        for i in range(p.t, min(p.t + 8, red.lam_all.size)):
            f.write(f"next {red.lam_all[i]:.17e}\n")
    return path


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["C1", "C2"]:
        print(write(nm))
