"""Reader of the stored oracle values under tests/golden/ (plain text).

Imports nothing from the oracle: the GPU tests and the benchmark read the
stored numbers through this module without loading the oracle package.
"""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def read(name: str) -> dict:
    path = os.path.join(HERE, f"oracle_{name}.txt")
    out = {"lam": [], "log_lam": [], "pair_floor": [], "next": []}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "next":
                out["next"].append(float(parts[1]))
            elif parts[0].isdigit():
                out["lam"].append(float(parts[1]))
                out["log_lam"].append(float(parts[2]))
                out["pair_floor"].append(float(parts[3]))
            else:
                out[parts[0]] = float(parts[1])
    return {k: (np.array(v) if isinstance(v, list) else v) for k, v in out.items()}
