"""Reader of tests/golden/hand_examples.txt (hand-worked counts and tau)."""
import math
import os

import numpy as np

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_examples.txt")


def load():
    out = []
    with open(PATH) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, u, v, counts, tb, ta = [p.strip() for p in line.split("|")]
            nc, nd, n1, n2, n3 = (int(t) for t in counts.split())
            out.append({
                "name": name,
                "u": np.array([float(t) for t in u.split()], np.float32),
                "v": np.array([float(t) for t in v.split()], np.float32),
                "nc": nc, "nd": nd, "n1": n1, "n2": n2, "n3": n3,
                "tau_b": float(tb), "tau_a": float(ta),
            })
    return out


def close(got, want, tol=1e-15):
    if math.isnan(want):
        return math.isnan(got)
    return abs(got - want) <= tol
