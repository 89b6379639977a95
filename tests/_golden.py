"""Reader for the closed-form fixtures in tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    i = 0
    while i < len(lines):
        key, *rest = lines[i].split()
        if rest:
            out[key] = int(rest[0])
            i += 1
            continue
        rows = out["m"] if key in ("A", "Q") else out["n"]
        M = np.array([[float(x) for x in lines[i + 1 + r].split()] for r in range(rows)])
        out[key] = np.asfortranarray(M)
        i += 1 + rows
    return out


def names():
    return sorted(f for f in os.listdir(GOLDEN) if f.endswith(".txt"))
