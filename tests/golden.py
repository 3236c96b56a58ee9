"""Reader for the hand-derived fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split(":", 1)
            vals = [float(v) for v in val.split()]
            out[key.strip()] = vals[0] if len(vals) == 1 else np.array(vals)
    n = int(out["n"])
    out["n"] = n
    for k in ("H", "D", "X0"):
        if k in out:
            out[k] = out[k].reshape(n, n)
    return out
