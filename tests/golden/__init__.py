"""Small text fixtures, each citing the passage of the paper it follows."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name):
    """Parses a fixture: n, edges (u-v or u-v:w), int lists for other keys."""
    out = {}
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            if key == "n":
                out["n"] = int(vals[0])
            elif key == "edges":
                edges, weights = [], {}
                for tok in vals:
                    uv, _, w = tok.partition(":")
                    u, v = (int(x) for x in uv.split("-"))
                    edges.append((u, v))
                    if w:
                        weights[(min(u, v), max(u, v))] = float(w)
                out["edges"] = edges
                out["weights"] = weights or None
            else:
                out[key] = np.array([int(x) for x in vals], dtype=np.int64)
    return out
