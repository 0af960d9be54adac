"""Writes dcsbm4m_oracle.json: the oracle's whole runs on the 4M-vertex
degree-corrected SBM (seed 1000, the held-out graph of the learned-pruning
workload), plain and learned-pruned, for the full-size GPU parity test.

Only the oracle and the seeded input generators are used.  The learned run's
network is not a trained one: gate_params() draws it from a seeded uniform
law (Glorot-sized layers, output layer scaled by `sharp` so that few logits
lie near the threshold), so no input of the oracle comes from the GPU path.

    python tests/golden/make_dcsbm4m.py      # about 4 minutes on one core
"""
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "dcsbm4m_oracle.json")
SEED = 1000
THETA = 0.5
GATE_PARAMS = 4801


def gate_params(seed: int = 61, b3: float = 0.5, sharp: float = 32.0) -> np.ndarray:
    """8 -> 64 -> 64 -> 1 network, flat layout W1[64][8], b1, W2[64][64], b2,
    w3[64], b3: uniform(-1, 1) draws scaled by sqrt(6 / fan_in) (biases by
    0.1), output layer and its bias scaled by `sharp`."""
    sys.path.insert(0, ROOT)
    import gsp_inputs as gi
    p = (gi.uniform(seed, GATE_PARAMS) * 2.0 - 1.0).astype(np.float32)
    p[0:512] *= math.sqrt(6 / 8)
    p[512:576] *= 0.1
    p[576:4672] *= math.sqrt(6 / 64)
    p[4672:4736] *= 0.1
    p[4736:4800] *= math.sqrt(6 / 64) * sharp
    p[4800] = b3 * sharp
    return p


def membership_digest(m) -> str:
    return hashlib.sha1(np.ascontiguousarray(m, dtype=np.int32).tobytes()).hexdigest()


def main():
    sys.path.insert(0, ROOT)
    import gsp_inputs as gi
    import oracle
    g = gi.dcsbm_4m(SEED)
    out = {"graph": f"dcsbm_4m({SEED})", "n": int(g.n), "nnz": int(g.nnz), "tolerance": 1e-2, "max_passes": 10,
           "rounds": 8, "theta": THETA}
    t = time.time()
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    out["plain"] = {"modularity": r.modularity, "iterations": list(r.iterations),
                    "communities": list(r.communities), "membership_sha1": membership_digest(r.membership)}
    print(f"plain: {time.time() - t:.0f}s Q={r.modularity:.6f} iterations={r.iterations}", flush=True)
    t = time.time()
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, prune_params=gate_params(),
                       theta=THETA)
    out["learned"] = {"modularity": r.modularity, "iterations": list(r.iterations),
                      "communities": list(r.communities), "counters": dict(r.counters),
                      "membership_sha1": membership_digest(r.membership)}
    print(f"learned: {time.time() - t:.0f}s Q={r.modularity:.6f} iterations={r.iterations} {r.counters}", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
