"""Writes rmat26_oracle.json: the oracle's synchronous whole run (the GPU
contract: 8 ordered sub-rounds, tolerance 1e-2, at most 10 passes, split
in every pass) on R-MAT scale 26 (2^30 samples, a/b/c/d .57/.19/.19/.05,
seed 26, weights U[1, 10) taken onto the grid of exact sums), for the
full-size GPU parity test: membership digest, iterations and communities
per pass, modularity.

Only the oracle and the seeded input generators are used.

    python tests/golden/make_rmat26.py      # about 20 minutes on one core, about 50 GB of host memory
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "rmat26_oracle.json")


def main():
    sys.path.insert(0, ROOT)
    import gsp_inputs as gi
    import oracle
    t = time.time()
    g = gi.rmat(26, 16, *gi.RMAT_ABC, 26, weights=(1.0, 10.0), name="rmat-26")
    print(f"rmat26: n={g.n} nnz={g.nnz} generated in {time.time() - t:.0f}s", flush=True)
    g = oracle.CSR.of(g)   # fp64 weights on the grid; the generator's arrays go
    t = time.time()
    oracle.set_verbose(True)
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    oracle.set_verbose(False)
    dt = time.time() - t
    sha = hashlib.sha1(np.ascontiguousarray(r.membership, dtype=np.int32).tobytes()).hexdigest()
    out = {"graph": "rmat(26, 16, .57, .19, .19, seed 26, weights U[1, 10))", "n": int(g.n), "nnz": int(g.nnz),
           "tolerance": 1e-2, "max_passes": 10, "rounds": 8, "modularity": r.modularity, "passes": r.passes,
           "iterations": list(r.iterations), "communities": list(r.communities), "membership_sha1": sha,
           "seconds": round(dt, 1)}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print(f"rmat26: sync Q={r.modularity:.6f} passes={r.passes} iterations={r.iterations} in {dt:.0f}s", flush=True)


if __name__ == "__main__":
    main()
