"""Writes leiden_oracle.json: the oracle's GSP-Leiden whole runs (the GPU
contract: 8 ordered sub-rounds, tolerance 1e-2, at most 10 passes, split in
every pass) on full-size workloads, for the full-size GPU parity tests:
membership digest, per-pass local-moving iterations, communities,
refinement iterations and refined sub-communities, modularity.

    dcsbm4m  the 4M-vertex degree-corrected SBM of seed 1000
    rmat26   R-MAT scale 26 (2^30 samples, a/b/c/d .57/.19/.19/.05, seed 26,
             weights U[1, 10) taken onto the grid of exact sums)

Only the oracle and the seeded input generators are used.  Each case
replaces its own entry of the file.

    python tests/golden/make_leiden.py dcsbm4m   # about 6 minutes on one core
    python tests/golden/make_leiden.py rmat26    # about 40 minutes on one core, about 50 GB of host memory
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "leiden_oracle.json")


def graph(name):
    sys.path.insert(0, ROOT)
    import gsp_inputs as gi
    import oracle
    if name == "dcsbm4m":
        return "dcsbm_4m(1000)", gi.dcsbm_4m(1000)
    if name == "rmat26":
        g = gi.rmat(26, 16, *gi.RMAT_ABC, 26, weights=(1.0, 10.0), name="rmat-26")
        return "rmat(26, 16, .57, .19, .19, seed 26, weights U[1, 10))", oracle.CSR.of(g)
    raise SystemExit(f"unknown case {name}")


def main():
    sys.path.insert(0, ROOT)
    import oracle
    name = sys.argv[1] if len(sys.argv) > 1 else "dcsbm4m"
    t = time.time()
    desc, g = graph(name)
    print(f"{name}: n={g.n} nnz={g.nnz} generated in {time.time() - t:.0f}s", flush=True)
    t = time.time()
    oracle.set_verbose(True)
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, leiden=True)
    oracle.set_verbose(False)
    dt = time.time() - t
    sha = hashlib.sha1(np.ascontiguousarray(r.membership, dtype=np.int32).tobytes()).hexdigest()
    entry = {"graph": desc, "n": int(g.n), "nnz": int(g.nnz), "tolerance": 1e-2, "max_passes": 10, "rounds": 8,
             "modularity": r.modularity, "passes": r.passes, "iterations": list(r.iterations),
             "communities": list(r.communities), "refine_iterations": list(r.refine_iterations),
             "refined": list(r.refined), "membership_sha1": sha, "seconds": round(dt, 1)}
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data[name] = entry
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    print(f"{name}: GSP-Leiden Q={r.modularity:.6f} passes={r.passes} iterations={r.iterations} "
          f"refined={r.refined} in {dt:.0f}s", flush=True)


if __name__ == "__main__":
    main()
