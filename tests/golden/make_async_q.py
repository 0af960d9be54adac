"""Writes async_q.json: the modularity the paper's own local-moving loop
(asynchronous, one thread: the oracle's quality reference) reaches on the
full-size workloads, so that the GPU runs can be held to Q >= Q_async - 0.005
without rerunning that loop in every test.

Only the oracle and the seeded input generators are used.

    python tests/golden/make_async_q.py              # R-MAT 20, DC-SBM 4M (seed 1000): a few minutes
    python tests/golden/make_async_q.py rmat26       # only R-MAT 26 (about 50 GB of host memory)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "async_q.json")


def graphs(names):
    sys.path.insert(0, ROOT)
    import gsp_inputs as gi
    make = {
        "sbm10k": lambda: gi.planted_sbm_10k(),
        "rmat20": lambda: gi.rmat20(),
        "dcsbm4m_s1000": lambda: gi.dcsbm_4m(1000),
        "rmat26": lambda: gi.rmat(26, 16, *gi.RMAT_ABC, 26, weights=(1.0, 10.0), name="rmat-26"),
    }
    for name in names:
        yield name, make[name]


def main():
    sys.path.insert(0, ROOT)
    import oracle
    names = ["rmat26"] if "rmat26" in sys.argv[1:] else ["sbm10k", "rmat20", "dcsbm4m_s1000"]
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    for name, make in graphs(names):
        t = time.time()
        g = make()
        print(f"{name}: n={g.n} nnz={g.nnz} generated in {time.time() - t:.0f}s", flush=True)
        g = oracle.CSR.of(g)   # the oracle's types (fp64 weights on the grid); the generator's arrays go
        t = time.time()
        oracle.set_verbose(True)
        r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=False)
        oracle.set_verbose(False)
        dt = time.time() - t
        out[name] = {"n": int(g.n), "nnz": int(g.nnz), "modularity": r.modularity, "passes": r.passes,
                     "iterations": list(r.iterations), "communities": list(r.communities),
                     "tolerance": 1e-2, "max_passes": 10, "seconds": round(dt, 1)}
        print(f"{name}: async Q={r.modularity:.6f} passes={r.passes} in {dt:.0f}s", flush=True)
        del g
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main()
