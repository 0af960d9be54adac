"""Timings of the other workloads (beside bench.py's R-MAT 26): the batch of
512 planted-partition SBMs and the 4M-vertex degree-corrected SBM, plain
and learned-pruned, with the return-move option off (the tolerance test as
written) and on.  Whole runs, graph resident in device memory, best of
`--reps` runs after one warm-up run; prints one line per case.

    python bench_workloads.py [--batch] [--dcsbm] [--reps 3]
"""
import argparse
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


def _best(run, reps):
    run()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        run()
        best = min(best, time.perf_counter() - t0)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", action="store_true", help="512 SBM graphs, n log-uniform in [1e3, 2e5]")
    ap.add_argument("--dcsbm", action="store_true", help="DC-SBM, 4M vertices, held-out seed 1000")
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    if not (a.batch or a.dcsbm):
        a.batch = a.dcsbm = True
    import gsp_inputs as gi
    import paper_2402_11454_amd as gsp
    from paper_2402_11454_amd.train_pruner import DEFAULT_OUT, load_params

    ctx = gsp.Context(0)
    ctx.pruner_set(load_params(DEFAULT_OUT))
    modes = (("plain", {}), ("learned", dict(prune_mode=gsp.PRUNE_LEARNED, prune_threshold=0.5)))
    if a.batch:
        gs = gi.batch_sbm(512, 4, 1.0)
        entries = sum(g.nnz for g in gs)
        ctx.load_batch(gs)
        del gs
        for rm in (0, 1):
            for name, kw in modes:
                dt = _best(lambda: ctx.run_batch(1e-2, 10, return_moves=rm, **kw), a.reps)
                st = ctx.stats()
                q = ctx.batch_modularity()
                print(f"batch512 return_moves={rm} {name}: {dt * 1e3:.1f} ms per run, {entries / dt / 1e9:.3f} G "
                      f"entries/s, sweeps {st['sweeps']}, iterations per pass (max over graphs) {st['iterations']}, "
                      f"per-graph Q mean {q.mean():.6f}", flush=True)
    if a.dcsbm:
        g = gi.dcsbm_4m(1000)
        ctx.load_graph(g)
        for rm in (0, 1):
            for name, kw in modes:
                dt = _best(lambda: ctx.run(1e-2, 10, return_moves=rm, **kw), a.reps)
                st = ctx.stats()
                print(f"dcsbm4m return_moves={rm} {name}: {dt * 1e3:.2f} ms per run, {g.nnz / dt / 1e9:.3f} G "
                      f"entries/s, iterations {st['iterations']}, scanned {st['scanned_entries']}, "
                      f"Q {ctx.result_modularity():.6f}", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
