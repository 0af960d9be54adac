"""Timings of the other workloads (beside bench.py's R-MAT 26): the batch of
512 planted-partition SBMs and the 4M-vertex degree-corrected SBM, plain
and learned-pruned, with the return-move option off (the tolerance test as
written) and on; the split ablation; GSP-Leiden against GSP-Louvain.  Whole
runs, graph resident in device memory, best of `--reps` runs after one
warm-up run; prints one line per case.

    python bench_workloads.py [--batch] [--dcsbm] [--road] [--reps 3]
    python bench_workloads.py --split-ablation rmat20,dcsbm4m,road,rmat26
    python bench_workloads.py --leiden rmat20,dcsbm4m,road,rmat26
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


def split_ablation(ctx, gsp, name, g, reps):
    """Section 4.1 ablation on the GPU: no split (GVE-Louvain), split after
    the last pass (SL) and in every pass (SP), each by union-find and by
    label propagation (LPP); runtime, modularity, split time and the
    fraction of internally-disconnected communities."""
    rows = [("none", gsp.SPLIT_NONE, gsp.SPLIT_UF)]
    for mode, mv in (("SL", gsp.SPLIT_LAST), ("SP", gsp.SPLIT_PASS)):
        for algo, av in (("UF", gsp.SPLIT_UF), ("LPP", gsp.SPLIT_LPP)):
            rows.append((f"{mode}-{algo}", mv, av))
    for label, mode, algo in rows:
        dt = _best(lambda: ctx.run(1e-2, 10, split_mode=mode, split_algo=algo), reps)
        ctx.run(1e-2, 10, split_mode=mode, split_algo=algo, timing=1)
        st = ctx.stats()
        m = ctx.membership()
        ncomm = int(m.max()) + 1
        disc = ctx.count_disconnected(m)
        print(f"split {name} {label}: {dt * 1e3:.2f} ms per run, {g.nnz / dt / 1e9:.3f} G entries/s, "
              f"split {st['ms_split']:.2f} ms ({st['split_rounds']} LPP rounds), Q {ctx.result_modularity():.6f}, "
              f"{disc} of {ncomm} communities disconnected ({disc / ncomm:.2%}), passes {st['passes']}", flush=True)


def leiden_vs_louvain(ctx, name, g, reps):
    """GSP-Leiden (refinement in every pass) beside GSP-Louvain on one graph:
    time per run, phase times, passes, modularity and disconnected
    communities."""
    for label, lei in (("louvain", 0), ("leiden", 1)):
        dt = _best(lambda: ctx.run(1e-2, 10, leiden=lei), reps)
        ctx.run(1e-2, 10, leiden=lei, timing=1)
        st = ctx.stats()
        m = ctx.membership()
        print(f"leiden {name} {label}: {dt * 1e3:.2f} ms per run, {g.nnz / dt / 1e9:.3f} G entries/s, "
              f"passes {st['passes']}, iterations {st['iterations']}, refine iterations {st['refine_iterations']}, "
              f"communities {st['communities']}, refined {st['refined']}, phases ms move {st['ms_move']:.1f} "
              f"refine {st['ms_refine']:.1f} split {st['ms_split']:.1f} aggregate {st['ms_aggregate']:.1f} "
              f"other {st['ms_other']:.1f}, scanned {st['scanned_entries']}, Q {ctx.result_modularity():.6f}, "
              f"{ctx.count_disconnected(m)} of {int(m.max()) + 1} communities disconnected", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", action="store_true", help="512 SBM graphs, n log-uniform in [1e3, 2e5]")
    ap.add_argument("--dcsbm", action="store_true", help="DC-SBM, 4M vertices, held-out seed 1000")
    ap.add_argument("--road", action="store_true", help="road-like graph, 59M vertices, average degree 2.1")
    ap.add_argument("--split-ablation", default="", help="comma list of bench.py workloads (rmat20, dcsbm4m, "
                                                          "rmat26) or road: split modes x algorithms")
    ap.add_argument("--leiden", default="", help="comma list of bench.py workloads or road: GSP-Leiden beside "
                                                  "GSP-Louvain")
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    if a.leiden:
        import gsp_inputs as gi
        import paper_2402_11454_amd as gsp
        from bench import make_graph
        ctx = gsp.Context(0)
        for name in a.leiden.split(","):
            g = gi.road_network() if name == "road" else make_graph(name)
            ctx.load_graph(g)
            leiden_vs_louvain(ctx, name, g, a.reps)
            del g
        ctx.close()
        return
    if a.split_ablation:
        import gsp_inputs as gi
        import paper_2402_11454_amd as gsp
        from bench import make_graph
        ctx = gsp.Context(0)
        for name in a.split_ablation.split(","):
            g = gi.road_network() if name == "road" else make_graph(name)
            ctx.load_graph(g)
            split_ablation(ctx, gsp, name, g, a.reps)
            del g
        ctx.close()
        return
    if not (a.batch or a.dcsbm or a.road):
        a.batch = a.dcsbm = a.road = True
    import gsp_inputs as gi
    import paper_2402_11454_amd as gsp
    from paper_2402_11454_amd.train_pruner import DEFAULT_OUT, DEFAULT_THETA, load_params

    ctx = gsp.Context(0)
    ctx.pruner_set(load_params(DEFAULT_OUT))
    modes = (("plain", {}), ("learned", dict(prune_mode=gsp.PRUNE_LEARNED, prune_threshold=DEFAULT_THETA)))
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
    if a.road:
        g = gi.road_network()
        ctx.load_graph(g)
        for rm in (0, 1):
            dt = _best(lambda: ctx.run(1e-2, 10, return_moves=rm), a.reps)
            ctx.run(1e-2, 10, return_moves=rm, timing=1)
            st = ctx.stats()
            print(f"road return_moves={rm} plain: {dt * 1e3:.2f} ms per run, {g.nnz / dt / 1e9:.3f} G entries/s "
                  f"(n={g.n}, {g.nnz} entries), passes {st['passes']}, iterations {st['iterations']}, phases ms "
                  f"move {st['ms_move']:.1f} split {st['ms_split']:.1f} aggregate {st['ms_aggregate']:.1f} other "
                  f"{st['ms_other']:.1f}, Q {ctx.result_modularity():.6f}", flush=True)
        del g
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
