"""Benchmark: full GSP-Louvain runs on one MI355X.

Workload: R-MAT scale 20 (2^20 vertices, 16 samples per vertex, a/b/c/d =
.57/.19/.19/.05, symmetrised, deduplicated, no self-loops, unit weights),
the graph the headline metric is quoted on.  The graph is generated (seeded),
loaded once into the library's device memory, then `warmup` untimed runs and
`steps` timed runs of gsp_run (tolerance 1e-2, at most 10 passes) follow.

Prints ONE JSON line: edges/s = directed CSR entries / seconds per run, the
per-run time, a roofline object for the dominant kernel (algorithmic bytes
from the library's counters over its HIP-event time in the timed region)
and a CPU baseline: the sequential oracle timed on one host core on the same
graph.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edges/s per full GSP-Louvain run; learned-pruned vs plain at equal modularity"
HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {  # kernel class -> its kernel (as rocprof names it)
    "move_small": "k_move_small",
    "move_wave": "k_move_wave",
    "move_block": "k_move_block",
    "move_hub": "k_move_hub_insert",
    "move_hub_finish": "k_move_hub_part + k_move_hub_final",
    "move_apply": "k_move_apply",
    "frontier": "k_move_compact",
    "split": "k_split_hook + k_split_compress",
    "aggregate": "aggregation kernels",
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--scale", type=int, default=20)
    p.add_argument("--seed", type=int, default=20)
    p.add_argument("--tolerance", type=float, default=1e-2)
    p.add_argument("--max-passes", type=int, default=10)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--timing", type=int, default=2, help="0 none, 1 phases, 2 phases+kernels")
    return p.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {a.gpus} is not supported "
              "(the multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import gsp_inputs as gi
    import paper_2402_11454_amd as gsp

    t0 = time.time()
    g = gi.rmat(a.scale, 16, *gi.RMAT_ABC, a.seed, name=f"rmat-{a.scale}")
    print(f"[bench] generated R-MAT scale {a.scale}: n={g.n} nnz={g.nnz} in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = gsp.Context(0, stream=stream)
    ctx.load_graph(g)
    opt = gsp.default_options(timing=a.timing)
    for w in range(a.warmup):
        ctx.run(a.tolerance, a.max_passes, options=opt)
        print(f"[bench] warmup {w + 1}/{a.warmup} done", file=sys.stderr, flush=True)

    # timed region: `steps` whole runs, the graph already resident in HBM
    kstats = {k: dict(launches=0, ms=0.0, bytes=0.0, items=0) for k in gsp.KERNEL_CLASSES}
    phase = dict(ms_move=0.0, ms_split=0.0, ms_aggregate=0.0, ms_other=0.0)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(a.steps):
        ctx.run(a.tolerance, a.max_passes, options=opt)
        st = ctx.stats()
        for name, v in st["kernels"].items():
            for f in ("launches", "ms", "bytes", "items"):
                kstats[name][f] += v[f]
        for f in phase:
            phase[f] += st[f]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1000.0 * elapsed / a.steps
    value = g.nnz / (elapsed / a.steps)

    memb = ctx.membership()
    q = ctx.result_modularity()
    disc = ctx.count_disconnected(memb)
    st = ctx.stats()
    print(f"[bench] {a.steps} runs: {ms_per_step:.3f} ms/run, Q={q:.6f}, disconnected={disc}, "
          f"passes={st['passes']} iterations={st['iterations']} communities={st['communities']}",
          file=sys.stderr, flush=True)

    roofline = None
    if a.timing >= 2:
        cand = {k: v for k, v in kstats.items() if v["ms"] > 0 and v["bytes"] > 0}
        if cand:
            dom = max(cand, key=lambda k: cand[k]["ms"])
            v = cand[dom]
            achieved = v["bytes"] / (v["ms"] * 1e-3) / 1e9
            roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": KERNEL_NAMES.get(dom, dom), "kernel_class": dom,
                        "launches": v["launches"], "avg_launch_us": round(1000.0 * v["ms"] / max(v["launches"], 1), 3),
                        "bytes_per_launch": round(v["bytes"] / max(v["launches"], 1), 1)}
        print("[bench] kernel classes over the timed region: " +
              ", ".join(f"{k}={v['ms']:.2f}ms/{v['launches']}" for k, v in kstats.items()), file=sys.stderr,
              flush=True)

    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        og = oracle.CSR.of(g)
        t1 = time.perf_counter()
        r = oracle.louvain(og, tolerance=a.tolerance, max_passes=a.max_passes, sync=False)
        dt = time.perf_counter() - t1
        cpu = {"value": round(g.nnz / dt, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": f"one full run of the sequential oracle (asynchronous, the paper's loop on one thread) "
                         f"on the same R-MAT scale {a.scale} graph: {dt:.2f}s, Q={r.modularity:.6f}"}
        print(f"[bench] oracle run {dt:.2f}s Q={r.modularity:.6f}", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "edges/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"rmat{a.scale}: R-MAT scale {a.scale}, 16 samples/vertex, a/b/c/d .57/.19/.19/.05, "
                               f"symmetrised, dedup, unit weights; plain GSP-Louvain tol {a.tolerance}, "
                               f"<= {a.max_passes} passes, 8 sub-rounds",
                   "n": g.n, "nnz": g.nnz, "modularity": round(q, 6), "disconnected": disc,
                   "passes": st["passes"], "prune": "plain",
                   "phase_ms_per_run": {k: round(v / a.steps, 3) for k, v in phase.items()}},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
