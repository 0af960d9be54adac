"""Benchmark: full GSP-Louvain runs on one MI355X.

Workload: R-MAT scale 20 (2^20 vertices, 16 samples per vertex, a/b/c/d =
.57/.19/.19/.05, symmetrised, deduplicated, no self-loops, unit weights).
The graph is generated (seeded) and loaded once into the library's device
memory; `warmup` untimed runs and `steps` timed runs of gsp_run (tolerance
1e-2, at most 10 passes) follow.

Prints ONE JSON line: edges/s = directed CSR entries / seconds per run of the
plain method; a roofline object for the dominant single-kernel class (its
algorithmic bytes from the library's counters over its HIP-event time,
events recorded around that class only, on the stream it runs on, inside the
timed region; a sub-round's scans then run one after another, so that an
event pair holds one kernel; --timing 3 keeps them side by side, each pair
on its kernel's stream); the same runs without events (scans side by side,
sweeps replayed from captured graphs) as config.untimed; the
learned-pruned method on the same graph (its edges/s, modularity and ratio
to plain, the network trained on the degree-corrected SBM workload); and a
CPU baseline: the sequential oracle timed on one host core on the same
graph (the synchronous method the GPU computes; the paper's asynchronous
loop beside it in the sample text).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edges/s per full GSP-Louvain run; learned-pruned vs plain at equal modularity"
HBM_PEAK_GBS = 8000.0
# single-kernel classes (the roofline names one kernel) -> the kernel
KERNEL_NAMES = {
    "move_small": "k_move_small",
    "move_wave": "k_move_wave",
    "move_block": "k_move_block",
    "move_hub": "k_hub_bucket",
    "move_hub_gather": "k_hub_gather",
    "move_apply": "k_move_apply",
    "frontier": "k_move_compact",
    "gate": "k_gate",
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--scale", type=int, default=20)
    p.add_argument("--seed", type=int, default=20)
    p.add_argument("--weights", default="", help="lo,hi: symmetric fp32 weights U[lo,hi) (e.g. 1,10 at scale 26)")
    p.add_argument("--tolerance", type=float, default=1e-2)
    p.add_argument("--max-passes", type=int, default=10)
    p.add_argument("--theta", type=float, default=0.5, help="learned gate threshold on p")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-learned", action="store_true")
    p.add_argument("--timing", type=int, default=2, choices=(0, 2, 3),
                   help="0: no per-kernel events (no roofline); 2: events with the scans of a sub-round one "
                        "after another; 3: events on each kernel's own stream, scans side by side")
    p.add_argument("--no-untimed", action="store_true", help="skip the runs without per-kernel events")
    return p.parse_args()


def _code_only(text: str) -> str:
    """C++ source without its comments and blank lines (comments do not
    change the compiled code)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = []
    for line in text.splitlines():
        # a // inside a string literal is no comment: mask literals, same length
        q = re.sub(r'"(\\.|[^"\\])*"', lambda m: '"' + "x" * (len(m.group(0)) - 2) + '"', line)
        cut = q.find("//")
        line = line[:cut] if cut >= 0 else line
        if line.strip():
            lines.append(line.rstrip())
    return "\n".join(lines)


def kernel_source_hash(kernel):
    """Hash of what decides a kernel's memory traffic: the code (comments
    left out) of the source file that defines it, the shared headers and
    the host code that launches it."""
    import re
    csrc = os.path.join(ROOT, "paper_2402_11454_amd", "csrc")
    names = sorted(os.listdir(csrc))
    pat = re.compile(r"__global__\s+void\s+(__launch_bounds__\([^)]*\)\s+)?" + re.escape(kernel) + r"\s*\(")
    files = [f for f in names if f.endswith(".hip") and pat.search(open(os.path.join(csrc, f)).read())]
    files += [f for f in names if f.endswith(".h")] + ["capi.hip"]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(csrc, f)) as fh:
            h.update(f.encode() + b"\0" + _code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken on this workload and on the kernel's current sources
    (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    k = t.get("kernels", {}).get(kernel)
    if t.get("workload") != workload or k is None or k.get("source_hash") != kernel_source_hash(kernel):
        return None
    return k.get("bytes_per_launch")


def timed_runs(ctx, gsp, a, steps, **kw):
    kstats = {k: dict(launches=0, ms=0.0, bytes=0.0, items=0) for k in gsp.KERNEL_CLASSES}
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run(a.tolerance, a.max_passes, **kw)
        st = ctx.stats()
        for name, v in st["kernels"].items():
            for f in ("launches", "ms", "bytes", "items"):
                kstats[name][f] += v[f]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, kstats


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
    wts = tuple(float(x) for x in a.weights.split(",")) if a.weights else None
    gi.set_verbose(a.scale > 22)
    g = gi.rmat(a.scale, 16, *gi.RMAT_ABC, a.seed, weights=wts, name=f"rmat-{a.scale}")
    print(f"[bench] generated R-MAT scale {a.scale}: n={g.n} nnz={g.nnz} in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = gsp.Context(0, stream=stream)
    ctx.load_graph(g)
    for w in range(a.warmup):
        ctx.run(a.tolerance, a.max_passes)
    print(f"[bench] {a.warmup} warm-up runs done", file=sys.stderr, flush=True)

    # which single-kernel class dominates: one probe run per class with only
    # that class's events (events around every kernel would slow the host and
    # inflate the short kernels' times)
    dom = None
    if a.timing >= 2:
        cand = {}
        for k in KERNEL_NAMES:
            ctx.run(a.tolerance, a.max_passes, timing=a.timing, timing_mask=1 << gsp.KERNEL_CLASSES.index(k))
            ms = ctx.stats()["kernels"][k]["ms"]
            if ms > 0:
                cand[k] = ms
        dom = max(cand, key=cand.get) if cand else None
        print("[bench] probe ms per class: " + ", ".join(f"{k} {v:.3f}" for k, v in sorted(cand.items())),
              file=sys.stderr, flush=True)
    mask = (1 << gsp.KERNEL_CLASSES.index(dom)) if dom else 0

    # timed region: `steps` whole runs of the plain method, graph resident in HBM
    elapsed, kstats = timed_runs(ctx, gsp, a, a.steps, timing=a.timing if dom else 0, timing_mask=mask)
    ms_per_step = 1000.0 * elapsed / a.steps
    value = g.nnz / (elapsed / a.steps)
    memb = ctx.membership()
    q = ctx.result_modularity()
    disc = ctx.count_disconnected(memb)
    st = ctx.stats()
    print(f"[bench] plain: {a.steps} runs, {ms_per_step:.3f} ms/run, Q={q:.6f}, disconnected={disc}, "
          f"passes={st['passes']} iterations={st['iterations']}", file=sys.stderr, flush=True)

    # the same runs without per-kernel events (sweeps then replayed from
    # captured graphs): context beside the timed value
    untimed = None
    if dom and not a.no_untimed:
        el0, _ = timed_runs(ctx, gsp, a, a.steps, timing=0)
        untimed = {"ms_per_step": round(1000.0 * el0 / a.steps, 4), "value": round(g.nnz / (el0 / a.steps), 1)}
        print(f"[bench] plain, no per-kernel events: {untimed['ms_per_step']:.3f} ms/run", file=sys.stderr, flush=True)

    roofline = None
    if dom:
        v = kstats[dom]
        achieved = v["bytes"] / (v["ms"] * 1e-3) / 1e9
        kern = KERNEL_NAMES[dom]
        per_launch = v["bytes"] / max(v["launches"], 1)
        tb = measured_traffic(kern, f"rmat{a.scale}" + (f"-w{a.weights}" if a.weights else ""))
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tb,
                    "kernel": kern, "kernel_class": dom, "launches": v["launches"],
                    "avg_launch_us": round(1000.0 * v["ms"] / max(v["launches"], 1), 3),
                    "bytes_per_launch": round(per_launch, 1)}

    learned = None
    if not a.no_learned:
        from paper_2402_11454_amd.train_pruner import DEFAULT_OUT, load_params
        if os.path.exists(DEFAULT_OUT):
            ctx.pruner_set(load_params(DEFAULT_OUT))
            kw = dict(prune_mode=gsp.PRUNE_LEARNED, prune_threshold=a.theta)
            for _ in range(a.warmup):
                ctx.run(a.tolerance, a.max_passes, **kw)
            el, _ = timed_runs(ctx, gsp, a, a.steps, **kw)
            # learned runs carry no per-kernel events: compare them with the
            # plain runs without events when those ran
            plain_ref = untimed["value"] if untimed else value
            ql = ctx.result_modularity()
            dl = ctx.count_disconnected(ctx.membership())
            sl = ctx.stats()
            learned = {"value": round(g.nnz / (el / a.steps), 1), "ms_per_step": round(1000.0 * el / a.steps, 4),
                       "vs_plain": round((g.nnz / (el / a.steps)) / plain_ref, 4), "modularity": round(ql, 6),
                       "modularity_minus_plain": round(ql - q, 6), "disconnected": dl, "theta": a.theta,
                       "scanned_entries": sl["scanned_entries"], "plain_scanned_entries": st["scanned_entries"],
                       "pruned": sl["pruned"], "iterations": sl["iterations"],
                       "network": "8-64-64-1, trained on degree-corrected SBM traces (seeds 0-31)"}
            print(f"[bench] learned: {learned['ms_per_step']:.3f} ms/run, Q={ql:.6f}, ratio {learned['vs_plain']}",
                  file=sys.stderr, flush=True)

    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        og = oracle.CSR.of(g)
        # the oracle of the GPU's results (ordered synchronous sub-rounds),
        # and the paper's asynchronous loop beside it
        t1 = time.perf_counter()
        r = oracle.louvain(og, tolerance=a.tolerance, max_passes=a.max_passes, sync=True, rounds=8)
        dt = time.perf_counter() - t1
        t1 = time.perf_counter()
        ra = oracle.louvain(og, tolerance=a.tolerance, max_passes=a.max_passes, sync=False)
        dta = time.perf_counter() - t1
        cpu = {"value": round(g.nnz / dt, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": f"one full run of the sequential oracle on the same R-MAT scale {a.scale} graph, the "
                         f"synchronous sub-round method the GPU computes (same membership): {dt:.2f}s, "
                         f"Q={r.modularity:.6f}; the paper's asynchronous loop on one thread: {dta:.2f}s "
                         f"({g.nnz / dta:.4g} edges/s), Q={ra.modularity:.6f}"}
        print(f"[bench] oracle runs: synchronous {dt:.2f}s Q={r.modularity:.6f}, asynchronous {dta:.2f}s "
              f"Q={ra.modularity:.6f}", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "edges/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"rmat{a.scale}: R-MAT scale {a.scale}, 16 samples/vertex, a/b/c/d .57/.19/.19/.05, "
                               f"symmetrised, dedup, {'weights U' + str(wts) if wts else 'unit weights'}; "
                               f"GSP-Louvain tol {a.tolerance}, "
                               f"<= {a.max_passes} passes, 8 sub-rounds; value = plain method",
                   "n": g.n, "nnz": g.nnz, "modularity": round(q, 6), "disconnected": disc,
                   "passes": st["passes"], "prune": "plain", "learned": learned, "untimed": untimed},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
