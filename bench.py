"""Benchmark: full GSP-Louvain runs on one MI355X, learned-pruned against plain.

Default workload (the largest single-GPU one): R-MAT scale 26 (2^26
vertices, 2^30 samples, a/b/c/d = .57/.19/.19/.05, symmetrised, deduplicated,
no self-loops, symmetric fp32 weights U[1, 10), about 2.1e9 directed
entries).  --workload rmat20 / dcsbm4m selects the smaller ones.  The graph
is generated (seeded) and loaded once into the library's device memory; runs
of gsp_run (tolerance 1e-2, at most 10 passes) follow:

  * warm-up: `warmup` plain and `warmup` learned-pruned runs;
  * timed region: `steps` learned-pruned runs (network 8-64-64-1 trained on
    the degree-corrected SBM traces, threshold theta), bracketed by
    synchronisations; value = directed CSR entries / seconds per run.  HIP
    events record the dominant kernel class only (picked by one probe run
    per class); with them a sub-round's scans run one after another (timing
    2), so that an event pair holds that kernel alone (--timing 3 keeps the
    scans side by side, each pair on its kernel's stream, and then times the
    kernel as it shares the GPU);
  * the same number of plain runs with the same events: the comparison
    (config.plain, config.vs_plain) and the local-moving phase's
    algorithmic GB/s (scan bytes over the phase's event time);
  * the same runs without any events (config.untimed);
  * GSP-Leiden runs (the refinement in every pass) without events, after one
    warm-up run (config.leiden);
  * a CPU baseline: the sequential oracle on one pinned host core, on a
    bounded sample of the same graph.

Prints ONE JSON line (metric, value, roofline of the dominant kernel,
cpu_baseline, ...); progress goes to stderr.
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
# kernel classes of the local-moving scans whose algorithmic bytes the
# library counts (compaction and apply are left out: a lower bound)
SCAN_CLASSES = ("move_small", "move_wave", "move_block", "move_hub", "move_hub_finish", "move_hub_gather", "gate")
WORKLOADS = {
    "rmat26": dict(kind="rmat", scale=26, seed=26, weights=(1.0, 10.0),
                   text="R-MAT scale 26, 2^30 samples, a/b/c/d .57/.19/.19/.05, symmetrised, dedup, no "
                        "self-loops, fp32 weights U[1,10)"),
    "rmat20": dict(kind="rmat", scale=20, seed=20, weights=None,
                   text="R-MAT scale 20, 16 samples/vertex, a/b/c/d .57/.19/.19/.05, symmetrised, dedup, "
                        "unit weights"),
    "dcsbm4m": dict(kind="dcsbm", seed=1000,
                    text="degree-corrected SBM, 4M vertices, degrees power law 2.5 on [5, 5000], communities "
                         "power law 1.5 on [20, 50000], mixing 0.3, fp32 weights U[1,4), held-out seed 1000"),
}
ORDERS = {"auto": 0, "loaded": 1, "degree": 2}
GOLDEN_ASYNC = os.path.join(ROOT, "tests", "golden", "async_q.json")
GOLDEN_KEY = {"rmat26": "rmat26", "rmat20": "rmat20", "dcsbm4m": "dcsbm4m_s1000"}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="rmat26", choices=sorted(WORKLOADS))
    p.add_argument("--tolerance", type=float, default=1e-2)
    p.add_argument("--max-passes", type=int, default=10)
    p.add_argument("--theta", type=float, default=None, help="learned gate threshold on p (default: the shipped network's)")
    p.add_argument("--timing", type=int, default=2, choices=(2, 3),
                   help="2: events with a sub-round's scans one after another; 3: events on each kernel's own "
                        "stream, scans side by side")
    p.add_argument("--cpu-sample", type=int, default=4, help="the CPU baseline scans every k-th vertex")
    p.add_argument("--vertex-order", default="auto", choices=sorted(ORDERS),
                   help="storage order of the graph inside the runs (auto: degree order from 2^25 entries)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-untimed", action="store_true", help="skip the runs without events")
    p.add_argument("--no-leiden", action="store_true", help="skip the GSP-Leiden runs")
    p.add_argument("--kernel-class", default="", choices=[""] + sorted(KERNEL_NAMES),
                   help="time this kernel class (no probe runs)")
    p.add_argument("--only-timed", action="store_true",
                   help="warm-up and timed learned-pruned runs only, all with the same events (for a kernel "
                        "trace whose per-kernel averages are those of the timed region)")
    return p.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


def traffic_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    this workload, if taken on the kernel's current sources (else None)."""
    try:
        with open(traffic_file(workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    k = t.get("kernels", {}).get(kernel)
    if t.get("workload") != workload or k is None or k.get("source_hash") != kernel_source_hash(kernel):
        return None
    return k.get("bytes_per_launch")


def make_graph(name):
    import gsp_inputs as gi
    w = WORKLOADS[name]
    if w["kind"] == "rmat":
        gi.set_verbose(w["scale"] > 22)
        g = gi.rmat(w["scale"], 16, *gi.RMAT_ABC, w["seed"], weights=w["weights"], name=f"rmat-{w['scale']}")
        gi.set_verbose(False)
        return g
    return gi.dcsbm_4m(w["seed"])


def timed_runs(ctx, gsp, a, steps, **kw):
    """`steps` whole runs between two device synchronisations: (seconds,
    per-class kernel totals, per-phase ms totals, last stats)."""
    import torch
    kst = {k: dict(launches=0, ms=0.0, bytes=0.0, items=0) for k in gsp.KERNEL_CLASSES}
    ph = dict(ms_move=0.0, ms_split=0.0, ms_aggregate=0.0, ms_other=0.0, ms_total=0.0)
    st = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run(a.tolerance, a.max_passes, vertex_order=ORDERS[a.vertex_order], **kw)
        st = ctx.stats()
        for name, v in st["kernels"].items():
            for f in ("launches", "ms", "bytes", "items"):
                kst[name][f] += v[f]
        for f in ph:
            ph[f] += st[f]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, kst, ph, st


def host_cpu():
    """(model name, logical CPUs of the host, CPUs this process may use)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except OSError:
        allowed = os.cpu_count() or 1
    return model, os.cpu_count() or 1, allowed


def cpu_baseline(g, every, gpu_scanned, nnz):
    """The oracle's synchronous scan-and-decide step (its local-moving inner
    loop) from singleton communities over every `every`-th vertex, timed on
    one pinned host core; scaled to the metric's unit by the entries the
    GPU's run scanned in its local-moving phases."""
    import numpy as np
    import oracle
    model, ncpu, allowed = host_cpu()
    cpu = sorted(os.sched_getaffinity(0))[0] if hasattr(os, "sched_getaffinity") else 0
    og = oracle.CSR.of(g)
    K, M2 = oracle.vertex_weights(og)
    memb = np.arange(og.n, dtype=np.int32)
    active = np.zeros(og.n, dtype=np.uint8)
    active[::every] = 1
    entries = int(np.diff(og.off)[::every].sum())
    prev = os.sched_getaffinity(0) if hasattr(os, "sched_setaffinity") else None
    if prev is not None:
        os.sched_setaffinity(0, {cpu})
    try:
        t0 = time.perf_counter()
        dec, gain, moved = oracle.move_sync_step(og, memb, active, K=K, M2=M2)
        dt = time.perf_counter() - t0
    finally:
        if prev is not None:
            os.sched_setaffinity(0, prev)
    rate = entries / dt
    run_s = gpu_scanned / rate          # the GPU run's scanned entries at the oracle's rate
    return {"value": round(nnz / run_s, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
            "scan_entries_per_s": round(rate, 1), "cpu_model": model, "host_cpus": ncpu, "cpus_allowed": allowed,
            "pinned_cpu": cpu,
            "sample": f"the oracle's synchronous scan-and-decide step (its local-moving inner loop) from singleton "
                      f"communities over every {every}-th vertex of the same graph: {entries} entries in {dt:.2f}s "
                      f"on 1 of {ncpu} host cores ({model}), pinned to core {cpu}; scaled to a full run by the "
                      f"{gpu_scanned} entries the GPU run's local-moving phases scan (split and aggregation left "
                      f"out, which favours the CPU); {moved} of the sampled vertices moved"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {a.gpus} is not supported "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2402_11454_amd as gsp
    from paper_2402_11454_amd.train_pruner import DEFAULT_OUT, THETA_BY_CLASS, load_params

    if a.theta is None:   # the shipped network's threshold for this graph class
        a.theta = THETA_BY_CLASS[WORKLOADS[a.workload]["kind"]]
    t0 = time.time()
    g = make_graph(a.workload)
    log(f"generated {a.workload}: n={g.n} nnz={g.nnz} in {time.time() - t0:.1f}s")
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = gsp.Context(0, stream=stream)
    ctx.load_graph(g)
    grid = ctx.weight_grid()
    ctx.pruner_set(load_params(DEFAULT_OUT))
    learned_kw = dict(prune_mode=gsp.PRUNE_LEARNED, prune_threshold=a.theta)
    if a.only_timed:
        if not a.kernel_class:
            sys.exit("--only-timed needs --kernel-class")
        ev = dict(timing=a.timing, timing_mask=1 << gsp.KERNEL_CLASSES.index(a.kernel_class))
        for _ in range(a.warmup):
            ctx.run(a.tolerance, a.max_passes, vertex_order=ORDERS[a.vertex_order], **ev, **learned_kw)
        elapsed, kst, _, st_l = timed_runs(ctx, gsp, a, a.steps, **ev, **learned_kw)
        v = kst[a.kernel_class]
        print(json.dumps({"workload": a.workload, "ms_per_step": round(1000.0 * elapsed / a.steps, 4),
                          "kernel": KERNEL_NAMES[a.kernel_class], "launches": v["launches"],
                          "avg_launch_us": round(1000.0 * v["ms"] / max(v["launches"], 1), 3),
                          "bytes_per_launch": round(v["bytes"] / max(v["launches"], 1), 1)}), flush=True)
        ctx.close()
        return
    for _ in range(a.warmup):
        ctx.run(a.tolerance, a.max_passes, vertex_order=ORDERS[a.vertex_order])
        ctx.run(a.tolerance, a.max_passes, vertex_order=ORDERS[a.vertex_order], **learned_kw)
    log(f"{a.warmup} warm-up run(s) of each method done")

    # the dominant single-kernel class of the learned runs: one probe run per
    # class with only that class's events (events around every kernel would
    # slow the host and inflate the short kernels' times)
    if a.kernel_class:
        dom = a.kernel_class
    else:
        cand = {}
        for k in KERNEL_NAMES:
            ctx.run(a.tolerance, a.max_passes, vertex_order=ORDERS[a.vertex_order], timing=a.timing, timing_mask=1 << gsp.KERNEL_CLASSES.index(k),
                    **learned_kw)
            ms = ctx.stats()["kernels"][k]["ms"]
            if ms > 0:
                cand[k] = ms
        dom = max(cand, key=cand.get)
        log("probe ms per class: " + ", ".join(f"{k} {v:.3f}" for k, v in sorted(cand.items())))
    ev = dict(timing=a.timing, timing_mask=1 << gsp.KERNEL_CLASSES.index(dom))

    # timed region: `steps` learned-pruned runs, graph resident in HBM
    elapsed, kst, ph_l, st_l = timed_runs(ctx, gsp, a, a.steps, **ev, **learned_kw)
    ms_per_step = 1000.0 * elapsed / a.steps
    value = g.nnz / (elapsed / a.steps)
    memb_l = ctx.membership()
    q_l = ctx.result_modularity()
    disc_l = ctx.count_disconnected(memb_l)
    log(f"learned: {a.steps} runs, {ms_per_step:.3f} ms/run, Q={q_l:.6f}, disconnected={disc_l}, "
        f"iterations={st_l['iterations']}, scanned={st_l['scanned_entries']}")

    # the comparison: plain runs with the same events
    el_p, kst_p, ph_p, st_p = timed_runs(ctx, gsp, a, a.steps, **ev)
    ms_p = 1000.0 * el_p / a.steps
    value_p = g.nnz / (el_p / a.steps)
    memb_p = ctx.membership()
    q_p = ctx.result_modularity()
    disc_p = ctx.count_disconnected(memb_p)
    log(f"plain: {ms_p:.3f} ms/run, Q={q_p:.6f}, disconnected={disc_p}, iterations={st_p['iterations']}, "
        f"scanned={st_p['scanned_entries']}")

    def move_phase(kstats, phases):
        b = sum(kstats[k]["bytes"] for k in SCAN_CLASSES)
        s = phases["ms_move"] * 1e-3
        return {"scan_bytes_per_run": round(b / a.steps, 1), "ms_per_run": round(phases["ms_move"] / a.steps, 3),
                "algorithmic_GBps": round(b / s / 1e9, 1) if s > 0 else None,
                "frac_of_hbm_peak": round(b / s / 1e9 / HBM_PEAK_GBS, 4) if s > 0 else None}

    untimed = None
    if not a.no_untimed:
        el0, _, _, _ = timed_runs(ctx, gsp, a, a.steps)
        el1, _, _, _ = timed_runs(ctx, gsp, a, a.steps, **learned_kw)
        untimed = {"plain_ms_per_step": round(1000.0 * el0 / a.steps, 3),
                   "learned_ms_per_step": round(1000.0 * el1 / a.steps, 3),
                   "vs_plain": round(el0 / el1, 4)}
        log(f"no events: plain {untimed['plain_ms_per_step']} ms, learned {untimed['learned_ms_per_step']} ms")

    leiden = None
    if not a.no_leiden:
        vo = ORDERS[a.vertex_order]
        ctx.run(a.tolerance, a.max_passes, vertex_order=vo, leiden=1)
        el_d, _, _, st_d = timed_runs(ctx, gsp, a, a.steps, leiden=1)
        memb_d = ctx.membership()
        q_d = ctx.result_modularity()
        leiden = {"ms_per_step": round(1000.0 * el_d / a.steps, 3), "value": round(g.nnz / (el_d / a.steps), 1),
                  "modularity": round(q_d, 6), "disconnected": ctx.count_disconnected(memb_d),
                  "passes": st_d["passes"], "iterations": st_d["iterations"], "refined": st_d["refined"],
                  "time_vs_plain_untimed": None if untimed is None else
                  round(1000.0 * el_d / a.steps / untimed["plain_ms_per_step"], 4)}
        log(f"GSP-Leiden: {leiden['ms_per_step']} ms/run, Q={q_d:.6f}, passes={st_d['passes']}")

    v = kst[dom]
    achieved = v["bytes"] / (v["ms"] * 1e-3) / 1e9
    kern = KERNEL_NAMES[dom]
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kern, a.workload),
                "kernel": kern, "kernel_class": dom, "launches": v["launches"],
                "avg_launch_us": round(1000.0 * v["ms"] / max(v["launches"], 1), 3),
                "bytes_per_launch": round(v["bytes"] / max(v["launches"], 1), 1)}

    q_async = None
    if os.path.exists(GOLDEN_ASYNC):
        ref = json.load(open(GOLDEN_ASYNC)).get(GOLDEN_KEY[a.workload])
        if ref and ref.get("nnz") == g.nnz:
            q_async = ref["modularity"]
    ratio = value / value_p
    equal_q = abs(q_l - q_p) <= 0.005
    quality = {"plain_minus_async": None if q_async is None else round(q_p - q_async, 6),
               "learned_minus_async": None if q_async is None else round(q_l - q_async, 6),
               "async_oracle": q_async}
    target = {"ratio_at_least": 1.3, "ratio": round(ratio, 4), "equal_modularity": equal_q,
              "no_disconnected": disc_l == 0 and disc_p == 0,
              "met": bool(ratio >= 1.3 and equal_q and disc_l == 0 and disc_p == 0)}

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(g, a.cpu_sample, st_p["scanned_entries"], g.nnz)
        log(f"cpu baseline: {cpu['sample']}")

    w = WORKLOADS[a.workload]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "edges/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {w['text']}; GSP-Louvain tol {a.tolerance}, <= {a.max_passes} "
                               f"passes, 8 sub-rounds; value = learned-pruned runs (8-64-64-1 gate trained on "
                               f"DC-SBM traces, theta {a.theta}: this class's threshold, chosen on a held-out "
                               f"graph), plain runs beside",
                   "n": g.n, "nnz": g.nnz, "weight_grid_exp": grid[0], "weights_moved_to_grid": grid[1],
                   "vertex_order": a.vertex_order + (" (degree order at this size)" if a.vertex_order == "auto"
                                                     and g.nnz >= 1 << 25 else ""),
                   "modularity": round(q_l, 6), "disconnected": disc_l, "passes": st_l["passes"],
                   "iterations": st_l["iterations"], "scanned_entries": st_l["scanned_entries"],
                   "pruned": st_l["pruned"], "confirm_sweeps": st_l["confirm_sweeps"],
                   "vs_plain": round(ratio, 4),
                   "plain": {"value": round(value_p, 1), "ms_per_step": round(ms_p, 4), "modularity": round(q_p, 6),
                             "disconnected": disc_p, "passes": st_p["passes"], "iterations": st_p["iterations"],
                             "scanned_entries": st_p["scanned_entries"],
                             "local_moving": move_phase(kst_p, ph_p),
                             "phase_ms_per_run": {k: round(x / a.steps, 3) for k, x in ph_p.items()}},
                   "learned_local_moving": move_phase(kst, ph_l),
                   "modularity_minus_plain": round(q_l - q_p, 6), "quality": quality, "target": target,
                   "untimed": untimed, "leiden": leiden},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
