"""HBM traffic of the library's kernels from rocprofv3 hardware counters,
for bench.py's roofline (its `traffic` field).

Two profiling passes over the same workload, one per counter (FETCH_SIZE,
then WRITE_SIZE, in KiB per dispatch), each also covering an elementwise
kernel of known traffic (y = 2x over 1 GiB: reads 1 GiB, writes 1 GiB);
its counters give the scale from counter KiB to bytes.  The summary (per
kernel: dispatches, mean KiB read and written, scaled bytes per dispatch)
goes to profiles/traffic_<workload>.json with a hash of the kernel's sources
(its file, the headers, the host code), and a readable table to
profiles/traffic_<workload>.md.  Workloads as bench.py names them
(rmat26, rmat20, dcsbm4m); --learned profiles learned-pruned runs.

    python bench_traffic.py --run --workload rmat26            # the workload (under rocprofv3)
    python bench_traffic.py --summarize FETCH_DB WRITE_DB --workload rmat26 --cmd "..."

Per phase: the counters' bytes of one run, phase by phase (local moving,
split, aggregation, the rest), over the phases' wall times from HIP events
(timing = 1: scans side by side, sweeps replayed from graphs, as in runs
without events):

    python bench_traffic.py --phase-times OUT.json --workload rmat26        # on the GPU
    python bench_traffic.py --phases TRAFFIC.json OUT.json --cmd "..."
"""
import argparse
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30


def run_workload(runs: int, workload: str, learned: bool, order: str = "auto", leiden: bool = False):
    sys.path.insert(0, ROOT)
    import torch
    import paper_2402_11454_amd as gsp
    from bench import make_graph
    from paper_2402_11454_amd.train_pruner import DEFAULT_OUT, THETA_BY_CLASS, load_params
    torch.cuda.init()
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    g = make_graph(workload)
    print(f"[pmc] graph ready: n={g.n} nnz={g.nnz}", flush=True)
    ctx = gsp.Context(0, stream=torch.cuda.current_stream())
    ctx.load_graph(g)
    from bench import ORDERS
    kw = dict(vertex_order=ORDERS[order])
    if learned:
        ctx.pruner_set(load_params(DEFAULT_OUT))
        from bench import WORKLOADS
        kw.update(prune_mode=gsp.PRUNE_LEARNED, prune_threshold=THETA_BY_CLASS[WORKLOADS[workload]["kind"]])
    if leiden:
        kw.update(leiden=1)
    for k in range(runs):
        ctx.run(1e-2, 10, **kw)
        print(f"[pmc] run {k + 1}/{runs}", flush=True)
    ctx.close()


def per_kernel(db: str, counter: str):
    """{kernel name: (dispatches, mean counter value)} from a results db."""
    con = sqlite3.connect(db)
    cur = con.cursor()
    tables = [r[0] for r in cur.execute("select name from sqlite_master where type in ('table','view')")]
    # rocprofv3 keeps one row per (dispatch, counter); the view joins names
    view = next((t for t in ("counters_collection", "counters") if t in tables), None)
    if view is None:
        raise SystemExit(f"{db}: no counter table among {tables}")
    cols = [r[1] for r in cur.execute(f"pragma table_info({view})")]
    name_col = next(c for c in ("kernel_name", "name") if c in cols)
    cnt_col = next(c for c in ("counter_name", "counter") if c in cols)
    val_col = next(c for c in ("value", "counter_value") if c in cols)
    disp_col = next((c for c in ("dispatch_id", "correlation_id", "id") if c in cols), None)
    q = (f"select {name_col}, count(distinct {disp_col}), sum({val_col}) from {view} "
         f"where {cnt_col} = ? group by {name_col}")
    out = {}
    for name, n, total in cur.execute(q, (counter,)):
        out[name] = (int(n), float(total) / max(int(n), 1))
    return out


def short(name: str) -> str:
    import re
    s = re.sub(r"gsp::\(anonymous namespace\)::", "", name)
    s = re.sub(r"\(.*", "", s)
    return s.replace("void ", "")


def summarize(fetch_db, write_db, cmd, workload: str, runs: int = 2, tag: str = ""):
    sys.path.insert(0, ROOT)
    from bench import kernel_source_hash
    fe = per_kernel(fetch_db, "FETCH_SIZE")
    wr = per_kernel(write_db, "WRITE_SIZE")
    copy = [k for k in fe if "MulFunctor" in k]
    copy = max(copy, key=lambda k: fe[k][1])
    # y = 2x over COPY_BYTES reads and writes COPY_BYTES
    f_scale = COPY_BYTES / (fe[copy][1] * 1024.0)
    w_scale = COPY_BYTES / (wr[copy][1] * 1024.0) if copy in wr else f_scale
    kernels = {}
    rows = []
    for name, (n, f_kib) in sorted(fe.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        if name == copy:
            continue
        w_kib = wr.get(name, (0, 0.0))[1]
        b = f_kib * 1024.0 * f_scale + w_kib * 1024.0 * w_scale
        # every instantiation of a kernel together (bench times them as one
        # class): dispatch-weighted means
        k = short(name).split("<")[0]
        acc = kernels.setdefault(k, {"dispatches": 0, "fetch_kib": 0.0, "write_kib": 0.0, "bytes_per_launch": 0.0})
        acc["dispatches"] += n
        acc["fetch_kib"] += f_kib * n
        acc["write_kib"] += w_kib * n
        acc["bytes_per_launch"] += b * n
        rows.append((short(name), n, f_kib, w_kib, b))
    for name, acc in kernels.items():
        n = max(acc["dispatches"], 1)
        for f in ("fetch_kib", "write_kib", "bytes_per_launch"):
            acc[f] = round(acc[f] / n, 1)
        acc["source_hash"] = kernel_source_hash(name)
    out = {"workload": workload, "command": cmd, "runs": runs, "copy_kernel": short(copy),
           "scale_fetch": f_scale, "scale_write": w_scale, "kernels": kernels}
    prof = os.path.join(ROOT, "profiles")
    with open(os.path.join(prof, f"traffic_{workload}{tag}.json"), "w") as f:
        json.dump(out, f, indent=1)
    with open(os.path.join(prof, f"traffic_{workload}{tag}.md"), "w") as f:
        kind = "plain" if tag == "_plain" else "learned-pruned"
        f.write(f"# Memory traffic per dispatch (FETCH_SIZE / WRITE_SIZE): {kind} GSP-Louvain on {workload}\n\n")
        f.write(f"Command (two passes, one counter each):\n\n```\n{cmd}\n```\n\n")
        f.write(f"Scale: y = 2x over {COPY_BYTES} bytes (`{short(copy)[:60]}`) reads {fe[copy][1]:.0f} KiB "
                f"(FETCH_SIZE) -> factor {f_scale:.4f}; write factor {w_scale:.4f}.\n\n")
        f.write("| kernel | dispatches | FETCH KiB | WRITE KiB | scaled bytes / dispatch |\n|---|---:|---:|---:|---:|\n")
        for k, n, fk, wk, b in rows[:30]:
            f.write(f"| `{k}` | {n} | {fk:.1f} | {wk:.1f} | {b:.0f} |\n")
    print(json.dumps(out)[:400])


def phase_times(out_path: str, runs: int, workload: str):
    """Mean phase wall times (ms) of `runs` plain runs after two warm-up
    runs, and the algorithmic bytes of each kernel class (the library's
    counts) from one more run with per-kernel events."""
    sys.path.insert(0, ROOT)
    import paper_2402_11454_amd as gsp
    from bench import make_graph
    g = make_graph(workload)
    ctx = gsp.Context(0)
    ctx.load_graph(g)
    for _ in range(2):
        ctx.run(1e-2, 10, timing=1)
    acc = {k: 0.0 for k in ("ms_move", "ms_split", "ms_aggregate", "ms_other", "ms_total")}
    for k in range(runs):
        ctx.run(1e-2, 10, timing=1)
        st = ctx.stats()
        for f in acc:
            acc[f] += st[f] / runs
        print(f"[phases] run {k + 1}/{runs}: {st['ms_total']:.3f} ms", flush=True)
    ctx.run(1e-2, 10, timing=2)
    alg = {k: v["bytes"] for k, v in ctx.stats()["kernels"].items()}
    ctx.close()
    out = {"workload": workload, "n": int(g.n), "nnz": int(g.nnz), "runs": runs, **acc, "algorithmic_bytes": alg}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


# kernels that belong to one phase only (by name prefix); the fills, scans
# and renumbering kernels that every phase shares are not attributed, so a
# phase's bytes are a lower bound while its time includes them
PHASE_OF = (("move", ("k_move", "k_hub", "k_gate")), ("split", ("k_split",)),
            ("aggregate", ("k_agg", "k_member_degrees")))
# the library's kernel classes of each phase (algorithmic bytes)
PHASE_CLASSES = {"move": ("move_small", "move_wave", "move_block", "move_hub", "move_hub_finish", "move_hub_gather",
                          "move_apply", "frontier", "gate"),
                 "split": ("split",), "aggregate": ("aggregate",)}


def phases(traffic_json: str, times_json: str, cmd: str):
    with open(traffic_json) as f:
        tr = json.load(f)
    with open(times_json) as f:
        tm = json.load(f)
    runs = tr.get("runs", 1)
    byts = {"move": 0.0, "split": 0.0, "aggregate": 0.0}
    for name, v in tr["kernels"].items():
        ph = next((p for p, pre in PHASE_OF if name.startswith(pre)), None)
        if ph:
            byts[ph] += v["bytes_per_launch"] * v["dispatches"] / runs
    ms = {"move": tm["ms_move"], "split": tm["ms_split"], "aggregate": tm["ms_aggregate"]}
    alg = {p: sum(tm.get("algorithmic_bytes", {}).get(k, 0.0) for k in cl) for p, cl in PHASE_CLASSES.items()}
    w = tm["workload"]
    path = os.path.join(ROOT, "profiles", f"phases_{w}.md")
    with open(path, "w") as f:
        f.write(f"# Bytes per phase: plain GSP-Louvain on {w} (n={tm['n']}, {tm['nnz']} entries)\n\n")
        f.write(f"Commands:\n\n```\n{cmd}\n```\n\n")
        f.write(f"Time: the phases' wall times from HIP events, mean of {tm['runs']} runs with timing = 1 (scans "
                f"side by side, sweeps replayed from graphs); whole run {tm['ms_total']:.3f} ms (other steps "
                f"{tm['ms_other']:.3f} ms).\n\n"
                f"Algorithmic bytes: the bytes the method must move by the library's per-class counts (one run "
                f"with per-kernel events); their rate is the one compared with the HBM peak (8000 GB/s).\n\n"
                f"Counter bytes: FETCH + WRITE of one run ({traffic_json}, {runs} run(s) under counters) of the "
                f"kernels that belong to one phase (fills, scans and renumbering shared by the phases left out), "
                f"scaled by an elementwise kernel of known traffic.  FETCH_SIZE / WRITE_SIZE count the L2's "
                f"requests to the memory side, Infinity Cache hits included, and every random 4- or 8-byte "
                f"gather moves a whole line: this rate is memory-side traffic, an upper bound of HBM traffic, "
                f"not HBM bandwidth.\n\n")
        f.write("| phase | ms per run | algorithmic GB per run | algorithmic GB/s | of HBM peak | counter GB per run "
                "| counter GB/s | counter / algorithmic |\n|---|---:|---:|---:|---:|---:|---:|---:|\n")
        for p in ("move", "split", "aggregate"):
            t = ms[p] * 1e-3
            ga = alg[p] / 1e9 / t if t > 0 else 0.0
            gc = byts[p] / 1e9 / t if t > 0 else 0.0
            amp = f"{byts[p] / alg[p]:.1f}x" if alg[p] > 0 else ""
            f.write(f"| {p} | {ms[p]:.3f} | {alg[p] / 1e9:.3f} | {ga:.0f} | {ga / 8000.0:.1%} | "
                    f"{byts[p] / 1e9:.3f} | {gc:.0f} | {amp} |\n")
    print(open(path).read())


def counter_summary(dbs, cmd: str, title: str, out_md: str, kernels):
    """Per-kernel means of every counter found in one or more rocprofv3
    --pmc databases (all instantiations of a kernel together), as a
    markdown table restricted to `kernels` (short names; empty: all)."""
    vals = {}
    for db in dbs:
        con = sqlite3.connect(db)
        cur = con.cursor()
        cols = [r[1] for r in cur.execute("pragma table_info(counters_collection)")]
        name_col = next(c for c in ("kernel_name", "name") if c in cols)
        cnt_col = next(c for c in ("counter_name", "counter") if c in cols)
        val_col = next(c for c in ("value", "counter_value") if c in cols)
        disp_col = next((c for c in ("dispatch_id", "correlation_id", "id") if c in cols), None)
        q = (f"select {name_col}, {cnt_col}, count(distinct {disp_col}), sum({val_col}) from counters_collection "
             f"group by {name_col}, {cnt_col}")
        for name, ctr, n, tot in cur.execute(q):
            k = short(name).split("<")[0]
            if kernels and k not in kernels:
                continue
            d = vals.setdefault(k, {})
            a = d.setdefault(ctr, [0, 0.0])
            a[0] += int(n)
            a[1] += float(tot)
    ctrs = sorted({c for d in vals.values() for c in d})
    with open(out_md, "w") as f:
        f.write(f"# Hardware counters per dispatch: {title}\n\nCommand (one pass per counter group):\n\n```\n{cmd}\n```\n\n")
        f.write("Mean per dispatch over every dispatch of the kernel (all instantiations).\n\n")
        f.write("| kernel | dispatches | " + " | ".join(ctrs) + " |\n|---|---:|" + "---:|" * len(ctrs) + "\n")
        for k in sorted(vals):
            n = max(a[0] for a in vals[k].values())
            row = [f"{vals[k][c][1] / max(vals[k][c][0], 1):.4g}" if c in vals[k] else "" for c in ctrs]
            f.write(f"| `{k}` | {n} | " + " | ".join(row) + " |\n")
        # ratios of counters of one kernel (means per dispatch)
        def mean(k, c):
            return vals[k][c][1] / max(vals[k][c][0], 1) if c in vals[k] else None
        f.write("\nDerived, per kernel: L2 hit rate = TCC_HIT / (TCC_HIT + TCC_MISS); L1 hit rate = 1 - "
                "TCP_TCC_READ_REQ / TCP_TOTAL_CACHE_ACCESSES; issue-wait share = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES "
                "(wave-cycles waiting for an instruction to issue over wave-cycles resident; waits on memory counters are SQ_WAIT_ANY, not this); waves per CU = 4 SQ_WAVE_CYCLES / "
                "(GRBM_GUI_ACTIVE / 8 XCDs) / 256 CUs (SQ wave-cycle counters taken in units of 4 cycles, "
                "GRBM_GUI_ACTIVE summed over the 8 XCDs); VMEM reads per wave = SQ_INSTS_VMEM_RD / SQ_WAVES.\n\n")
        f.write("| kernel | L2 hit | L1 hit | issue-wait share | waves per CU | VMEM reads per wave |\n|---|---:|---:|---:|---:|---:|\n")
        for k in sorted(vals):
            h, m = mean(k, "TCC_HIT_sum"), mean(k, "TCC_MISS_sum")
            rq, acc = mean(k, "TCP_TCC_READ_REQ_sum"), mean(k, "TCP_TOTAL_CACHE_ACCESSES_sum")
            wi, wc, ga = mean(k, "SQ_WAIT_INST_ANY"), mean(k, "SQ_WAVE_CYCLES"), mean(k, "GRBM_GUI_ACTIVE")
            vr, wv = mean(k, "SQ_INSTS_VMEM_RD"), mean(k, "SQ_WAVES")
            cells = [f"{100 * h / (h + m):.1f}%" if h is not None and m is not None and h + m > 0 else "",
                     f"{100 * (1 - rq / acc):.1f}%" if rq is not None and acc else "",
                     f"{100 * wi / wc:.1f}%" if wi is not None and wc else "",
                     f"{4 * wc / (ga / 8) / 256:.1f}" if wc is not None and ga else "",
                     f"{vr / wv:.0f}" if vr is not None and wv else ""]
            f.write(f"| `{k}` | " + " | ".join(cells) + " |\n")
    print(open(out_md).read())


def kernel_summary(db: str, cmd: str, title: str, out_md: str, bench_out: str = ""):
    """Per-kernel durations (all instantiations of a kernel together) from a
    rocprofv3 --kernel-trace database, as a markdown table."""
    con = sqlite3.connect(db)
    cur = con.cursor()
    rows = {}
    for name, dur in cur.execute("select name, duration from kernels"):
        k = short(name).split("<")[0]
        r = rows.setdefault(k, [0, 0.0, float("inf"), 0.0])
        d = float(dur) / 1e3   # ns -> us
        r[0] += 1
        r[1] += d
        r[2] = min(r[2], d)
        r[3] = max(r[3], d)
    total = sum(r[1] for r in rows.values())
    line = ""
    if bench_out and os.path.exists(bench_out):
        last = [x for x in open(bench_out).read().splitlines() if x.startswith("{")]
        if last:
            b = json.loads(last[-1])
            if "value" not in b:   # bench.py --only-timed: the timed runs' line
                b = {"ms_per_step": b["ms_per_step"], "value": None, "roofline": b,
                     "config": {"plain": {"ms_per_step": None}}}
            line = (f"Bench line of this command: {b['ms_per_step']} ms per learned-pruned run "
                    + (f"({b['value'] / 1e9:.3f} G entries/s), plain {b['config']['plain']['ms_per_step']} ms"
                       if b["value"] else "(warm-up and timed runs only)") + "; roofline "
                    f"kernel `{b['roofline']['kernel']}` {b['roofline']['avg_launch_us']} us per launch by events, "
                    f"{b['roofline']['bytes_per_launch']:.0f} algorithmic bytes per launch.\n\n")
    with open(out_md, "w") as f:
        f.write(f"# Kernel trace: {title}\n\nCommand:\n\n```\n{cmd}\n```\n\n")
        f.write(f"Kernel time summed over kernels (overlapping kernels on concurrent streams counted each): "
                f"{total / 1e3:.3f} ms, warm-up and probe runs included.\n\n{line}")
        f.write("| kernel | calls | total ms | avg us | min us | max us | share |\n"
                "|---|---:|---:|---:|---:|---:|---:|\n")
        for k, (n, t, lo, hi) in sorted(rows.items(), key=lambda kv: -kv[1][1])[:30]:
            f.write(f"| `{k}` | {n} | {t / 1e3:.3f} | {t / n:.2f} | {lo:.2f} | {hi:.2f} | {t / total:.1%} |\n")
    print(open(out_md).read())


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--run", action="store_true")
    ap.add_argument("--runs", type=int, default=2)
    ap.add_argument("--summarize", nargs=2)
    ap.add_argument("--cmd", default="")
    ap.add_argument("--workload", default="rmat26")
    ap.add_argument("--learned", action="store_true", help="learned-pruned runs (bench.py's timed runs)")
    ap.add_argument("--leiden", action="store_true", help="GSP-Leiden runs")
    ap.add_argument("--tag", default="", help="suffix of the summary's file names (e.g. _plain)")
    ap.add_argument("--vertex-order", default="auto", choices=("auto", "loaded", "degree"),
                    help="storage order of the graph inside the --run runs")
    ap.add_argument("--phase-times", default="", help="write the phases' mean wall times to this JSON")
    ap.add_argument("--phases", nargs=2, help="TRAFFIC_JSON TIMES_JSON: per-phase summary")
    ap.add_argument("--kernel-summary", nargs=2, metavar=("DB", "OUT_MD"),
                    help="per-kernel durations of a --kernel-trace database into a markdown table")
    ap.add_argument("--title", default="")
    ap.add_argument("--bench-out", default="", help="stdout of the profiled bench.py run (its JSON line)")
    ap.add_argument("--counter-summary", nargs="+", metavar="DB_OR_OUT",
                    help="DB [DB ...] OUT_MD: per-kernel means of the counters of --pmc databases")
    ap.add_argument("--kernels", default="", help="comma list of kernels for --counter-summary")
    a = ap.parse_args()
    if a.counter_summary:
        counter_summary(a.counter_summary[:-1], a.cmd, a.title, a.counter_summary[-1],
                        [k for k in a.kernels.split(",") if k])
    if a.kernel_summary:
        kernel_summary(a.kernel_summary[0], a.cmd, a.title, a.kernel_summary[1], a.bench_out)
    if a.run:
        run_workload(a.runs, a.workload, a.learned, a.vertex_order, a.leiden)
    if a.summarize:
        summarize(a.summarize[0], a.summarize[1], a.cmd, a.workload, a.runs, a.tag)
    if a.phase_times:
        phase_times(a.phase_times, 3, a.workload)
    if a.phases:
        phases(a.phases[0], a.phases[1], a.cmd)
