"""HBM traffic of the library's kernels from rocprofv3 hardware counters.

Two profiling passes over the same workload, one per counter (FETCH_SIZE,
then WRITE_SIZE, in KiB per dispatch), each also covering an elementwise
kernel of known traffic (y = 2x over 1 GiB: reads 1 GiB, writes 1 GiB);
its counters give the scale from counter KiB to bytes.  The summary (per kernel: dispatches, mean KiB read and written,
scaled bytes per dispatch) goes to profiles/traffic.json with a hash of the
kernel's sources (its file, the headers, the host code), and a readable table to profiles/traffic_rmat20.md.

    python -m paper_2402_11454_amd.pmc_traffic --run            # the workload (under rocprofv3)
    python -m paper_2402_11454_amd.pmc_traffic --summarize FETCH_DB WRITE_DB --cmd "..."

--scale/--seed/--weights choose another R-MAT graph (as bench.py builds
it); its summary goes to profiles/traffic_rmat<scale>.json and .md (the
R-MAT 20 one, which bench.py reads, to profiles/traffic.json).
"""
import argparse
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_BYTES = 1 << 30


def run_workload(runs: int, scale: int = 20, seed: int = 20, weights=None):
    sys.path.insert(0, ROOT)
    import torch
    import gsp_inputs as gi
    import paper_2402_11454_amd as gsp
    torch.cuda.init()
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    if scale == 20 and seed == 20 and weights is None:
        g = gi.rmat20()
    else:
        g = gi.rmat(scale, 16, *gi.RMAT_ABC, seed, weights=weights, name=f"rmat-{scale}")
    print(f"[pmc] graph ready: n={g.n} nnz={g.nnz}", flush=True)
    ctx = gsp.Context(0, stream=torch.cuda.current_stream())
    ctx.load_graph(g)
    for k in range(runs):
        ctx.run(1e-2, 10)
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


def summarize(fetch_db, write_db, cmd, scale: int = 20):
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
    out = {"workload": f"rmat{scale}", "command": cmd, "copy_kernel": short(copy),
           "scale_fetch": f_scale, "scale_write": w_scale, "kernels": kernels}
    prof = os.path.join(ROOT, "profiles")
    with open(os.path.join(prof, "traffic.json" if scale == 20 else f"traffic_rmat{scale}.json"), "w") as f:
        json.dump(out, f, indent=1)
    with open(os.path.join(prof, f"traffic_rmat{scale}.md"), "w") as f:
        f.write(f"# HBM traffic per dispatch: plain GSP-Louvain on R-MAT scale {scale}\n\n")
        f.write(f"Command (two passes, one counter each):\n\n```\n{cmd}\n```\n\n")
        f.write(f"Scale: y = 2x over {COPY_BYTES} bytes (`{short(copy)[:60]}`) reads {fe[copy][1]:.0f} KiB "
                f"(FETCH_SIZE) -> factor {f_scale:.4f}; write factor {w_scale:.4f}.\n\n")
        f.write("| kernel | dispatches | FETCH KiB | WRITE KiB | scaled bytes / dispatch |\n|---|---:|---:|---:|---:|\n")
        for k, n, fk, wk, b in rows[:30]:
            f.write(f"| `{k}` | {n} | {fk:.1f} | {wk:.1f} | {b:.0f} |\n")
    print(json.dumps(out)[:400])


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--run", action="store_true")
    ap.add_argument("--runs", type=int, default=2)
    ap.add_argument("--summarize", nargs=2)
    ap.add_argument("--cmd", default="")
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--seed", type=int, default=20)
    ap.add_argument("--weights", default="", help="lo,hi: symmetric fp32 weights U[lo,hi)")
    a = ap.parse_args()
    if a.run:
        wts = tuple(float(v) for v in a.weights.split(",")) if a.weights else None
        run_workload(a.runs, a.scale, a.seed, wts)
    if a.summarize:
        summarize(a.summarize[0], a.summarize[1], a.cmd, a.scale)
