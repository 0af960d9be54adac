"""GSP-Leiden on the GPU (gsp_options.leiden, gsp_refine_phase) against the
oracle: the refinement phase alone (sub-community labels, iterations and
per-iteration gain totals, bit for bit) and whole runs (memberships,
modularity, per-pass local-moving and refinement statistics), in the loaded
order and in degree order, with every split mode.

The graphs cover hubs of more than 2048 entries (their same-community
subgraph rows are built chunk by chunk), rows of up to 2048 entries (in
256-row tiles) and short rows, unit, fp32 and fp64 weights, self-loops,
exact ties and a low-degree grid; the bounds cover a local-moving result,
one community for all, random communities and every vertex alone; the
options cover the split modes and algorithms, other sub-round counts, the
hubs' global-table path, per-kernel events and the return-move option.
"""
import numpy as np
import pytest

import gsp_inputs as gi
import oracle
import paper_2402_11454_amd as gsp

pytestmark = pytest.mark.gpu


def _gpu_count():
    try:
        import torch
        return torch.cuda.device_count()
    except Exception:
        return 0


@pytest.fixture(scope="module")
def ctx():
    if _gpu_count() == 0:
        pytest.skip("no GPU")
    c = gsp.Context(0)
    yield c
    c.close()


GRAPHS = {
    "sbm10k": lambda: gi.planted_sbm_10k(),
    "rmat12": lambda: gi.rmat_small(12, 12),
    "rmat15": lambda: gi.rmat_small(15, 3),
    "rmat15w": lambda: gi.rmat_small(15, 3, weights=(1.0, 4.0)),
    "rmat16w": lambda: gi.rmat_small(16, 7, weights=(1.0, 10.0)),
    "dcsbm50k": lambda: gi.dcsbm_small(50_000, 5),
    "road120": lambda: gi.road_small(120, 5),
}
_cache = {}


def _graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name]()
    return _cache[name]


def _bound(g, kind):
    if kind == "louvain":
        return oracle.louvain(g, tolerance=1e-2, max_passes=1, sync=True).membership
    if kind == "one":
        return np.zeros(g.n, dtype=np.int32)
    if kind == "alone":
        return np.arange(g.n, dtype=np.int32)
    return gi.random_membership(g.n, 40, 11)


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("kind", ["louvain", "one", "random", "alone"])
def test_refinement_equals_oracle(ctx, name, kind):
    g = _graph(name)
    ctx.load_graph(g)
    b = _bound(g, kind)
    print(f"[leiden] refine {name} bound={kind}", flush=True)
    got, li, dq, mv = ctx.refine_phase(b, tolerance=0.0)
    want, wli, wdq, wmv = oracle.refine_sync(g, b, tau=0.0, max_iter=20, rounds=8)
    np.testing.assert_array_equal(got, want)
    assert li == wli
    np.testing.assert_array_equal(mv, wmv)
    np.testing.assert_array_equal(dq, wdq)


@pytest.mark.parametrize("rounds", [1, 2, 64])
def test_refinement_other_sub_rounds(ctx, rounds):
    g = _graph("rmat15w")
    ctx.load_graph(g)
    b = _bound(g, "louvain")
    got, li, dq, _ = ctx.refine_phase(b, tolerance=1e-4, sub_rounds=rounds)
    want, wli, wdq, _ = oracle.refine_sync(g, b, tau=1e-4, max_iter=20, rounds=rounds)
    np.testing.assert_array_equal(got, want)
    assert li == wli
    np.testing.assert_array_equal(dq, wdq)


def test_refinement_from_merged_start(ctx):
    """Sub-communities of several vertices at the start keep their members."""
    g = _graph("rmat12")
    ctx.load_graph(g)
    b = _bound(g, "louvain")
    start = np.arange(g.n, dtype=np.int32)
    # pair up vertices of the same bound community
    for c in np.unique(b)[:200]:
        mem = np.flatnonzero(b == c)
        if mem.size >= 2:
            start[mem[1]] = mem[0]
    got, li, dq, _ = ctx.refine_phase(b, membership=start, tolerance=0.0)
    want, wli, wdq, _ = oracle.refine_sync(g, b, memb=start, tau=0.0, max_iter=20, rounds=8)
    np.testing.assert_array_equal(got, want)
    assert li == wli


def test_refinement_rejects_bad_start(ctx):
    g = _graph("rmat12")
    ctx.load_graph(g)
    b = _bound(g, "random")
    start = np.arange(g.n, dtype=np.int32)
    i = int(np.flatnonzero(b != b[0])[0])
    start[i] = 0   # vertex i joins vertex 0's sub-community across two bounds
    with pytest.raises(gsp.GspError):
        ctx.refine_phase(b, membership=start)
    bad = b.copy()
    bad[3] = g.n
    with pytest.raises(gsp.GspError):
        ctx.refine_phase(bad)
    # no refinement scans in the gate's training traces
    ctx.capture_traces(1000, 1.0, 1)
    try:
        with pytest.raises(gsp.GspError):
            ctx.refine_phase(b)
        with pytest.raises(gsp.GspError):
            ctx.louvain(1e-2, 10, leiden=1)
    finally:
        ctx.capture_traces(0, 1.0, 1)


def _check_run(res, ref):
    np.testing.assert_array_equal(res.membership, ref.membership)
    assert abs(res.modularity - ref.modularity) <= 1e-9
    st = res.stats
    assert st["passes"] == ref.passes
    assert st["iterations"] == ref.iterations
    assert st["communities"] == ref.communities
    assert st["vertices"] == ref.vertices
    assert st["refine_iterations"] == ref.refine_iterations
    assert st["refined"] == ref.refined


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("order", [gsp.ORDER_LOADED, gsp.ORDER_DEGREE])
def test_leiden_run_equals_oracle(ctx, name, order):
    g = _graph(name)
    ctx.load_graph(g)
    print(f"[leiden] run {name} order={order}", flush=True)
    res = ctx.louvain(1e-2, 10, leiden=1, vertex_order=order)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, leiden=True)
    _check_run(res, ref)
    assert ctx.count_disconnected(res.membership) == 0


@pytest.mark.parametrize("split_mode", [gsp.SPLIT_LAST, gsp.SPLIT_NONE])
@pytest.mark.parametrize("name", ["rmat15", "dcsbm50k"])
def test_leiden_split_modes(ctx, name, split_mode):
    g = _graph(name)
    ctx.load_graph(g)
    res = ctx.louvain(1e-2, 10, leiden=1, split_mode=split_mode)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, leiden=True,
                         split_mode=int(split_mode))
    _check_run(res, ref)


@pytest.mark.parametrize("max_passes", [0, 1, 2])
def test_leiden_pass_limits(ctx, max_passes):
    g = _graph("rmat15w")
    ctx.load_graph(g)
    res = ctx.louvain(1e-2, max_passes, leiden=1)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=max_passes, sync=True, rounds=8, leiden=True)
    np.testing.assert_array_equal(res.membership, ref.membership)
    assert res.stats["passes"] == ref.passes


def test_leiden_split_lpp_and_no_graphs(ctx):
    """The split algorithm and sweep replay do not change a run."""
    g = _graph("dcsbm50k")
    ctx.load_graph(g)
    a = ctx.louvain(1e-2, 10, leiden=1)
    b = ctx.louvain(1e-2, 10, leiden=1, split_algo=gsp.SPLIT_LPP, use_graphs=0)
    np.testing.assert_array_equal(a.membership, b.membership)
    assert a.stats["refined"] == b.stats["refined"]


def test_leiden_without_edges(ctx):
    g = gi.from_edges(50, [])
    ctx.load_graph(g)
    res = ctx.louvain(1e-2, 10, leiden=1)
    np.testing.assert_array_equal(res.membership, np.arange(50, dtype=np.int32))


def test_leiden_rejects_gate_and_batch(ctx):
    g = _graph("rmat12")
    ctx.load_graph(g)
    with pytest.raises(gsp.GspError):
        ctx.louvain(1e-2, 10, leiden=1, prune_mode=gsp.PRUNE_LEARNED)
    with pytest.raises(gsp.GspError):
        ctx.louvain(1e-2, 10, leiden=2)
    ctx.load_batch([gi.sbm(300, 5, 0.2, 0.01, k) for k in range(3)])
    with pytest.raises(gsp.GspError):
        ctx.run_batch(1e-2, 10, leiden=1)


def test_leiden_louvain_runs_unchanged(ctx):
    """A GSP-Louvain run after GSP-Leiden runs on the same context gives
    the oracle's GSP-Louvain result."""
    g = _graph("rmat15")
    ctx.load_graph(g)
    ctx.louvain(1e-2, 10, leiden=1)
    res = ctx.louvain(1e-2, 10)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    np.testing.assert_array_equal(res.membership, ref.membership)


def _run_both(ctx, g):
    res = ctx.louvain(1e-2, 10, leiden=1)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, leiden=True)
    _check_run(res, ref)


def test_leiden_self_loops_and_weights(ctx):
    """Self-loops (skipped by every scan, kept in the same-community
    subgraph) and fp32 weights."""
    base = gi.rmat_small(13, 21, weights=(1.0, 4.0))
    g = gi.with_self_loops(base, {3: 2.0, 77: 0.5, 4000: 3.0})
    ctx.load_graph(g)
    _run_both(ctx, g)


def test_leiden_fp64_weights(ctx):
    """fp64 weights through gsp_load_csr_f64 (on the exact-sum grid): the
    subgraph keeps them in fp64."""
    g = gi.rmat_small(12, 22, weights=(1.0, 3.0))
    w = g.weights.astype(np.float64) * 0.75
    ctx.load(g.offsets, g.cols, w, n=g.n)
    res = ctx.louvain(1e-2, 10, leiden=1)
    wg = w.copy()
    oracle.weight_grid(wg)   # the load's rounding, applied on the host
    ref = oracle.louvain(oracle.CSR(g.n, g.offsets, g.cols, wg), tolerance=1e-2, max_passes=10, sync=True,
                         rounds=8, leiden=True)
    _check_run(res, ref)


@pytest.mark.parametrize("rounds", [1, 4, 16])
def test_leiden_other_sub_rounds(ctx, rounds):
    g = _graph("rmat15")
    ctx.load_graph(g)
    res = ctx.louvain(1e-2, 10, leiden=1, sub_rounds=rounds)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=rounds, leiden=True)
    _check_run(res, ref)


def test_leiden_hub_paths_and_event_timing(ctx):
    """The hubs' global-table path, a small partition limit and per-kernel
    events change the launches, not the run."""
    g = _graph("rmat16w")
    ctx.load_graph(g)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, leiden=True)
    for kw in (dict(hub_global=1, use_graphs=0), dict(hub_max_parts=2, use_graphs=0), dict(timing=2),
               dict(timing=3)):
        res = ctx.louvain(1e-2, 10, leiden=1, **kw)
        _check_run(res, ref)
        if kw.get("timing"):
            assert res.stats["ms_refine"] > 0.0


def test_leiden_return_moves_option(ctx):
    """The return-move option applies to the local-moving phases (the
    refinement moves only vertices alone in their sub-community, so it has
    no swap cycles): equal to the oracle's run with the option."""
    g = _graph("dcsbm50k")
    ctx.load_graph(g)
    res = ctx.louvain(1e-2, 10, leiden=1, return_moves=1)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, leiden=True, return_moves=True)
    _check_run(res, ref)
