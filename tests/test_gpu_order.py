"""The input graph stored in degree order inside gsp_run (vertex_order =
GSP_ORDER_DEGREE): a storage layout only, so a run's results equal the
oracle's on the graph as given, bit for bit, and equal the run in the loaded
order (memberships, modularity, per-pass statistics, scan counters, traces).

The graphs cover many exact ties (unit weights: the tie-break and the
singleton rule compare the caller's ids), long rows (at least 256 entries,
copied and summed in entry chunks), isolated vertices, self-loops and fp32 /
fp64 weights; the options cover every split mode and split algorithm, the
return-move option, graph replay on and off, the learned gate with traces,
and other numbers of sub-rounds (the layout groups the shorter rows by
sub-round and is rebuilt for another number).
"""
import math

import numpy as np
import pytest

import gsp_inputs as gi
import oracle
import paper_2402_11454_amd as gsp

pytestmark = pytest.mark.gpu

DEG = dict(vertex_order=gsp.ORDER_DEGREE)
LOADED = dict(vertex_order=gsp.ORDER_LOADED)


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
    "sbm_w10": lambda: gi.sbm(4000, 25, 0.08, 0.002, 9, weights=(1.0, 10.0)),
    "road60": lambda: gi.road_small(60, 3),
}
_cache = {}


def _graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name]()
    return _cache[name]


def _same_run(a, b):
    np.testing.assert_array_equal(a.membership, b.membership)
    assert a.modularity == b.modularity
    for k in ("passes", "iterations", "vertices", "communities", "moves", "scanned_entries",
              "scanned_vertices", "pruned", "confirm_sweeps", "sweeps"):
        assert a.stats[k] == b.stats[k], k


@pytest.mark.parametrize("name", list(GRAPHS))
def test_degree_order_equals_oracle(ctx, name):
    g = _graph(name)
    ctx.load_graph(g)
    res = ctx.louvain(1e-2, 10, **DEG)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    np.testing.assert_array_equal(res.membership, ref.membership)
    assert abs(res.modularity - ref.modularity) <= 1e-9
    assert res.stats["iterations"] == ref.iterations
    assert res.stats["communities"] == ref.communities
    assert ctx.count_disconnected(res.membership) == 0
    _same_run(res, ctx.louvain(1e-2, 10, **LOADED))
    if name.startswith("rmat1"):   # hubs: rows cut into entry chunks
        assert int(np.diff(g.offsets).max()) >= 256


@pytest.mark.parametrize("mode,algo,returns,graphs", [
    (gsp.SPLIT_PASS, gsp.SPLIT_LPP, 0, 1),
    (gsp.SPLIT_LAST, gsp.SPLIT_UF, 0, 1),
    (gsp.SPLIT_NONE, gsp.SPLIT_UF, 1, 1),
    (gsp.SPLIT_PASS, gsp.SPLIT_UF, 1, 0),
    (gsp.SPLIT_LAST, gsp.SPLIT_LPP, 1, 0),
])
def test_degree_order_options(ctx, mode, algo, returns, graphs):
    g = _graph("rmat15")
    ctx.load_graph(g)
    kw = dict(split_mode=mode, split_algo=algo, return_moves=returns, use_graphs=graphs)
    res = ctx.louvain(1e-2, 10, **kw, **DEG)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, split_mode=mode,
                         return_moves=bool(returns))
    np.testing.assert_array_equal(res.membership, ref.membership)
    assert res.stats["iterations"] == ref.iterations
    assert abs(res.modularity - ref.modularity) <= 1e-9
    _same_run(res, ctx.louvain(1e-2, 10, **kw, **LOADED))


def _random_graph(seed):
    """Planted partition of random size with dyadic weights, self-loops and
    isolated vertices."""
    u = gi.uniform(5000 + seed, 8)
    n = int(100 + u[0] * 6000)
    blocks = max(1, int(n / (20 + u[1] * 200)))
    base = gi.sbm(n, blocks, 0.05 + 0.3 * u[2], 0.0005 + 0.005 * u[3], 177 + seed)
    rows = np.repeat(np.arange(n), np.diff(base.offsets))
    keep = (rows < base.cols) & (rows % 17 != 3)   # some vertices lose every edge
    ew = gi.uniform(6000 + seed, int(keep.sum()))
    edges = list(zip(rows[keep].tolist(), base.cols[keep].tolist()))
    weights = {e: 0.25 * (1 + int(x * 15)) for e, x in zip(edges, ew)} if seed % 2 else None
    g = gi.from_edges(n, edges, weights=weights)
    lv = gi.uniform(7000 + seed, 4)
    return gi.with_self_loops(g, {int(lv[0] * n): 0.5, int(lv[1] * n): 2.0})


@pytest.mark.parametrize("seed", range(6))
def test_degree_order_random_graphs(ctx, seed):
    g = _random_graph(seed)
    ctx.load_graph(g)
    res = ctx.louvain(1e-2, 10, **DEG)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    np.testing.assert_array_equal(res.membership, ref.membership)
    assert res.stats["iterations"] == ref.iterations
    assert abs(res.modularity - ref.modularity) <= 1e-9
    assert ctx.count_disconnected(res.membership) == 0


def _gate_params(seed):
    u = gi.uniform(seed, gsp.GATE_PARAMS)
    p = (u * 2.0 - 1.0).astype(np.float32)
    p[0:512] *= math.sqrt(6 / 8)
    p[512:576] *= 0.1
    p[576:4672] *= math.sqrt(6 / 64)
    p[4672:4736] *= 0.1
    p[4736:4800] *= math.sqrt(6 / 64) * 4.0
    p[4800] = 1.0
    return p


def _sorted_traces(ctx):
    x, y, v, meta, seen = ctx.traces()
    order = np.lexsort((v, meta))
    return x[order], y[order], v[order], meta[order], seen


def test_degree_order_learned_gate_and_traces(ctx):
    g = _graph("rmat15w")
    ctx.load_graph(g)
    ctx.pruner_set(_gate_params(31))
    kw = dict(prune_mode=gsp.PRUNE_LEARNED, prune_threshold=0.5)
    runs = []
    for order in (DEG, LOADED):
        ctx.capture_traces(1_000_000, rate=0.3, seed=5)
        res = ctx.louvain(1e-2, 10, **kw, **order)
        runs.append((res, _sorted_traces(ctx)))
        ctx.capture_traces(0)
    (a, ta), (b, tb) = runs
    _same_run(a, b)
    assert a.stats["pruned"] > 0
    assert ta[4] == tb[4] and ta[0].shape[0] > 1000
    for u, w in zip(ta[:4], tb[:4]):
        np.testing.assert_array_equal(u, w)


def test_degree_order_rmat20_full_size(ctx):
    """R-MAT scale 20 (unit weights, hubs of tens of thousands of entries):
    the run in degree order equals the run in the loaded order (which the
    parity tests hold to the oracle), twice."""
    g = gi.rmat20()
    ctx.load_graph(g)
    ref = ctx.louvain(1e-2, 10, **LOADED)
    for _ in range(2):
        _same_run(ctx.louvain(1e-2, 10, **DEG), ref)


def test_degree_order_errors_and_defaults(ctx):
    g = _graph("rmat12")
    ctx.load_graph(g)
    assert gsp.default_options().vertex_order == gsp.ORDER_AUTO
    with pytest.raises(gsp.GspError):
        ctx.run(1e-2, 10, vertex_order=3)
    # no pass: every vertex its own community in either order
    res = ctx.louvain(1e-2, 0, **DEG)
    np.testing.assert_array_equal(res.membership, np.arange(g.n, dtype=np.int32))
    # a reload drops the ordered copy; the next run builds it for the new graph
    h = _graph("sbm_w10")
    ctx.load_graph(h)
    ref = oracle.louvain(h, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    np.testing.assert_array_equal(ctx.louvain(1e-2, 10, **DEG).membership, ref.membership)


@pytest.mark.parametrize("name", ["rmat15w", "sbm10k"])
def test_degree_order_other_sub_rounds(ctx, name):
    """The layout groups the shorter rows by sub-round; a run with another
    number of sub-rounds rebuilds it, and every run still equals the run in
    the loaded order."""
    g = _graph(name)
    ctx.load_graph(g)
    for rounds in (8, 4, 1, 8, 16):
        ref = ctx.louvain(1e-2, 10, sub_rounds=rounds, **LOADED)
        _same_run(ctx.louvain(1e-2, 10, sub_rounds=rounds, **DEG), ref)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=4)
    np.testing.assert_array_equal(ctx.louvain(1e-2, 10, sub_rounds=4, **DEG).membership, ref.membership)
