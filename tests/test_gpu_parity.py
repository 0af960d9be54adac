"""GPU-vs-oracle parity through the C ABI (needs an MI355X).

Bars (stated per test): modularity within 1e-9 in fp64; split labels,
aggregated graphs (rows canonicalised by column), synchronous move decisions,
gain numerators, whole local-moving phases and whole runs bit-exact.  All
graphs here have integer weights or fp32 weights whose fp64 sums are exact,
so the GPU's atomics cannot change a membership, a table value or a score
(other weights are taken onto the grid of exact sums at load, as the
oracle takes them); the per-iteration gain totals are exact sums of
fixed-point shares and compared bit for bit too.
"""
import numpy as np
import pytest

import gsp_inputs as gi
import oracle
import paper_2402_11454_amd as gsp

pytestmark = pytest.mark.gpu


def _hip_device_count():
    try:
        import torch
        return torch.cuda.device_count()
    except Exception:
        return 0


@pytest.fixture(scope="module")
def ctx():
    if _hip_device_count() == 0:
        pytest.skip("no GPU")
    c = gsp.Context(0)
    yield c
    c.close()


def _aggregated(g, k, seed):
    """A super-vertex graph (fp64 weights, self-loops) from the oracle."""
    m, G = oracle.renumber(gi.random_membership(g.n, k, seed))
    h = oracle.aggregate(g, m, G)
    return h


GRAPHS = {
    "sbm10k": lambda: gi.planted_sbm_10k(),
    "rmat12": lambda: gi.rmat_small(12, 12),
    "rmat13w": lambda: gi.rmat_small(13, 5, weights=(1.0, 4.0)),
    "rmat15": lambda: gi.rmat_small(15, 3),
    "sbm_w10": lambda: gi.sbm(4000, 25, 0.08, 0.002, 9, weights=(1.0, 10.0)),
    "road60": lambda: gi.road_small(60, 3),
}

_cache = {}


def _graph(name):
    if name not in _cache:
        if name == "agg_rmat14":
            _cache[name] = _aggregated(gi.rmat_small(14, 2), 3000, 1)
        elif name == "rmat15w":   # fp32 weights with hubs of several chunks
            _cache[name] = gi.rmat_small(15, 3, weights=(1.0, 4.0))
        else:
            _cache[name] = GRAPHS[name]()
    return _cache[name]


ALL = list(GRAPHS) + ["agg_rmat14"]


def _integer_weights(g):
    w = g.w if isinstance(g, oracle.CSR) else g.weights
    return w is None or bool(np.all(np.asarray(w, dtype=np.float64) == np.round(w)))


def _load(ctx, g):
    if isinstance(g, oracle.CSR):
        ctx.load(g.off, g.col, g.w, n=g.n)
    else:
        ctx.load_graph(g)


def _memberships(n, seed):
    yield np.arange(n, dtype=np.int32)
    yield np.zeros(n, dtype=np.int32)
    for k in (2, 37, max(2, n // 50), max(2, n // 3)):
        yield gi.random_membership(n, k, seed + k)


@pytest.mark.parametrize("name", ALL)
def test_modularity(ctx, name):
    g = _graph(name)
    _load(ctx, g)
    for m in _memberships(g.n, 11):
        q_gpu = ctx.modularity(m)
        q_ref = oracle.modularity(g, m)
        assert abs(q_gpu - q_ref) <= 1e-9, (q_gpu, q_ref)


@pytest.mark.parametrize("name", ALL)
def test_split_bit_exact(ctx, name):
    g = _graph(name)
    _load(ctx, g)
    for m in _memberships(g.n, 21):
        lab = ctx.step_split(m)
        np.testing.assert_array_equal(lab, oracle.split_bfs(g, m))


@pytest.mark.parametrize("name", ALL)
def test_split_lp_bit_exact(ctx, name):
    """The split by label propagation (LPP with pointer jumping) gives the
    labels of the oracle's one-thread LPP (Algorithm splitDisconnectedLp)."""
    g = _graph(name)
    _load(ctx, g)
    for m in _memberships(g.n, 23):
        lab, rounds = ctx.step_split_lp(m)
        ref, sweeps = oracle.split_lp(g, m, pruned=True)
        np.testing.assert_array_equal(lab, ref)
        assert rounds >= 1


@pytest.mark.parametrize("name", ["rmat15", "road300", "rmat13w"])
def test_split_algorithms_give_the_same_runs(ctx, name):
    g = gi.road_small(300, 3) if name == "road300" else _graph(name)
    _load(ctx, g)
    a = ctx.louvain(tolerance=1e-2, max_passes=10)
    b = ctx.louvain(tolerance=1e-2, max_passes=10, split_algo=gsp.SPLIT_LPP)
    np.testing.assert_array_equal(a.membership, b.membership)
    assert a.stats["iterations"] == b.stats["iterations"] and b.stats["split_rounds"] > 0
    c = ctx.louvain(tolerance=1e-2, max_passes=10, split_algo=gsp.SPLIT_LPP, split_mode=gsp.SPLIT_LAST)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, split_mode=gsp.SPLIT_LAST)
    np.testing.assert_array_equal(c.membership, ref.membership)


@pytest.mark.parametrize("name", ALL)
def test_disconnected_count(ctx, name):
    g = _graph(name)
    _load(ctx, g)
    for m in _memberships(g.n, 31):
        assert ctx.count_disconnected(m) == oracle.disconnected(g, m)[0]


def _canonical_rows(n, off, col, w):
    rows = []
    for c in range(n):
        s, e = int(off[c]), int(off[c + 1])
        o = np.argsort(col[s:e], kind="stable")
        rows.append((col[s:e][o], w[s:e][o]))
    return rows


@pytest.mark.parametrize("name", ALL)
def test_aggregate_bit_exact(ctx, name):
    g = _graph(name)
    _load(ctx, g)
    for m in list(_memberships(g.n, 41))[1:]:
        mr, G = oracle.renumber(m)
        ref = oracle.aggregate(g, mr, G)
        n2, off, col, w = ctx.step_aggregate(m)
        assert n2 == G
        np.testing.assert_array_equal(off, ref.off)
        for (c1, w1), (c2, w2) in zip(_canonical_rows(n2, off, col, w), _canonical_rows(G, ref.off, ref.col, ref.w)):
            np.testing.assert_array_equal(c1, c2)
            np.testing.assert_array_equal(w1, w2)


@pytest.mark.parametrize("name", ALL)
def test_step_move_bit_exact(ctx, name):
    g = _graph(name)
    _load(ctx, g)
    for t, m in enumerate(_memberships(g.n, 51)):
        active = None if t % 2 == 0 else (gi.uniform(t, g.n) < 0.6).astype(np.uint8)
        dec, gain, moved = ctx.step_move(m, active)
        rdec, rgain, rmoved = oracle.move_sync_step(g, m, active)
        np.testing.assert_array_equal(dec, rdec)
        np.testing.assert_array_equal(gain, rgain)
        assert moved == rmoved


@pytest.mark.parametrize("name", ALL)
@pytest.mark.parametrize("rounds", [1, 8])
@pytest.mark.parametrize("returns", [0, 1])
def test_move_phase_bit_exact(ctx, name, rounds, returns):
    g = _graph(name)
    _load(ctx, g)
    for tol in (0.0, 1e-2):
        m, li, dq, mv = ctx.move_phase(None, tolerance=tol, max_iterations=20, sub_rounds=rounds,
                                       return_moves=returns)
        rm, rli, rdq, rmv = oracle.move_sync(g, None, tau=tol, max_iter=20, rounds=rounds, returns=bool(returns))
        np.testing.assert_array_equal(m, rm)
        assert li == rli
        np.testing.assert_array_equal(mv, rmv)
        # the gain totals are exact sums of fixed-point shares on any weights
        np.testing.assert_array_equal(dq, rdq)


def test_swap_cycle_return_moves(ctx):
    """One group of six vertices whose two communities trade labels back
    and forth from the second iteration on: as written the phase runs to
    max_iterations; with return_moves = 1 it stops at the first iteration
    made only of return moves (its gain total 0).  Both as the oracle's."""
    g = gi.from_edges(6, [(0, 1), (0, 3), (0, 4), (1, 2), (1, 3), (1, 4), (1, 5), (2, 3), (2, 4), (3, 4), (3, 5),
                          (4, 5)])
    _load(ctx, g)
    m, li, dq, mv = ctx.move_phase(None, tolerance=0.0, max_iterations=12, sub_rounds=1)
    rm, rli, rdq, rmv = oracle.move_sync(g, None, tau=0.0, max_iter=12, rounds=1)
    assert li == rli == 12
    np.testing.assert_array_equal(m, rm)
    np.testing.assert_array_equal(dq, rdq)
    m, li, dq, mv = ctx.move_phase(None, tolerance=0.0, max_iterations=12, sub_rounds=1, return_moves=1)
    rm, rli, rdq, rmv = oracle.move_sync(g, None, tau=0.0, max_iter=12, rounds=1, returns=True)
    assert li == rli == 4 and dq[3] == 0.0 and mv[3] > 0
    np.testing.assert_array_equal(m, rm)
    np.testing.assert_array_equal(dq, rdq)
    np.testing.assert_array_equal(mv, rmv)


@pytest.mark.parametrize("name", list(GRAPHS))
def test_run_bit_exact_and_quality(ctx, name):
    g = _graph(name)
    _load(ctx, g)
    res = ctx.louvain(tolerance=1e-2, max_passes=10)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    np.testing.assert_array_equal(res.membership, ref.membership)
    assert abs(res.modularity - ref.modularity) <= 1e-9
    assert res.stats["iterations"] == ref.iterations
    assert res.stats["communities"] == ref.communities
    assert ctx.count_disconnected(res.membership) == 0
    qa = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=False).modularity
    assert res.modularity >= qa - 0.005


def _random_graph(seed):
    """A planted-partition graph of random size and density with dyadic
    weights (exact sums in fp64) and a few self-loops."""
    u = gi.uniform(1000 + seed, 8)
    n = int(50 + u[0] * 4000)
    blocks = max(1, int(n / (20 + u[1] * 200)))
    base = gi.sbm(n, blocks, 0.05 + 0.3 * u[2], 0.0005 + 0.005 * u[3], 77 + seed)
    rows = np.repeat(np.arange(n), np.diff(base.offsets))
    keep = rows < base.cols
    ew = gi.uniform(2000 + seed, int(keep.sum()))
    edges = list(zip(rows[keep].tolist(), base.cols[keep].tolist()))
    weights = {e: 0.25 * (1 + int(x * 15)) for e, x in zip(edges, ew)} if seed % 2 else None
    g = gi.from_edges(n, edges, weights=weights)
    lv = gi.uniform(3000 + seed, 4)
    return gi.with_self_loops(g, {int(lv[0] * n): 0.5, int(lv[1] * n): 2.0})


@pytest.mark.parametrize("seed", range(12))
def test_random_graphs_match_oracle(ctx, seed):
    g = _random_graph(seed)
    _load(ctx, g)
    returns = seed % 3 == 2   # a third of them with the return-move option
    res = ctx.louvain(tolerance=1e-2, max_passes=10, return_moves=int(returns))
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, return_moves=returns)
    np.testing.assert_array_equal(res.membership, ref.membership)
    assert res.stats["iterations"] == ref.iterations
    assert res.stats["communities"] == ref.communities
    assert abs(res.modularity - ref.modularity) <= 1e-9
    assert ctx.count_disconnected(res.membership) == 0


@pytest.mark.parametrize("returns", [0, 1])
def test_road_network_runs(ctx, returns):
    """The low-degree, high-diameter class (road / k-mer graphs, average
    degree about 2.1): 594 K vertices whose communities are long chains and
    grids, many passes; whole runs equal to the oracle's, with and without
    the return-move option."""
    g = gi.road_small(300, 3)
    _load(ctx, g)
    res = ctx.louvain(tolerance=1e-2, max_passes=10, return_moves=returns)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, return_moves=bool(returns))
    np.testing.assert_array_equal(res.membership, ref.membership)
    assert res.stats["iterations"] == ref.iterations
    assert res.stats["communities"] == ref.communities
    assert abs(res.modularity - ref.modularity) <= 1e-9
    assert ctx.count_disconnected(res.membership) == 0
    assert res.stats["passes"] >= 6


def test_run_rmat20_full_size(ctx):
    """R-MAT scale 20: whole run bit-exact vs the oracle's synchronous run,
    0 disconnected, Q within 0.005 of the asynchronous oracle's (stored)."""
    import json
    import os
    g = gi.rmat20()
    _load(ctx, g)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    for rep in range(3):   # repeated runs on one context: no state carried over
        res = ctx.louvain(tolerance=1e-2, max_passes=10)
        np.testing.assert_array_equal(res.membership, ref.membership)
        assert abs(res.modularity - ref.modularity) <= 1e-9
    assert ctx.count_disconnected(res.membership) == 0
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "async_q.json")))["rmat20"]
    assert gold["nnz"] == g.nnz
    assert res.modularity >= gold["modularity"] - 0.005


@pytest.mark.parametrize("mode", [gsp.SPLIT_LAST, gsp.SPLIT_NONE])
def test_split_modes(ctx, mode):
    g = _graph("rmat15")
    _load(ctx, g)
    res = ctx.louvain(tolerance=1e-2, max_passes=10, split_mode=mode)
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, split_mode=mode)
    np.testing.assert_array_equal(res.membership, ref.membership)


@pytest.mark.parametrize("seed", range(3))
def test_weight_grid_equals_oracle(ctx, seed):
    """fp64 weights whose fp64 sums depend on their order: the load takes
    them onto the grid of exact sums with the oracle's S, and the whole run
    then equals the oracle's (which takes the same grid)."""
    g0 = gi.rmat_small(13, 40 + seed, weights=(1.0, 4.0))
    # symmetric fp64 weights: the generator's weight of the undirected edge
    # times 1 + (a hash of the edge) 2^-30, which needs all 53 bits
    rows = np.repeat(np.arange(g0.n, dtype=np.uint64), np.diff(g0.offsets))
    cols = g0.cols.astype(np.uint64)
    key = np.minimum(rows, cols) * np.uint64(g0.n) + np.maximum(rows, cols) + np.uint64(seed)
    frac = ((key * np.uint64(0x9E3779B97F4A7C15)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    w_sym = g0.weights.astype(np.float64) * (1.0 + frac * 2.0 ** -30)
    h = oracle.CSR(g0.n, g0.offsets, g0.cols, w_sym)
    wg = w_sym.copy()
    S, moved = oracle.weight_grid(wg)
    assert moved > 0
    ctx.load(h.off, h.col, h.w, n=h.n)
    assert ctx.weight_grid() == (S, moved)
    hg = oracle.CSR(g0.n, g0.offsets, g0.cols, wg)
    res = ctx.louvain(tolerance=1e-2, max_passes=10)
    ref = oracle.louvain(hg, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    np.testing.assert_array_equal(res.membership, ref.membership)
    assert res.stats["iterations"] == ref.iterations
    assert abs(res.modularity - ref.modularity) <= 1e-9
    m, li, dq, mv = ctx.move_phase(None, tolerance=1e-2)
    rm, rli, rdq, rmv = oracle.move_sync(hg, None, tau=1e-2)
    np.testing.assert_array_equal(m, rm)
    np.testing.assert_array_equal(dq, rdq)


def test_edge_cases(ctx):
    # no edges: singletons, Q = 0
    ctx.load(np.zeros(6, np.int64), np.zeros(0, np.int32))
    res = ctx.louvain()
    assert res.membership.tolist() == list(range(5)) and res.modularity == 0.0
    # isolated vertices and a self-loop-only vertex
    g = gi.with_self_loops(gi.from_edges(7, [(0, 1), (1, 2), (0, 2), (3, 4)]), {6: 2.0})
    _load(ctx, g)
    res = ctx.louvain(tolerance=0.0)
    ref = oracle.louvain(g, tolerance=0.0, sync=True, rounds=8)
    np.testing.assert_array_equal(res.membership, ref.membership)
    # zero passes
    g = _graph("sbm10k")
    _load(ctx, g)
    ctx.run(max_passes=0)
    assert ctx.membership().tolist() == list(range(g.n))
    # int32 offsets give the same graph
    ctx.load(g.offsets.astype(np.int32), g.cols)
    assert ctx.n == g.n and ctx.modularity(np.zeros(g.n, np.int32)) == 0.0


@pytest.mark.parametrize("order", [gsp.ORDER_LOADED, gsp.ORDER_DEGREE])
def test_zero_weight_entries(ctx, order):
    """Entries of weight 0 (weights need only be finite and >= 0): a fifth
    of the pairs weigh 0, and vertices whose entries all weigh 0 have
    K_i = 0; GSP-Louvain and GSP-Leiden equal the oracle.  With every weight
    0 (2m = 0) no move has a positive gain: singletons, Q = 0."""
    g = gi.rmat_small(12, 23, weights=(1.0, 4.0))
    rows = np.repeat(np.arange(g.n), np.diff(g.offsets))
    w = g.weights.copy()
    w[(rows + g.cols.astype(np.int64)) % 5 == 0] = 0.0        # the same for (i, j) and (j, i)
    z = gi.Graph(n=g.n, offsets=g.offsets, cols=g.cols, weights=w, name="rmat12-zero")
    K = np.add.reduceat(w.astype(np.float64), g.offsets[:-1])
    assert ((K == 0.0) & (np.diff(g.offsets) > 0)).sum() > 0
    ctx.load_graph(z)
    for leiden in (0, 1):
        res = ctx.louvain(1e-2, 10, leiden=leiden, vertex_order=order)
        ref = oracle.louvain(z, tolerance=1e-2, max_passes=10, sync=True, rounds=8, leiden=bool(leiden))
        np.testing.assert_array_equal(res.membership, ref.membership)
        assert abs(res.modularity - ref.modularity) <= 1e-9
        assert res.stats["iterations"] == ref.iterations
        assert ctx.count_disconnected(res.membership) == 0
    ctx.load_graph(gi.Graph(n=g.n, offsets=g.offsets, cols=g.cols, weights=np.zeros_like(w), name="zero"))
    res = ctx.louvain(1e-2, 10, vertex_order=order)
    assert res.membership.tolist() == list(range(g.n)) and res.modularity == 0.0


def _clique(n):
    iu = np.triu_indices(n, 1)
    return gi.from_edges(n, list(zip(iu[0].tolist(), iu[1].tolist())), name=f"clique{n}")


def _star(leaves):
    """A hub joined to every leaf, and every 7th leaf to the leaf 7 further."""
    edges = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 7) for i in range(1, leaves - 6, 7)]
    return gi.from_edges(leaves + 1, edges, name=f"star{leaves}")


@pytest.mark.parametrize("order", [gsp.ORDER_LOADED, gsp.ORDER_DEGREE])
@pytest.mark.parametrize("make", [lambda: _clique(2100), lambda: _star(60000)], ids=["clique2100", "star60000"])
def test_clique_and_star(ctx, make, order):
    """Degenerate shapes: a clique of 2100 vertices (every vertex a hub of
    2099 entries, one community at the end) and a star (one hub of 60,000
    entries among leaves of degree 1-3); GSP-Louvain and GSP-Leiden equal
    the oracle."""
    g = make()
    ctx.load_graph(g)
    for leiden in (0, 1):
        res = ctx.louvain(1e-2, 10, leiden=leiden, vertex_order=order)
        ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, leiden=bool(leiden))
        np.testing.assert_array_equal(res.membership, ref.membership)
        assert abs(res.modularity - ref.modularity) <= 1e-9
        assert res.stats["iterations"] == ref.iterations
        assert ctx.count_disconnected(res.membership) == 0


def test_error_paths(ctx):
    with pytest.raises(gsp.GspError):
        ctx.run(return_moves=2)                         # an option of 0 or 1
    with pytest.raises(gsp.GspError) as e:
        ctx.load(np.array([0, 2, 1], np.int64), np.array([1, 0], np.int32))
    assert e.value.status == gsp.GSP_EGRAPH
    with pytest.raises(gsp.GspError) as e:
        ctx.load(np.array([0, 1, 2], np.int64), np.array([1, 5], np.int32))
    assert e.value.status == gsp.GSP_EGRAPH
    with pytest.raises(gsp.GspError) as e:
        ctx.load(np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32), np.array([1.0, -1.0], np.float32))
    assert e.value.status == gsp.GSP_EGRAPH
    with pytest.raises(gsp.GspError) as e:
        ctx.run()
    assert e.value.status == gsp.GSP_ESTATE      # the failed load left no graph
    g = _graph("rmat12")
    _load(ctx, g)
    with pytest.raises(gsp.GspError) as e:
        ctx.modularity(np.full(g.n, g.n, np.int32))
    assert e.value.status == gsp.GSP_EINVAL
    with pytest.raises(gsp.GspError) as e:
        ctx.run(sub_rounds=3)
    assert e.value.status == gsp.GSP_EINVAL
    # an empty graph (no vertex) is refused, and the graph loaded before stays
    with pytest.raises(gsp.GspError) as e:
        ctx.load(np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert e.value.status == gsp.GSP_EINVAL
    ctx.run(max_passes=0)
    assert ctx.membership().tolist() == list(range(g.n))
    with pytest.raises(gsp.GspError) as e:
        ctx.run(mem_limit_bytes=1024)
    assert e.value.status == gsp.GSP_ENOMEM


def test_deterministic(ctx):
    g = _graph("rmat15")
    _load(ctx, g)
    a = ctx.louvain().membership
    b = ctx.louvain().membership
    np.testing.assert_array_equal(a, b)


def test_device_pointers(ctx):
    import torch
    g = _graph("rmat12")
    dev = torch.device("cuda:0")
    off = torch.from_numpy(g.offsets).to(dev)
    col = torch.from_numpy(g.cols).to(dev)
    ctx.load(off, col)
    m = torch.from_numpy(gi.random_membership(g.n, 40, 3)).to(dev)
    torch.cuda.synchronize()
    assert abs(ctx.modularity(m) - oracle.modularity(g, m.cpu().numpy())) <= 1e-9
    lab = ctx.step_split(m)
    np.testing.assert_array_equal(lab.cpu().numpy(), oracle.split_bfs(g, m.cpu().numpy()))
    ctx.run()
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    ctx.membership(out)
    np.testing.assert_array_equal(out.cpu().numpy(), ctx.membership())


@pytest.mark.parametrize("name", ["rmat15", "sbm_w10"])
def test_graph_replay_equals_direct_launches(ctx, name):
    """Plain sweeps replayed from a captured HIP graph give exactly what the
    same launches give one by one, over several runs in a row (each replay
    checked, with other work and synchronisations between them)."""
    g = _graph(name)
    _load(ctx, g)
    direct = ctx.louvain(tolerance=1e-2, max_passes=10, use_graphs=0)
    for rep in range(3):
        res = ctx.louvain(tolerance=1e-2, max_passes=10, use_graphs=1)
        assert np.array_equal(res.membership, direct.membership)
        assert res.stats["iterations"] == direct.stats["iterations"]
        assert abs(res.modularity - direct.modularity) <= 1e-12   # Q itself is summed with atomics
        ctx.modularity(res.membership)                      # other work between replays
    m, li, dq, mv = ctx.move_phase(None, tolerance=1e-2)
    ref = oracle.move_sync(g, tau=1e-2)
    assert np.array_equal(m, ref[0]) and li == ref[1]


def test_timed_runs_equal_untimed(ctx):
    """Per-kernel timing (the scans of a sub-round run one after another,
    launch by launch, or side by side with timing = 3) gives the result of the
    untimed runs (scans side by side on four streams, replayed graphs); a
    class mask times only that class."""
    g = _graph("rmat15")
    _load(ctx, g)
    fast = ctx.louvain(tolerance=1e-2, max_passes=10)
    timed = ctx.louvain(tolerance=1e-2, max_passes=10, timing=2)
    assert np.array_equal(timed.membership, fast.membership)
    k = timed.stats["kernels"]
    for name in gsp.KERNEL_CLASSES:
        assert (k[name]["ms"] > 0) == (k[name]["launches"] > 0), name
    small = gsp.KERNEL_CLASSES.index("move_small")
    res = ctx.louvain(tolerance=1e-2, max_passes=10, timing=2, timing_mask=1 << small)
    k = res.stats["kernels"]
    assert k["move_small"]["ms"] > 0 and k["move_wave"]["ms"] == 0
    assert np.array_equal(res.membership, fast.membership)
    # timing = 3: events on each kernel's own stream, scans side by side
    wave = gsp.KERNEL_CLASSES.index("move_wave")
    for mask in (0, 1 << wave):
        res = ctx.louvain(tolerance=1e-2, max_passes=10, timing=3, timing_mask=mask)
        k = res.stats["kernels"]
        assert k["move_wave"]["ms"] > 0 and (k["move_small"]["ms"] > 0) == (mask == 0)
        assert np.array_equal(res.membership, fast.membership)
    with pytest.raises(gsp.GspError):
        ctx.run(timing=4)


@pytest.mark.parametrize("name", ["rmat15", "rmat15w", "agg_rmat14", "sbm_w10"])
def test_global_hub_tables_equal_partitions(ctx, name):
    """Hubs scored through global hash tables only (hub_global = 1) and
    through LDS hash partitions (the default) give the same runs."""
    g = _graph(name)
    _load(ctx, g)
    # the runs share the context, so b and c would replay a's captured sweeps
    # if the hub options were not part of their key: the pairs read back by
    # the partition gather (class move_hub_gather) show which path ran
    a = ctx.louvain(tolerance=1e-2, max_passes=10)
    b = ctx.louvain(tolerance=1e-2, max_passes=10, hub_global=1)
    assert np.array_equal(a.membership, b.membership)
    assert a.stats["iterations"] == b.stats["iterations"]
    off = g.off if isinstance(g, oracle.CSR) else g.offsets
    hubs = int(np.diff(off).max()) > 2048
    if hubs:
        assert a.stats["kernels"]["move_hub_gather"]["items"] > 0
    assert b.stats["kernels"]["move_hub_gather"]["items"] == 0
    # every hub of more than one chunk through the partition kernels' own
    # fallback (the hub's decision workgroup takes it through its global table)
    c = ctx.louvain(tolerance=1e-2, max_passes=10, hub_max_parts=1)
    assert np.array_equal(a.membership, c.membership)
    assert a.stats["iterations"] == c.stats["iterations"]
    assert c.stats["kernels"]["move_hub_gather"]["items"] == 0
    a2 = ctx.louvain(tolerance=1e-2, max_passes=10)          # back to the partitions
    assert a2.stats["kernels"]["move_hub_gather"]["items"] == a.stats["kernels"]["move_hub_gather"]["items"]
    if name == "rmat15w":
        ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
        assert np.array_equal(a.membership, ref.membership)


def _part_of(c, P):
    """The library's partition of community c among P (a murmur-style
    finaliser, high bits scaled to P), used here only to build an input
    whose hub overflows one partition."""
    h = c & 0xFFFFFFFF
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & 0xFFFFFFFF
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & 0xFFFFFFFF
    h ^= h >> 16
    return (h * P) >> 32


def test_hub_partition_overflow_falls_back(ctx):
    """A hub whose neighbours (singleton communities) all fall in one hash
    partition overflows that partition's LDS table: the hub is scored by the
    global-table path instead, with the oracle's decisions."""
    n = 20000
    P = 3                                            # hub degree 4097..6144 -> 3 chunks
    nb = [j for j in range(1, n) if _part_of(j, P) == 0][:4200]
    assert len(nb) == 4200
    edges = [(0, j) for j in nb]
    # some structure around: a ring so the other vertices have neighbours too
    edges += [(j, j + 1) for j in range(1, n - 1)]
    g = gi.from_edges(n, edges)
    _load(ctx, g)
    memb = np.arange(n, dtype=np.int32)
    dec, gain, moved = ctx.step_move(memb)
    rdec, rgain, rmoved = oracle.move_sync_step(g, memb)
    assert np.array_equal(dec, rdec) and moved == rmoved
    m, li, dq, mv = ctx.move_phase(None, tolerance=0.0)
    ref = oracle.move_sync(g, tau=0.0)
    assert np.array_equal(m, ref[0]) and li == ref[1]


def _check_aggregate(ctx, g, m):
    mr, G = oracle.renumber(m)
    ref = oracle.aggregate(g, mr, G)
    n2, off, col, w = ctx.step_aggregate(m)
    assert n2 == G
    np.testing.assert_array_equal(off, ref.off)
    for (c1, w1), (c2, w2) in zip(_canonical_rows(n2, off, col, w), _canonical_rows(G, ref.off, ref.col, ref.w)):
        np.testing.assert_array_equal(c1, c2)
        np.testing.assert_array_equal(w1, w2)


def test_aggregate_giant_communities(ctx):
    """Giant communities with many distinct neighbour communities go through
    hash partitions: 70% of the vertices in one community and the rest
    singletons (about 26 partitions, more than 2048 chunks, so the gather
    takes its source chunks in several windows), and eight giant communities
    beside singletons; rows bit-exact against the oracle."""
    g = gi.rmat_small(17, 5)
    _load(ctx, g)
    n = g.n
    cut = (7 * n) // 10
    big = np.where(np.arange(n) < cut, 0, np.arange(n)).astype(np.int32)
    assert int(g.offsets[cut]) > 2048 * 1024          # > 2048 chunks of 1024 entries
    _check_aggregate(ctx, g, big)
    eight = np.where(np.arange(n) % 3 == 0, (np.arange(n) % 8), np.arange(n)).astype(np.int32)
    _check_aggregate(ctx, g, eight)


def test_aggregate_partition_spill(ctx):
    """A giant community whose neighbour communities all fall in one hash
    partition overflows that partition's LDS table: its pairs go through the
    community's global table instead, with the same row."""
    n = 20000
    P = 3                                            # total degree 4200, n2 = n -> 3 partitions
    nb = [j for j in range(1, n) if _part_of(j, P) == 0][:4200]
    edges = [(0, j) for j in nb] + [(j, j + 1) for j in range(1, n - 1)]
    g = gi.from_edges(n, edges)
    _load(ctx, g)
    _check_aggregate(ctx, g, np.arange(n, dtype=np.int32))
