"""Pins of the oracle's split (Algorithms "splitDisconnectedLp" and
"splitDisconnectedBfs"), renumbering, aggregation (Algorithm
"louvainAggregate") and disconnected-community count (Algorithm
"disconnectedCommunities")."""
import numpy as np
import pytest

import gsp_inputs as gi
import oracle
from exact import components_union_find, dense, modularity_allpairs
from golden import load


def _graphs():
    yield "sbm", gi.planted_sbm_10k()
    yield "rmat12", gi.rmat_small(12, 12)
    yield "rmat12w", gi.rmat_small(12, 13, weights=(1.0, 4.0))


@pytest.mark.parametrize("name,g", list(_graphs()))
@pytest.mark.parametrize("k", [3, 40, 1000])
def test_split_is_components_with_min_label(name, g, k):
    memb = gi.random_membership(g.n, k, k + len(name))
    lab = oracle.split_bfs(g, memb)
    uf = components_union_find(g.n, g.offsets, g.cols, memb)
    np.testing.assert_array_equal(lab, uf)
    for pruned in (False, True):
        lp, sweeps = oracle.split_lp(g, memb, pruned=pruned)
        np.testing.assert_array_equal(lp, uf)
    # refinement of the input, every block connected, Q never decreases
    assert np.all(memb[lab] == memb)
    assert oracle.disconnected(g, lab)[0] == 0
    assert oracle.modularity(g, lab) >= oracle.modularity(g, memb) - 1e-15


def test_split_golden_bridge():
    fx = load("split_bridge.txt")
    g = gi.from_edges(fx["n"], fx["edges"])
    memb = fx["membership"].astype(np.int32)
    np.testing.assert_array_equal(oracle.split_bfs(g, memb), fx["expected_labels"])
    assert oracle.disconnected(g, memb)[0] == int(fx["expected_disconnected"][0])


def test_disconnected_count_matches_union_find():
    g = gi.rmat_small(12, 21)
    for k in (2, 50, 700):
        memb = gi.random_membership(g.n, k, k)
        uf = components_union_find(g.n, g.offsets, g.cols, memb)
        comps_per_comm = {}
        for v in range(g.n):
            comps_per_comm.setdefault(int(memb[v]), set()).add(int(uf[v]))
        expect = sum(1 for s in comps_per_comm.values() if len(s) > 1)
        cnt, flags = oracle.disconnected(g, memb)
        assert cnt == expect
        assert sorted(np.nonzero(flags)[0].tolist()) == sorted(c for c, s in comps_per_comm.items() if len(s) > 1)


def test_renumber_is_order_preserving_bijection():
    lab = np.array([5, 3, 3, 6, 5, 0, 6], dtype=np.int32)
    out, G = oracle.renumber(lab)
    assert G == 4
    np.testing.assert_array_equal(out, [2, 1, 1, 3, 2, 0, 3])


def _dense_aggregate(g, memb, ncomm):
    w = g.weights_f64()
    A = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), g.degrees())
    np.add.at(A, (rows, g.cols), w)
    P = np.zeros((g.n, ncomm))
    P[np.arange(g.n), memb] = 1.0
    return P.T @ A @ P


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("weighted", [False, True])
def test_aggregate_matches_dense_ptap(seed, weighted):
    g = gi.rmat_small(9, seed, weights=(1.0, 4.0) if weighted else None)
    k = [3, 17, 100, 400][seed]
    memb, G = oracle.renumber(gi.random_membership(g.n, k, seed))
    h = oracle.aggregate(g, memb, G)
    D = _dense_aggregate(g, memb, G)
    H = np.zeros((G, G))
    rows = np.repeat(np.arange(G), np.diff(h.off))
    np.add.at(H, (rows, h.col), h.w)
    np.testing.assert_array_equal(H, D)         # exact: small integers / fp32-exact sums
    # rows sorted, no duplicates, no gaps
    for c in range(G):
        r = h.col[h.off[c]:h.off[c + 1]]
        assert np.all(np.diff(r) > 0)
    assert h.nnz == int((D != 0).sum())


def test_aggregate_invariants():
    g = gi.rmat_small(12, 5, weights=(1.0, 4.0))
    memb, G = oracle.renumber(gi.random_membership(g.n, 300, 1))
    h = oracle.aggregate(g, memb, G)
    w = g.weights_f64()
    assert h.w.sum() == w.sum()                  # total weight 2m preserved
    # symmetry w''_cd = w''_dc
    D = {}
    for c in range(G):
        for e in range(h.off[c], h.off[c + 1]):
            D[(c, int(h.col[e]))] = h.w[e]
    for (c, d), x in D.items():
        assert D[(d, c)] == x
    # K''_c = Sigma_c, and Q(G'', singletons) = Q(G', C')
    K, _ = oracle.vertex_weights(g)
    K2, _ = oracle.vertex_weights(h)
    np.testing.assert_array_equal(K2, np.bincount(memb, weights=K, minlength=G))
    assert oracle.modularity(h, np.arange(G, dtype=np.int32)) == pytest.approx(oracle.modularity(g, memb), abs=1e-14)


def test_aggregate_self_loops_kept():
    # two triangles joined by one edge, one community each
    g = gi.from_edges(6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (2, 3)])
    h = oracle.aggregate(g, np.array([0, 0, 0, 1, 1, 1], np.int32), 2)
    assert h.off.tolist() == [0, 2, 4]
    assert h.col.tolist() == [0, 1, 0, 1]
    assert h.w.tolist() == [6.0, 1.0, 1.0, 6.0]
    # the self-loop entry of the super-vertex counts in Q like the original edges
    A = dense(h)
    assert oracle.modularity(h, np.array([0, 1], np.int32)) == pytest.approx(float(modularity_allpairs(A, [0, 1])))
