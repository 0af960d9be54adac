"""Pins of the oracle on entries of weight 0 (weights need only be finite
and >= 0).

Eq. 1 has no term for an entry of weight 0, so the modularity of any
partition is that of the graph without those entries.  A vertex whose
entries all weigh 0 has K_i = 0, so every candidate's gain for it (Eq. 2)
is 0 and it never moves by its own decision.  With every weight 0 the graph
has 2m = 0: no move has a positive gain, the run keeps the singletons, and Q
is 0 by convention.  Decisions, whole phases and GSP-Leiden's refinement
are replayed by brute force on the all-pairs modularity in exact
arithmetic, and both pass loops from their separately pinned steps.
"""
import numpy as np
import pytest

import gsp_inputs as gi
import oracle
from exact import dense, modularity_allpairs
from test_oracle_move import _sync_decide, _sync_replay


def _zero_small(seed, n=10, p=0.5):
    """A random graph on n vertices whose pair weights are drawn from
    {0, 1, 2, 3}; every pair at vertex 0 weighs 0 (so K_0 = 0)."""
    u = gi.uniform(seed, n * n * 2)
    edges, weights = [], {}
    k = 0
    for a in range(n):
        for b in range(a + 1, n):
            if u[k] < p:
                edges.append((a, b))
                weights[(a, b)] = 0.0 if a == 0 else float(int(u[k + n * n] * 4))
            k += 1
    return gi.from_edges(n, edges, weights=weights), edges, weights


def _without_zeros(n, edges, weights):
    keep = [e for e in edges if weights[e] != 0.0]
    return gi.from_edges(n, keep, weights={e: weights[e] for e in keep})


@pytest.mark.parametrize("seed", range(6))
def test_modularity_ignores_zero_entries(seed):
    g, edges, weights = _zero_small(300 + seed)
    h = _without_zeros(g.n, edges, weights)
    assert g.nnz > h.nnz
    A = dense(g)
    for t in range(4):
        memb = gi.random_membership(g.n, 1 + 2 * t, seed * 11 + t)
        exact = modularity_allpairs(A, list(memb))
        assert oracle.modularity(g, memb) == pytest.approx(float(exact), abs=1e-15)
        assert oracle.modularity(g, memb) == oracle.modularity(h, memb)


@pytest.mark.parametrize("seed", range(8))
def test_sync_step_with_zero_entries_matches_bruteforce(seed):
    g, _, _ = _zero_small(400 + seed)
    A = dense(g)
    K, _ = oracle.vertex_weights(g)
    assert K[0] == 0.0
    for t in range(3):
        memb = np.arange(g.n, dtype=np.int32) if t == 0 else gi.random_membership(g.n, 2 + 2 * t, seed * 5 + t)
        active = np.ones(g.n, np.uint8)
        dec, gains = _sync_decide(g, A, list(memb), active)
        gdec, ggain, moved = oracle.move_sync_step(g, memb, active)
        assert list(gdec) == dec
        np.testing.assert_array_equal(ggain, [float(x) for x in gains])
        # a vertex of weight 0 keeps its community
        assert all(gdec[i] == memb[i] for i in range(g.n) if K[i] == 0.0)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("rounds", [1, 8])
def test_sync_phase_with_zero_entries_matches_replay(seed, rounds):
    g, _, _ = _zero_small(500 + seed)
    memb, li, dqs = _sync_replay(g, 0.0, 20, rounds)
    got, gli, gdq, _ = oracle.move_sync(g, tau=0.0, max_iter=20, rounds=rounds)
    assert list(got) == memb and gli == li
    np.testing.assert_allclose(gdq, [float(x) for x in dqs], atol=1e-13)


def test_every_weight_zero_keeps_singletons():
    g, edges, _ = _zero_small(600)
    z = gi.from_edges(g.n, edges, weights={e: 0.0 for e in edges})
    r = oracle.louvain(z, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    assert r.membership.tolist() == list(range(z.n))
    assert r.modularity == 0.0 and r.passes == 1
    assert oracle.modularity(z, np.zeros(z.n, np.int32)) == 0.0


def _zero_rmat12():
    """R-MAT 12 with a fifth of its pairs at weight 0 (117 vertices with
    edges but K_i = 0)."""
    g = gi.rmat_small(12, 23, weights=(1.0, 4.0))
    rows = np.repeat(np.arange(g.n), np.diff(g.offsets))
    w = g.weights.copy()
    w[(rows + g.cols.astype(np.int64)) % 5 == 0] = 0.0
    return gi.Graph(n=g.n, offsets=g.offsets, cols=g.cols, weights=w, name="rmat12-zero")


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("kind", ["louvain", "one", "random"])
def test_refinement_with_zero_entries_matches_replay(seed, kind):
    from test_oracle_leiden import _bounds, _refine_replay
    g, _, _ = _zero_small(700 + seed, n=11)
    bound = _bounds(g, kind, seed)
    start = np.arange(g.n, dtype=np.int32)
    want, li, dqs = _refine_replay(g, bound, start, 0.0, 12, 8)
    got, gli, gdq, _ = oracle.refine_sync(g, bound, tau=0.0, max_iter=12, rounds=8)
    assert list(got) == want and gli == li
    np.testing.assert_allclose(gdq, [float(x) for x in dqs], atol=1e-13)


def test_pass_loops_with_zero_entries_replay_the_steps():
    from test_oracle_leiden import _leiden_replay
    from test_oracle_passloop import _replay
    g = _zero_rmat12()
    want, rec = _replay(g, 1e-2, 10, 0)
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    assert (r.passes, r.iterations, r.communities, r.tau) == (len(rec), [x[0] for x in rec],
                                                              [x[1] for x in rec], [x[3] for x in rec])
    np.testing.assert_array_equal(r.membership, want)
    want, rec = _leiden_replay(g, 1e-2, 10, 0)
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, leiden=True)
    assert (r.passes, r.iterations, r.refined) == (len(rec), [x[0] for x in rec], [x[5] for x in rec])
    np.testing.assert_array_equal(r.membership, want)
