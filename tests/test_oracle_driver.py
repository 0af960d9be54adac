"""Pins of the oracle's whole method (Algorithm "louvain").

The multi-pass result of a heuristic has no closed form; it is bounded here
by brute-force maximum modularity on graphs of at most 10 vertices, by
closed forms where the optimum is known, and by the planted partition.
"""
import numpy as np
import pytest

import gsp_inputs as gi
import oracle
from exact import clique_edges, dense, max_modularity_bruteforce


def _small(seed, n):
    u = gi.uniform(1000 + seed, n * n)
    edges = [(a, b) for k, (a, b) in enumerate((a, b) for a in range(n) for b in range(a + 1, n)) if u[k] < 0.35]
    return gi.from_edges(n, edges)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("sync", [False, True])
def test_bounded_by_bruteforce_optimum(seed, sync):
    n = 8 + seed % 3
    g = _small(seed, n)
    qmax, _ = max_modularity_bruteforce(dense(g))
    r = oracle.louvain(g, tolerance=0.0, sync=sync)
    assert r.modularity <= qmax + 1e-12
    assert r.modularity >= 0.0 or g.nnz == 0
    assert oracle.disconnected(g, r.membership)[0] == 0


@pytest.mark.parametrize("s", [3, 5, 8])
@pytest.mark.parametrize("sync", [False, True])
def test_two_cliques_reach_optimum(s, sync):
    g = gi.from_edges(2 * s, clique_edges(s) + clique_edges(s, s) + [(s - 1, s)])
    r = oracle.louvain(g, tolerance=0.0, sync=sync)
    expect = s * (s - 1) / (s * (s - 1) + 1) - 0.5
    assert r.modularity == pytest.approx(expect, abs=1e-14)
    assert r.membership.tolist() == [0] * s + [1] * s   # canonical numbering


@pytest.mark.parametrize("sync", [False, True])
def test_planted_partition_recovered(sync):
    g = gi.planted_sbm_10k()
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=sync)
    q_planted = oracle.modularity(g, g.block.astype(np.int32))
    assert abs(q_planted - 0.79) < 0.01          # 0.80 - 100 * (1/100)^2, up to sampling
    assert r.modularity >= q_planted - 0.005
    assert oracle.disconnected(g, r.membership)[0] == 0


def test_sync_quality_close_to_async():
    g = gi.rmat_small(15, 15)
    qa = oracle.louvain(g, sync=False).modularity
    qs = oracle.louvain(g, sync=True).modularity
    assert qs >= qa - 0.005


def test_no_edges_gives_singletons():
    g = gi.Graph(n=4, offsets=np.zeros(5, np.int64), cols=np.zeros(0, np.int32))
    r = oracle.louvain(g)
    assert r.membership.tolist() == [0, 1, 2, 3] and r.modularity == 0.0


def test_zero_passes_gives_singletons():
    g = gi.planted_sbm_10k()
    r = oracle.louvain(g, max_passes=0)
    assert r.membership.tolist() == list(range(g.n))


@pytest.mark.parametrize("sync", [False, True])
def test_membership_canonical_and_connected(sync):
    g = gi.rmat_small(13, 8, weights=(1.0, 4.0))
    r = oracle.louvain(g, sync=sync)
    m = r.membership
    # numbered by ascending smallest vertex id
    first = {}
    for v, c in enumerate(m.tolist()):
        first.setdefault(c, v)
    assert sorted(first, key=first.get) == list(range(len(first)))
    assert oracle.disconnected(g, m)[0] == 0
    assert r.modularity == pytest.approx(oracle.modularity(g, m), abs=1e-15)


def test_split_modes():
    # split last and split pass both leave no disconnected community; no
    # split at all may leave some (Section 4.1)
    g = gi.rmat_small(14, 3)
    for mode in (0, 1):
        r = oracle.louvain(g, split_mode=mode)
        assert oracle.disconnected(g, r.membership)[0] == 0
    r2 = oracle.louvain(g, split_mode=2)
    assert r2.modularity > 0


def test_deterministic():
    g = gi.rmat_small(13, 9)
    a = oracle.louvain(g, sync=True)
    b = oracle.louvain(g, sync=True)
    assert np.array_equal(a.membership, b.membership) and a.modularity == b.modularity
