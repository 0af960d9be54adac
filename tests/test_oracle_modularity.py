"""Pins of the oracle's modularity (Eq. 1) and delta-modularity (Eq. 2).

Every expected value is computed without the oracle: exact rational
arithmetic on the all-pairs form of Eq. 1, or closed forms of Q for graphs
whose structure fixes it.
"""
from fractions import Fraction

import numpy as np
import pytest

import gsp_inputs as gi
import oracle
from exact import clique_edges, dense, modularity_allpairs


def _two_cliques(s):
    return gi.from_edges(2 * s, clique_edges(s) + clique_edges(s, s) + [(s - 1, s)])


def _ring_of_cliques(k, s):
    edges = []
    for c in range(k):
        edges += clique_edges(s, c * s)
        edges.append((c * s + s - 1, ((c + 1) % k) * s))
    return gi.from_edges(k * s, edges)


@pytest.mark.parametrize("s", [3, 4, 7])
def test_two_cliques_closed_form(s):
    # each clique one community: Q = s(s-1)/(s(s-1)+1) - 1/2
    g = _two_cliques(s)
    memb = np.array([0] * s + [1] * s, dtype=np.int32)
    expect = s * (s - 1) / (s * (s - 1) + 1) - 0.5
    assert oracle.modularity(g, memb) == pytest.approx(expect, abs=1e-14)


@pytest.mark.parametrize("k,s", [(3, 3), (5, 4), (10, 5)])
def test_ring_of_cliques_closed_form(k, s):
    # one clique per community: Q = s(s-1)/(s(s-1)+2) - 1/k
    g = _ring_of_cliques(k, s)
    memb = np.repeat(np.arange(k), s).astype(np.int32)
    expect = s * (s - 1) / (s * (s - 1) + 2) - 1.0 / k
    assert oracle.modularity(g, memb) == pytest.approx(expect, abs=1e-14)


def test_one_community_is_zero():
    g = gi.planted_sbm_10k()
    assert oracle.modularity(g, np.zeros(g.n, np.int32)) == pytest.approx(0.0, abs=1e-14)


def test_singletons_closed_form():
    # no self-loops: Q = -sum_i K_i^2 / (2m)^2
    g = gi.rmat_small(10, 3)
    K = g.degrees().astype(np.float64)
    expect = -(K ** 2).sum() / K.sum() ** 2
    assert oracle.modularity(g, np.arange(g.n, dtype=np.int32)) == pytest.approx(expect, rel=1e-13)


def test_no_edges_is_zero():
    g = gi.Graph(n=5, offsets=np.zeros(6, np.int64), cols=np.zeros(0, np.int32))
    assert oracle.modularity(g, np.arange(5, dtype=np.int32)) == 0.0


def _random_small(seed, n=9, p=0.45, loops=True, weighted=True):
    u = gi.uniform(seed, n * n * 2)
    edges, weights = [], {}
    k = 0
    for a in range(n):
        for b in range(a + 1, n):
            if u[k] < p:
                edges.append((a, b))
                weights[(a, b)] = float(1 + int(u[k + n * n] * 4)) if weighted else 1.0
            k += 1
    g = gi.from_edges(n, edges, weights=weights)
    if loops:
        g = gi.with_self_loops(g, {0: 2.0, 3: 1.0})
    return g


@pytest.mark.parametrize("seed", range(6))
def test_matches_allpairs_exact(seed):
    g = _random_small(seed)
    A = dense(g)
    for t in range(4):
        memb = gi.random_membership(g.n, 1 + t * 2, seed * 10 + t)
        exact = modularity_allpairs(A, list(memb))
        assert oracle.modularity(g, memb) == pytest.approx(float(exact), abs=1e-15)


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("loops", [False, True])
def test_delta_modularity_equals_q_difference(seed, loops):
    # Eq. 2 must equal Q(after moving i to c) - Q(before), exactly
    g = _random_small(100 + seed, loops=loops)
    A = dense(g)
    memb = gi.random_membership(g.n, 3, seed)
    q0 = modularity_allpairs(A, list(memb))
    for i in range(g.n):
        for c in range(g.n):
            if c == memb[i]:
                continue
            m2 = memb.copy()
            m2[i] = c
            exact = modularity_allpairs(A, list(m2)) - q0
            got = oracle.delta_modularity(g, memb, i, c)
            assert got == pytest.approx(float(exact), abs=1e-14), (i, c)


def test_range_of_q():
    # modularity lies in [-1/2, 1] (Section 3.2)
    g = gi.rmat_small(10, 5)
    for t in range(5):
        memb = gi.random_membership(g.n, 2 + 10 * t, t)
        q = oracle.modularity(g, memb)
        assert -0.5 <= q <= 1.0


def test_vertex_weights_sum():
    g = gi.rmat_small(12, 7, weights=(1.0, 4.0))
    K, M2 = oracle.vertex_weights(g)
    w = g.weights.astype(np.float64)
    rows = np.repeat(np.arange(g.n), g.degrees())
    assert np.array_equal(K, np.bincount(rows, weights=w, minlength=g.n))
    assert M2 == pytest.approx(w.sum(), rel=1e-15)
