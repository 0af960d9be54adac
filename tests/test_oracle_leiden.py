"""Pins of the oracle's GSP-Leiden: the refinement phase (Section 3.5, the
greedy reading) and its pass loop.

The refinement is replayed here in exact arithmetic: every candidate gain is
the change of the all-pairs modularity (Eq. 1) computed with fractions, so
neither Eq. 2 nor the oracle's scan is reused.  The pass loop is replayed
from the separately pinned steps (synchronous local moving from a given
membership, BFS split, renumbering, refinement, aggregation), and the whole
method is bounded by brute force, by closed forms and by connectivity.
"""
from fractions import Fraction

import numpy as np
import pytest

import gsp_inputs as gi
import oracle
from exact import clique_edges, dense, max_modularity_bruteforce, modularity_allpairs


def _small(seed, n=11, p=0.4, loops=False, weighted=False):
    u = gi.uniform(seed, n * n * 2)
    edges, weights = [], {}
    k = 0
    for a in range(n):
        for b in range(a + 1, n):
            if u[k] < p:
                edges.append((a, b))
                weights[(a, b)] = float(1 + int(u[k + n * n] * 3)) if weighted else 1.0
            k += 1
    g = gi.from_edges(n, edges, weights=weights)
    if loops:
        g = gi.with_self_loops(g, {1: 2.0, 4: 3.0})
    return g


def _group(i, rounds):
    if rounds <= 1:
        return 0
    sh = rounds.bit_length() - 1
    return ((i * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)) >> (64 - sh)


def _refine_replay(g, bound, memb, tau, max_iter, rounds):
    """The refinement in exact arithmetic: sub-rounds of one snapshot each;
    a vertex alone in its sub-community takes the same-bound neighbour
    sub-community of largest modularity gain (lowest id on ties) if the gain
    is positive, unless both are singletons and the target's id is larger;
    movers mark their same-bound neighbours."""
    A = dense(g)
    n = g.n
    M2 = sum(sum(r) for r in A)
    memb = list(memb)
    unproc = [True] * n
    li, dqs = 0, []
    for it in range(max_iter):
        gs = Fraction(0)
        for p in range(rounds):
            q0 = modularity_allpairs(A, memb)
            size = np.bincount(memb, minlength=n)
            dec, gains = list(memb), [Fraction(0)] * n
            for i in range(n):
                if not (unproc[i] and _group(i, rounds) == p):
                    continue
                unproc[i] = False
                d = memb[i]
                if size[d] != 1:
                    continue
                cands = sorted({memb[int(j)] for j in g.cols[g.offsets[i]:g.offsets[i + 1]]
                                if j != i and bound[int(j)] == bound[i]} - {d})
                best, bg = None, None
                for c in cands:
                    m2 = list(memb)
                    m2[i] = c
                    gg = modularity_allpairs(A, m2) - q0
                    if best is None or gg > bg:
                        best, bg = c, gg
                if best is None or not bg > 0:
                    continue
                if size[best] == 1 and best > d:
                    continue
                dec[i] = best
                gains[i] = bg
            for i in range(n):
                if dec[i] != memb[i]:
                    gs += gains[i]
                    for j in g.cols[g.offsets[i]:g.offsets[i + 1]]:
                        if j != i and bound[int(j)] == bound[i]:
                            unproc[int(j)] = True
            memb = dec
        dqs.append(gs)
        li = it + 1
        if gs <= tau:
            break
    return memb, li, dqs


def _bounds(g, kind, seed):
    if kind == "louvain":
        return oracle.louvain(g, tolerance=0.0, sync=True).membership
    if kind == "one":
        return np.zeros(g.n, dtype=np.int32)
    return gi.random_membership(g.n, 3, seed)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("rounds", [1, 2, 8])
@pytest.mark.parametrize("kind", ["louvain", "one", "random"])
def test_refinement_matches_exact_replay(seed, rounds, kind):
    g = _small(500 + seed, loops=bool(seed % 2), weighted=bool(seed % 3 == 1))
    bound = _bounds(g, kind, seed)
    start = np.arange(g.n, dtype=np.int32)
    want, li, dqs = _refine_replay(g, bound, start, 0.0, 12, rounds)
    got, gli, gdq, _ = oracle.refine_sync(g, bound, tau=0.0, max_iter=12, rounds=rounds)
    assert list(got) == want
    assert gli == li
    np.testing.assert_allclose(gdq, [float(x) for x in dqs], atol=1e-13)


def test_refinement_from_merged_start_matches_replay():
    """Sub-communities of several vertices at the start never lose a member."""
    g = _small(611, n=12, p=0.45)
    bound = np.zeros(g.n, dtype=np.int32)
    start = np.arange(g.n, dtype=np.int32)
    start[[3, 7]] = 3          # a non-adjacent pair and a triple
    start[[5, 9, 11]] = 5
    want, li, _ = _refine_replay(g, bound, start, 0.0, 12, 8)
    got, gli, _, _ = oracle.refine_sync(g, bound, memb=start, tau=0.0, max_iter=12, rounds=8)
    assert list(got) == want and gli == li
    assert got[3] == got[7] and got[5] == got[9] == got[11]


def test_only_singletons_move():
    """Two cliques, one bound, 0 and 5 start together: neither leaves, although
    each would gain by joining its own clique."""
    g = gi.from_edges(10, clique_edges(5) + clique_edges(5, 5))
    start = np.arange(10, dtype=np.int32)
    start[5] = 0
    got, _, _, _ = oracle.refine_sync(g, np.zeros(10, dtype=np.int32), memb=start, tau=0.0, rounds=1)
    assert got[0] == got[5]


def test_singleton_bounds_move_nothing():
    g = gi.rmat_small(10, 3)
    ident = np.arange(g.n, dtype=np.int32)
    got, li, dq, mv = oracle.refine_sync(g, ident, tau=0.0, rounds=8)
    np.testing.assert_array_equal(got, ident)
    assert li == 1 and dq[0] == 0.0 and mv[0] == 0


@pytest.mark.parametrize("s", [3, 5, 8])
@pytest.mark.parametrize("rounds", [1, 8])
def test_cliques_in_one_bound_become_the_cliques(s, rounds):
    """Three disjoint s-cliques in one bound: each clique gathers into one
    sub-community and no two cliques merge."""
    g = gi.from_edges(3 * s, clique_edges(s) + clique_edges(s, s) + clique_edges(s, 2 * s))
    got, _, _, _ = oracle.refine_sync(g, np.zeros(3 * s, dtype=np.int32), tau=0.0, rounds=rounds)
    blocks = [set(got[k * s:(k + 1) * s].tolist()) for k in range(3)]
    assert all(len(b) == 1 for b in blocks)
    assert len(set.union(*blocks)) == 3


@pytest.mark.parametrize("seed", range(4))
def test_sub_communities_stay_inside_their_bound(seed):
    g = gi.rmat_small(12, 40 + seed)
    bound = gi.random_membership(g.n, 50, seed)
    got, _, _, _ = oracle.refine_sync(g, bound, tau=1e-6, rounds=8)
    for c in np.unique(got):
        assert len(np.unique(bound[got == c])) == 1
    # a start that crosses two bounds is rejected
    bad = np.arange(g.n, dtype=np.int32)
    i, j = np.flatnonzero(bound != bound[0])[0], 0
    bad[i] = bad[j]
    with pytest.raises(ValueError):
        oracle.refine_sync(g, bound, memb=bad)


def test_sequential_gains_are_the_modularity_change():
    """With every vertex in a sub-round of its own the moves are sequential,
    so each iteration's reported gain is the exact modularity change."""
    n = 9
    assert len({_group(i, 64) for i in range(n)}) == n
    g = _small(733, n=n, p=0.5, weighted=True)
    A = dense(g)
    bound = np.zeros(n, dtype=np.int32)
    start = list(range(n))
    got, li, dq, _ = oracle.refine_sync(g, bound, tau=0.0, max_iter=1, rounds=64)
    change = modularity_allpairs(A, list(got)) - modularity_allpairs(A, start)
    assert abs(dq[0] - float(change)) < 1e-13 and dq[0] > 0


# ---------------------------------------------------------------- pass loop

def _canonical(m):
    first = {}
    out = np.empty_like(m)
    for v, c in enumerate(m.tolist()):
        out[v] = first.setdefault(c, len(first))
    return out


def _leiden_replay(g, tol, max_passes, split_mode, rounds=8, max_iter=20, drop=10.0, agg_tol=0.8):
    """GSP-Leiden from the pinned steps; per pass (l_i, |P|, N', tau, refine
    iterations, |R|)."""
    top = np.arange(g.n, dtype=np.int32)
    level = oracle.CSR.of(g)
    start = None
    tau = tol
    rec = []
    for lp in range(max_passes):
        memb, li, _, _ = oracle.move_sync(level, memb=start, tau=tau, max_iter=max_iter, rounds=rounds)
        lab = oracle.split_bfs(level, memb) if split_mode == 0 else memb
        P, npc = oracle.renumber(lab)
        stop = li <= 1 or npc / level.n > agg_tol or lp == max_passes - 1
        ri, nr = 0, 0
        if not stop:
            R, ri, _, _ = oracle.refine_sync(level, P, tau=tau, max_iter=max_iter, rounds=rounds)
            if split_mode == 0:
                R = oracle.split_bfs(level, R)
            R, nr = oracle.renumber(R)
            stop = nr / level.n > agg_tol
        rec.append((li, npc, level.n, tau, ri, nr))
        if stop:
            top = P[top]
            break
        top = R[top]
        start = np.empty(nr, dtype=np.int32)
        start[R] = P
        level = oracle.aggregate(level, R, nr)
        tau = tau / drop
    if split_mode == 1:
        top = oracle.split_bfs(g, top)
    return _canonical(top), rec


def _ring_of_cliques(k, s):
    edges = []
    for c in range(k):
        edges += clique_edges(s, c * s)
        edges.append((c * s + s - 1, ((c + 1) % k) * s))
    return gi.from_edges(k * s, edges)


CASES = {
    "ring30x5": lambda: _ring_of_cliques(30, 5),
    "rmat12": lambda: gi.rmat_small(12, 12),
    "rmat13w": lambda: gi.rmat_small(13, 5, weights=(1.0, 4.0)),
    "rmat14": lambda: gi.rmat_small(14, 14),
    "dcsbm": lambda: gi.dcsbm_small(20_000, 3),
    "road": lambda: gi.road_small(120, 5),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("split_mode", [0, 1, 2])
def test_leiden_pass_loop_replays_the_steps(name, split_mode):
    g = CASES[name]()
    want, rec = _leiden_replay(g, 1e-2, 10, split_mode)
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, split_mode=split_mode, leiden=True)
    assert r.passes == len(rec)
    assert r.iterations == [x[0] for x in rec]
    assert r.communities == [x[1] for x in rec]
    assert r.vertices == [x[2] for x in rec]
    assert r.tau == [x[3] for x in rec]
    assert r.refine_iterations == [x[4] for x in rec]
    assert r.refined == [x[5] for x in rec]
    np.testing.assert_array_equal(r.membership, want)


@pytest.mark.parametrize("name", ["rmat12", "rmat14", "dcsbm"])
def test_one_pass_equals_louvain(name):
    """The first pass of GSP-Leiden is GSP-Louvain's: with one pass the
    results agree."""
    g = CASES[name]()
    a = oracle.louvain(g, tolerance=1e-2, max_passes=1, sync=True, leiden=True)
    b = oracle.louvain(g, tolerance=1e-2, max_passes=1, sync=True)
    np.testing.assert_array_equal(a.membership, b.membership)
    assert a.refined == [0]


@pytest.mark.parametrize("k,s", [(30, 5), (16, 6)])
def test_ring_of_cliques_is_found_and_equals_louvain(k, s):
    """On a ring of cliques the local-moving communities are the cliques and
    refinement keeps each whole, so the next level starts from singletons as
    Louvain's does: both runs give the cliques."""
    g = _ring_of_cliques(k, s)
    a = oracle.louvain(g, tolerance=1e-2, sync=True, leiden=True)
    b = oracle.louvain(g, tolerance=1e-2, sync=True)
    np.testing.assert_array_equal(a.membership, b.membership)
    assert a.communities[0] == k and (len(a.refined) == 1 or a.refined[0] == k)
    cliques = np.repeat(np.arange(k), s)
    q_cliques = oracle.modularity(g, cliques.astype(np.int32))
    assert a.modularity >= q_cliques - 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_bounded_by_bruteforce_optimum(seed):
    n = 8 + seed % 3
    u = gi.uniform(1000 + seed, n * n)
    edges = [(a, b) for k, (a, b) in enumerate((a, b) for a in range(n) for b in range(a + 1, n)) if u[k] < 0.35]
    g = gi.from_edges(n, edges)
    qmax, _ = max_modularity_bruteforce(dense(g))
    r = oracle.louvain(g, tolerance=0.0, sync=True, leiden=True)
    assert r.modularity <= qmax + 1e-12
    assert r.modularity >= 0.0 or g.nnz == 0
    assert oracle.disconnected(g, r.membership)[0] == 0


@pytest.mark.parametrize("seed", range(4))
def test_split_every_pass_leaves_no_disconnected_community(seed):
    g = gi.rmat_small(13, 70 + seed, weights=(1.0, 3.0) if seed % 2 else None)
    r = oracle.louvain(g, tolerance=1e-2, sync=True, leiden=True, split_mode=0)
    assert oracle.disconnected(g, r.membership)[0] == 0
    assert r.membership.max() + 1 == r.communities[-1]


def test_planted_partition_recovered():
    g = gi.planted_sbm_10k()
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, leiden=True)
    q_planted = oracle.modularity(g, g.block.astype(np.int32))
    assert r.modularity >= q_planted - 0.005
    assert oracle.disconnected(g, r.membership)[0] == 0


def test_rejects_async_and_gate():
    g = gi.rmat_small(8, 1)
    with pytest.raises(ValueError):
        oracle.louvain(g, sync=False, leiden=True)
    with pytest.raises(ValueError):
        oracle.louvain(g, sync=True, leiden=True, prune_params=np.zeros(4801, dtype=np.float32))
