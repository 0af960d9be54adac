"""Pins of the oracle's local-moving phase (Algorithm "louvainMove", Eq. 2).

Decisions are replayed here with brute force: the gain of every candidate
move is the exact change of the all-pairs modularity (Eq. 1) computed with
fractions, so neither Eq. 2 nor the oracle's scan is reused.
"""
from fractions import Fraction

import numpy as np
import pytest

import gsp_inputs as gi
import oracle
from exact import clique_edges, dense, modularity_allpairs


def _small(seed, n=10, p=0.4, loops=False, weighted=False):
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


def _neighbour_comms(g, memb, i):
    s, e = g.offsets[i], g.offsets[i + 1]
    return sorted({int(memb[j]) for j in g.cols[s:e] if j != i})


def _gain(A, memb, i, c, q0):
    m2 = list(memb)
    m2[i] = c
    return modularity_allpairs(A, m2) - q0


def _async_replay(g, tau, max_iter):
    """Brute-force replay of the one-thread asynchronous phase."""
    A = dense(g)
    n = g.n
    memb = list(range(n))
    unproc = [True] * n
    li, dqs = 0, []
    for it in range(max_iter):
        dq = Fraction(0)
        for i in range(n):
            if not unproc[i]:
                continue
            unproc[i] = False
            q0 = modularity_allpairs(A, memb)
            best, bg = None, None
            for c in _neighbour_comms(g, memb, i):
                if c == memb[i]:
                    continue
                gg = _gain(A, memb, i, c, q0)
                if best is None or gg > bg:
                    best, bg = c, gg
            if best is None or not bg > 0:
                continue
            memb[i] = best
            dq += bg
            for j in g.cols[g.offsets[i]:g.offsets[i + 1]]:
                if j != i:
                    unproc[int(j)] = True
        dqs.append(dq)
        li = it + 1
        if dq <= tau:
            break
    return memb, li, dqs


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("loops", [False, True])
def test_async_matches_bruteforce_replay(seed, loops):
    g = _small(seed, loops=loops, weighted=bool(seed % 2))
    memb, li, dqs = _async_replay(g, 0.0, 20)
    got, gli, gdq = oracle.move_async(g, tau=0.0, max_iter=20)
    assert list(got) == memb
    assert gli == li
    np.testing.assert_allclose(gdq, [float(x) for x in dqs], atol=1e-13)


def test_async_q_rises_by_reported_gain():
    g = gi.planted_sbm_10k()
    q0 = oracle.modularity(g, np.arange(g.n, dtype=np.int32))
    memb, li, dq = oracle.move_async(g, tau=0.0, max_iter=3)
    assert oracle.modularity(g, memb) - q0 == pytest.approx(dq.sum(), abs=1e-10)


def _group(i, rounds):
    if rounds == 1:
        return 0
    sh = rounds.bit_length() - 1
    return ((i * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)) >> (64 - sh)


def _sync_decide(g, A, memb, active):
    """Brute-force synchronous decisions from one snapshot."""
    n = g.n
    q0 = modularity_allpairs(A, memb)
    size = np.bincount(memb, minlength=n)
    M2 = sum(sum(r) for r in A)
    dec, gains = list(memb), [Fraction(0)] * n
    for i in range(n):
        if not active[i]:
            continue
        best, bg = None, None
        for c in _neighbour_comms(g, memb, i):
            if c == memb[i]:
                continue
            gg = _gain(A, memb, i, c, q0)
            if best is None or gg > bg:
                best, bg = c, gg
        if best is None or not bg > 0:
            continue
        d = memb[i]
        if size[d] == 1 and size[best] == 1 and best > d:
            continue
        dec[i] = best
        gains[i] = bg * M2 * M2 / 2      # numerator G(c*) - G(stay)
    return dec, gains


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("loops", [False, True])
def test_sync_step_matches_bruteforce(seed, loops):
    g = _small(200 + seed, loops=loops, weighted=bool(seed % 2))
    A = dense(g)
    for t in range(3):
        memb = gi.random_membership(g.n, 2 + 2 * t, seed * 7 + t)
        if t == 0:
            memb = np.arange(g.n, dtype=np.int32)
        active = (gi.uniform(seed + 99 * t, g.n) < 0.7).astype(np.uint8)
        dec, gains = _sync_decide(g, A, list(memb), active)
        gdec, ggain, moved = oracle.move_sync_step(g, memb, active)
        assert list(gdec) == dec
        assert moved == sum(1 for i in range(g.n) if dec[i] != memb[i])
        np.testing.assert_array_equal(ggain, [float(x) for x in gains])


def _sync_replay(g, tau, max_iter, rounds, trail=None, returns=False):
    """The synchronous phase in exact arithmetic.  With `returns`, a move back
    into the community the vertex left at its move of the previous iteration
    does not add its gain to the iteration's total.  `trail` collects each
    iteration's membership and its actual modularity change."""
    A = dense(g)
    n = g.n
    M2 = sum(sum(r) for r in A)
    memb = list(range(n))
    unproc = [True] * n
    last = {}          # vertex -> (community it left, iteration of that move)
    li, dqs = 0, []
    for it in range(max_iter):
        gs = Fraction(0)
        q0 = modularity_allpairs(A, memb)
        for p in range(rounds):
            active = [unproc[i] and _group(i, rounds) == p for i in range(n)]
            for i in range(n):
                if active[i]:
                    unproc[i] = False
            dec, gains = _sync_decide(g, A, memb, active)
            for i in range(n):
                if dec[i] != memb[i]:
                    if not (returns and last.get(i) == (dec[i], it - 1)):
                        gs += gains[i]
                    last[i] = (memb[i], it)
                    for j in g.cols[g.offsets[i]:g.offsets[i + 1]]:
                        if j != i:
                            unproc[int(j)] = True
            memb = dec
        dq = 2 * gs / (M2 * M2)
        dqs.append(dq)
        if trail is not None:
            trail.append((list(memb), modularity_allpairs(A, memb) - q0))
        li = it + 1
        if dq <= tau:
            break
    return memb, li, dqs


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("rounds", [1, 2, 8])
@pytest.mark.parametrize("returns", [False, True])
def test_sync_phase_matches_replay(seed, rounds, returns):
    g = _small(300 + seed, n=11, loops=bool(seed % 2))
    memb, li, dqs = _sync_replay(g, 0.0, 12, rounds, returns=returns)
    got, gli, gdq, _ = oracle.move_sync(g, tau=0.0, max_iter=12, rounds=rounds, returns=returns)
    assert list(got) == memb
    assert gli == li
    np.testing.assert_allclose(gdq, [float(x) for x in dqs], atol=1e-13)


def test_swap_cycle_and_return_moves():
    """Six vertices, one group: from iteration 2 on the two communities
    trade their labels back and forth (every other membership repeats, the
    actual modularity does not change).  As written, the tolerance test sees
    a positive predicted total each time and the phase runs to max_iter;
    with the return-move option it stops at the first iteration whose moves
    all return (its total is 0).  Both as the exact replay does."""
    g = gi.from_edges(6, [(0, 1), (0, 3), (0, 4), (1, 2), (1, 3), (1, 4), (1, 5), (2, 3), (2, 4), (3, 4), (3, 5),
                          (4, 5)])
    m0, li0, dq0 = _sync_replay(g, 0.0, 12, 1)
    got, gli, gdq, gmv = oracle.move_sync(g, tau=0.0, max_iter=12, rounds=1)
    assert list(got) == m0 and gli == li0 == 12 and min(gdq) > 0
    np.testing.assert_allclose(gdq, [float(x) for x in dq0], atol=1e-13)
    trail = []
    memb, li, dqs = _sync_replay(g, 0.0, 12, 1, trail, returns=True)
    got, gli, gdq, gmv = oracle.move_sync(g, tau=0.0, max_iter=12, rounds=1, returns=True)
    assert list(got) == memb and gli == li == 4
    assert gdq[li - 1] == 0.0 and gmv[li - 1] > 0
    np.testing.assert_allclose(gdq, [float(x) for x in dqs], atol=1e-13)
    # the cycle: iteration 4 restores iteration 2's labels, and iterations 3
    # and 4 leave the modularity where it was
    assert trail[1][0] == trail[3][0] != trail[2][0] and trail[2][1] == 0 and trail[3][1] == 0
    # without the rule the replay would not stop: iterations 3 and 4 repeat
    # the positive predicted totals (checked on the replay's own decisions)
    A = dense(g)
    m2 = trail[2][0]
    dec, gains = _sync_decide(g, A, m2, [True] * g.n)
    assert dec == trail[3][0] and sum(gains) > 0


def test_singleton_rule_pair():
    # one edge 0-1, both singletons: 1 joins 0, 0 stays (the rule keeps the
    # larger-id singleton from swapping)
    g = gi.from_edges(2, [(0, 1)])
    dec, gain, moved = oracle.move_sync_step(g, np.arange(2, dtype=np.int32))
    assert list(dec) == [0, 0] and moved == 1


def test_isolated_vertices_never_move():
    g = gi.from_edges(6, [(0, 1), (1, 2), (0, 2)])  # 3, 4, 5 isolated
    m, li, dq, mv = oracle.move_sync(g, tau=0.0, max_iter=10)
    assert list(m[3:]) == [3, 4, 5]
    m2, _, _ = oracle.move_async(g, tau=0.0, max_iter=10)
    assert list(m2[3:]) == [3, 4, 5]


def test_clique_collapses_to_one_community():
    g = gi.from_edges(6, clique_edges(6))
    for m in (oracle.move_sync(g, tau=0.0)[0], oracle.move_async(g, tau=0.0)[0]):
        assert len(set(m.tolist())) == 1


def test_decide_row_equals_the_step():
    """The per-row decision (used for sampled checks on graphs too large for
    a whole step) equals the whole synchronous step vertex by vertex."""
    g = gi.rmat_small(11, 4, weights=(1.0, 10.0))
    m = gi.random_membership(g.n, 300, 3)
    dec, gain, _ = oracle.move_sync_step(g, m)
    K, M2 = oracle.vertex_weights(g)
    sigma = np.bincount(m, weights=K, minlength=g.n)
    csize = np.bincount(m, minlength=g.n).astype(np.int32)
    w = g.weights_f64()
    for i in range(0, g.n, 3):
        s, e = g.offsets[i], g.offsets[i + 1]
        d, gn, sc = oracle.decide_row(i, g.cols[s:e], w[s:e], m, sigma, csize, K[i], M2)
        assert d == dec[i] and gn == gain[i]
