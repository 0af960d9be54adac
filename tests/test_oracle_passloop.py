"""Pins of the oracle's pass loop (Algorithm "louvain"), the weight grid and
the fixed-point gain totals.

The pass loop is replayed here from its separately pinned steps (the
synchronous local-moving phase, the BFS split, the renumbering and the
aggregation, each checked against brute force or a plain definition in the
other oracle tests): reset, local moving with the pass's tolerance, split,
renumber + dendrogram lookup, the two convergence tests, aggregation and
threshold scaling, in the order the paper's algorithm takes them.  The
oracle's whole run must give the replay's per-pass iteration counts,
community counts, level sizes, tolerances and final membership.
"""
from fractions import Fraction

import numpy as np
import pytest

import gsp_inputs as gi
import oracle
from exact import clique_edges


def _canonical(m):
    first = {}
    out = np.empty_like(m)
    for v, c in enumerate(m.tolist()):
        out[v] = first.setdefault(c, len(first))
    return out


def _replay(g, tol, max_passes, split_mode, rounds=8, max_iter=20, drop=10.0, agg_tol=0.8):
    """Algorithm "louvain" from the pinned steps; per pass (l_i, |Gamma|, N', tau)."""
    top = np.arange(g.n, dtype=np.int32)
    level = oracle.CSR.of(g)
    tau = tol
    rec = []
    for lp in range(max_passes):
        memb, li, _, _ = oracle.move_sync(level, tau=tau, max_iter=max_iter, rounds=rounds)
        lab = oracle.split_bfs(level, memb) if split_mode == 0 else memb
        cm, ncomm = oracle.renumber(lab)
        top = cm[top]
        rec.append((li, ncomm, level.n, tau))
        if li <= 1:
            break
        if ncomm / level.n > agg_tol:
            break
        if lp == max_passes - 1:
            break
        level = oracle.aggregate(level, cm, ncomm)
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
    "ring40x4": lambda: _ring_of_cliques(40, 4),
    "ring64x4": lambda: _ring_of_cliques(64, 4),
    "rmat12": lambda: gi.rmat_small(12, 12),
    "rmat13w": lambda: gi.rmat_small(13, 5, weights=(1.0, 4.0)),
    "rmat14": lambda: gi.rmat_small(14, 14),
    "dcsbm": lambda: gi.dcsbm_small(20_000, 3),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_pass_loop_replays_the_steps(name):
    g = CASES[name]()
    want, rec = _replay(g, 1e-2, 10, 0)
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    assert r.passes == len(rec)
    assert r.iterations == [x[0] for x in rec]
    assert r.communities == [x[1] for x in rec]
    assert r.vertices == [x[2] for x in rec]
    assert r.tau == [x[3] for x in rec]
    np.testing.assert_array_equal(r.membership, want)


def test_threshold_scaling_sequence():
    """tau of pass p is tolerance / 10^p: each pass divides it once."""
    g = CASES["rmat14"]()
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    assert r.passes >= 3
    expect = [1e-2]
    for _ in range(r.passes - 1):
        expect.append(expect[-1] / 10.0)
    assert r.tau == expect
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, tolerance_drop=4.0)
    assert r.tau[1] == 1e-2 / 4.0


def test_low_shrink_break():
    """A pass whose split leaves more than tau_agg * N' communities is the
    last one, although its phase ran more than one iteration."""
    g = CASES["ring64x4"]()
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    li, nc, nv = r.iterations[-1], r.communities[-1], r.vertices[-1]
    assert r.passes < 10 and li > 1 and nc / nv > 0.8
    # with a looser aggregation tolerance the same pass aggregates again
    r2 = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, aggregation_tolerance=0.999)
    assert r2.passes > r.passes
    _, rec = _replay(g, 1e-2, 10, 0, agg_tol=0.999)
    assert r2.iterations == [x[0] for x in rec] and r2.communities == [x[1] for x in rec]


def test_converged_pass_stops_the_loop():
    """l_i <= 1 ends the passes: a pass started from the previous pass's
    communities moves nothing in its first iteration."""
    g = CASES["ring40x4"]()
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
    assert r.iterations[-1] <= 1 or r.communities[-1] / r.vertices[-1] > 0.8
    _, rec = _replay(g, 1e-2, 10, 0)
    assert [x[0] for x in rec] == r.iterations


def _split_last_case():
    for seed in range(40):
        g = gi.rmat_small(11, 100 + seed, edge_factor=6)
        sp = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, split_mode=0)
        sl = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, split_mode=1)
        if not np.array_equal(sp.membership, sl.membership):
            return g, sp, sl
    raise AssertionError("no R-MAT 11 seed where the split modes differ")


def test_split_last_differs_from_split_pass_and_replays():
    g, sp, sl = _split_last_case()
    want_sp, _ = _replay(g, 1e-2, 10, 0)
    want_sl, _ = _replay(g, 1e-2, 10, 1)
    np.testing.assert_array_equal(sp.membership, want_sp)
    np.testing.assert_array_equal(sl.membership, want_sl)
    assert oracle.disconnected(g, sl.membership)[0] == 0
    assert oracle.disconnected(g, sp.membership)[0] == 0
    # without any split the same run leaves a disconnected community
    none = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, split_mode=2)
    assert oracle.disconnected(g, none.membership)[0] > 0


# ---------------------------------------------------------------- weight grid

def _exact_sum(w):
    return sum(Fraction(float(x)) for x in w)


def test_grid_leaves_workload_weights_alone():
    for g in (gi.rmat_small(12, 3, weights=(1.0, 4.0)), gi.rmat_small(12, 4, weights=(1.0, 10.0)),
              gi.dcsbm_small(20_000, 2)):
        w = g.weights.astype(np.float64)
        S, moved = oracle.weight_grid(w)
        assert moved == 0 and S >= 23
        np.testing.assert_array_equal(w, g.weights.astype(np.float64))
    w = np.ones(1000)
    S, moved = oracle.weight_grid(w)
    assert moved == 0 and S >= 0


@pytest.mark.parametrize("scale", [2.0 ** 30, 2.0 ** 40, 3.0e-9])
def test_grid_makes_every_sum_exact(scale):
    """fp64 weights, whose sums in fp64 depend on the order of the additions
    (their total is far above 2^53 units of their finest bit): after the
    grid every sum is exact, whatever the order."""
    u = gi.uniform(7, 50_000)
    w = scale * (1.0 + 9.0 * u)
    orig = w.copy()
    rng = np.random.default_rng(1)
    sums = set()
    for _ in range(4):
        acc = 0.0
        for x in w[rng.permutation(w.shape[0])]:
            acc += x
        sums.add(acc)
    assert len(sums) > 1                                         # order-dependent before
    S, moved = oracle.weight_grid(w)
    assert moved > 0
    step = Fraction(2) ** (-S)
    for a, b in zip(w[:2000], orig[:2000]):
        q = Fraction(float(a)) / step
        assert q.denominator == 1                                # on the grid
        assert abs(Fraction(float(a)) - Fraction(float(b))) <= step / 2   # the nearest point
    total = _exact_sum(w)
    assert total / step < 2 ** 52                                # every partial sum below 2^52 steps
    assert total / step >= 2 ** 49                               # and the grid is not needlessly coarse
    rng = np.random.default_rng(1)
    for _ in range(4):
        p = rng.permutation(w.shape[0])
        acc = 0.0
        for x in w[p]:
            acc += x
        assert Fraction(acc) == total
    # a subset sum too (a community's Sigma, a super-vertex weight)
    sub = w[::7]
    assert Fraction(float(np.sum(sub[::-1]))) == _exact_sum(sub)


def test_grid_ties_and_zero():
    # total 7 + 2^-49 (3 bits): steps of 2^-49; both off-grid weights lie half-way
    w = np.array([0.0, 1.0, 1.0 + 2.0 ** -50, 1.0 + 3 * 2.0 ** -50, 3.0])
    S, moved = oracle.weight_grid(w)
    assert S == 52 - 3 and moved == 2
    assert w.tolist() == [0.0, 1.0, 1.0, 1.0 + 2.0 ** -48, 3.0]     # ties to the even multiple
    w = np.zeros(5)
    assert oracle.weight_grid(w) == (0, 0)


# ---------------------------------------------------------------- gain totals

def test_gain_fixed_closed_forms():
    M2 = 12.0
    assert oracle.gain_fixed(M2 * M2 / 4.0, M2) == 2 ** 60       # dQ = 1/2
    assert oracle.gain_fixed(0.0, M2) == 0
    assert oracle.gain_fixed(1.0, 0.0) == 0
    # half a unit rounds to even
    M2 = 2.0 ** 30
    g_half = M2 * M2 * 2.0 ** -63                                # dQ = 2^-62 = half a unit
    assert oracle.gain_fixed(g_half, M2) == 0
    assert oracle.gain_fixed(3 * g_half, M2) == 2


def test_sync_phase_total_is_the_sum_of_fixed_point_gains():
    """One synchronous iteration (one sub-round): the reported total is the
    sum of the movers' fixed-point gains, exactly."""
    g = gi.rmat_small(10, 2, weights=(1.0, 4.0))
    K, M2 = oracle.vertex_weights(g)
    memb = np.arange(g.n, dtype=np.int32)
    dec, gain, moved = oracle.move_sync_step(g, memb)
    units = sum(oracle.gain_fixed(x, M2) for x in gain[dec != memb])
    _, li, dq, mv = oracle.move_sync(g, memb, tau=1.0, max_iter=1, rounds=1)
    assert li == 1 and mv[0] == moved
    assert dq[0] == np.ldexp(float(units), -61)
    assert abs(dq[0] - float(2 * Fraction(float(gain.sum())) / Fraction(M2 * M2))) <= 1e-15 * moved


# ---------------------------------------------------------------- the gated phase's last iteration

def _accept_all():
    p = np.zeros(oracle.MLP_PARAMS, np.float32)
    p[-1] = 10.0                      # no weights: the logit is the output bias
    return p


@pytest.mark.parametrize("max_iter", [1, 2, 3])
def test_gated_phase_ends_with_a_confirming_sweep(max_iter):
    """With a gate that keeps every vertex, the phase's last counted
    iteration is a confirming sweep (every vertex unprocessed), so it equals
    max_iter - 1 plain iterations followed by one more synchronous phase of
    one iteration from their result (which starts with every vertex
    unprocessed)."""
    g = gi.rmat_small(12, 9)
    got, gli, gdq, gmv, cnt = oracle.move_sync_gated(g, _accept_all(), pass_index=0, tau=0.0, max_iter=max_iter)
    m = np.arange(g.n, dtype=np.int32)
    li0 = 0
    if max_iter > 1:
        m, li0, _, _ = oracle.move_sync(g, m, tau=0.0, max_iter=max_iter - 1, rounds=8)
        assert li0 == max_iter - 1
    m2, li1, dq1, mv1 = oracle.move_sync(g, m, tau=0.0, max_iter=1, rounds=8)
    np.testing.assert_array_equal(got, m2)
    assert cnt["confirm_sweeps"] == 1
    assert gli == li0 + (1 if mv1[0] > 0 else 0)


# ---------------------------------------------------------------- gate confirmed once per run

def test_final_confirmation_replays_its_steps():
    """confirm_final: gated passes without confirming sweeps, then one plain
    local-moving phase over G from their result (tolerance of the last
    pass), then the split and the canonical numbering."""
    from test_oracle_prune import _rand_params
    g = gi.dcsbm_small(6000, 11)
    p = _rand_params(21)
    p[-65:-1] *= 16.0
    p[-1] = -8.0                                      # prunes a part of the vertices
    r = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, prune_params=p, confirm_final=True)
    assert r.counters["pruned"] > 0 and r.final_iterations >= 1
    # replay: the same passes (gated sweeps, no confirmation) ...
    top = np.arange(g.n, dtype=np.int32)
    level = oracle.CSR.of(g)
    tau = 1e-2
    for lp in range(r.passes):
        memb, li, _, _, _ = oracle.move_sync_gated(level, p, pass_index=lp, tau=tau, confirm=False)
        assert li == r.iterations[lp]
        cm, ncomm = oracle.renumber(oracle.split_bfs(level, memb))
        top = cm[top]
        if lp < r.passes - 1:
            level = oracle.aggregate(level, cm, ncomm)
            tau /= 10.0
    # ... then the plain phase over G and the split
    m, fi, _, _, _ = oracle.move_sync_gated(g, None, pass_index=r.passes, memb=top, tau=tau)
    assert fi == r.final_iterations
    m = oracle.split_bfs(g, m)
    np.testing.assert_array_equal(r.membership, _canonical(m))
    assert oracle.disconnected(g, r.membership)[0] == 0
