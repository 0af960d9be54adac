"""The large case on the GPU: R-MAT scale 26 (2^26 vertices, 2^30 samples,
weights U[1,10], about 2.1e9 directed entries, int64 offsets).

Its weight total needs more than 2^53 units of the finest fp32 weight, so
the load takes the weights onto the grid of exact sums (multiples of 2^-S,
S = 18 here): every sum the method forms is then exact and the run does not
depend on the order of the GPU's atomics.  The oracle cannot run a whole
pass at this size in a test, so the checks are:
  * the grid: the library's S and its count of moved weights equal the
    oracle's rule applied on the host;
  * one synchronous step from a non-trivial membership: the decisions and
    gain numerators of 4,096 sampled vertices equal the oracle's decision
    from each vertex's row alone (K, Sigma and 2m are exact on both sides,
    so there is no tie to excuse);
  * a whole run, twice on one context: bit-identical memberships, statistics
    and modularity; modularity equal (1e-9 relative) to Eq. 1 recomputed
    with numpy on the host; no internally disconnected community; the split
    of the result is the result; and, where the asynchronous oracle's
    modularity is stored (tests/golden/async_q.json), Q >= Q_async - 0.005.
  * the shipped network at the R-MAT class's threshold: Q within 0.005 of
    the plain run's, no disconnected community;
  * the whole run equal to the oracle's synchronous run (stored by
    tests/golden/make_rmat26.py): membership digest, iterations and
    communities per pass, Q within 1e-9, in the degree order the run picks
    at this size and in the loaded order;
  * GSP-Leiden's whole run equal to the oracle's (stored by
    tests/golden/make_leiden.py): the same, plus the refinement's per-pass
    iterations and sub-community counts; no disconnected community.

Needs about 60 GB of host memory and 150 GB of device memory (a few
minutes, most of it generating the graph).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import gsp_inputs as gi
import oracle
import paper_2402_11454_amd as gsp

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "async_q.json")


@pytest.fixture(scope="module")
def big():
    gi.set_verbose(True)
    g = gi.rmat(26, 16, *gi.RMAT_ABC, 26, weights=(1.0, 10.0), name="rmat-26")
    gi.set_verbose(False)
    print(f"[large] R-MAT 26: n={g.n} nnz={g.nnz}", flush=True)
    # the oracle's grid on the host (fp64 copy of the weights)
    w = g.weights.astype(np.float64)
    S, moved = oracle.weight_grid(w)
    print(f"[large] weight grid: S={S}, {moved} weights moved", flush=True)
    c = gsp.Context(0)
    c.load(g.offsets, g.cols, g.weights, n=g.n)
    print("[large] loaded", flush=True)
    yield g, w, S, moved, c
    c.close()


def _k_and_m2(g, w):
    """K_i and 2m from the gridded weights: every partial sum is exact."""
    K = np.add.reduceat(w, g.offsets[:-1]) if g.nnz else np.zeros(g.n)
    K[np.diff(g.offsets) == 0] = 0.0          # reduceat copies the next entry into empty rows
    return K, float(K.sum())


def test_weight_grid_matches_oracle(big):
    g, w, S, moved, ctx = big
    assert ctx.weight_grid() == (S, moved)
    assert S == 18 and moved > 0


def test_sampled_step_decisions(big):
    g, w, S, moved, ctx = big
    assert g.nnz > 2 ** 30 and g.offsets.dtype == np.int64
    memb = (np.arange(g.n, dtype=np.int64) // 4).astype(np.int32)
    dec, gain, nmoved = ctx.step_move(memb)
    K, M2 = _k_and_m2(g, w)
    sigma = np.bincount(memb, weights=K, minlength=g.n)
    csize = np.bincount(memb, minlength=g.n).astype(np.int32)
    picks = np.unique((gi.uniform(261, 4096) * g.n).astype(np.int64))
    moves = 0
    for i in picks:
        s, e = g.offsets[i], g.offsets[i + 1]
        d, gn, _ = oracle.decide_row(i, g.cols[s:e], w[s:e], memb, sigma, csize, K[i], M2)
        assert dec[i] == d, (int(i), int(dec[i]), d)
        assert gain[i] == gn, (int(i), float(gain[i]), gn)
        moves += d != memb[i]
    assert moves > 100 and nmoved > 0


def test_whole_run_properties_and_repeat(big):
    g, w, S, moved, ctx = big
    res = ctx.louvain(tolerance=1e-2, max_passes=10)
    m = res.membership
    print(f"[large] passes={res.stats['passes']} iterations={res.stats['iterations']} Q={res.modularity:.6f}",
          flush=True)
    again = ctx.louvain(tolerance=1e-2, max_passes=10)
    assert np.array_equal(again.membership, m)
    assert again.modularity == res.modularity
    for k in ("passes", "iterations", "communities", "vertices", "moves", "scanned_entries"):
        assert again.stats[k] == res.stats[k], k
    assert m.min() >= 0 and m.max() < g.n
    assert ctx.count_disconnected(m) == 0
    lab = ctx.step_split(m)
    # the split of the result leaves it whole: every vertex's split label is
    # the smallest vertex of its community (communities are numbered by
    # ascending smallest vertex, so the first occurrence of c is that vertex)
    cs, first = np.unique(m, return_index=True)
    assert np.array_equal(cs, np.arange(cs.shape[0]))
    assert np.array_equal(lab, first[m].astype(np.int32))
    # Eq. 1 on the host: Q = sum_c [sigma_c / 2m - (Sigma_c / 2m)^2], by rows in chunks
    K, M2 = _k_and_m2(g, w)
    inside = 0.0
    step = 1 << 22
    for r0 in range(0, g.n, step):
        r1 = min(g.n, r0 + step)
        s, e = g.offsets[r0], g.offsets[r1]
        rows = np.repeat(np.arange(r0, r1, dtype=np.int64), np.diff(g.offsets[r0:r1 + 1]))
        same = m[rows] == m[g.cols[s:e]]
        inside += float(w[s:e][same].sum())
    Sig = np.bincount(m, weights=K, minlength=g.n)
    q = inside / M2 - float(np.sum((Sig / M2) ** 2))
    assert abs(res.modularity - q) <= 1e-9 * max(1.0, abs(q))
    assert res.modularity > 0.05
    ref = json.load(open(GOLDEN)).get("rmat26") if os.path.exists(GOLDEN) else None
    if ref is not None:
        assert ref["nnz"] == g.nnz
        assert res.modularity >= ref["modularity"] - 0.005, (res.modularity, ref["modularity"])


def test_shipped_network_quality(big):
    """The shipped network at the R-MAT class's threshold (chosen on the
    held-out R-MAT 26 graph of seed 27): modularity within 0.005 of the plain
    run's, no internally-disconnected community, pruning happened."""
    from paper_2402_11454_amd.train_pruner import DEFAULT_OUT, THETA_BY_CLASS, load_params
    g, w, S, moved, ctx = big
    plain = ctx.louvain(tolerance=1e-2, max_passes=10)
    ctx.pruner_set(load_params(DEFAULT_OUT))
    res = ctx.louvain(tolerance=1e-2, max_passes=10, prune_mode=gsp.PRUNE_LEARNED,
                      prune_threshold=THETA_BY_CLASS["rmat"])
    print(f"[large] shipped gate: Q={res.modularity:.6f} plain {plain.modularity:.6f} "
          f"iterations={res.stats['iterations']} pruned={res.stats['pruned']}", flush=True)
    assert res.stats["pruned"] > 0
    assert abs(res.modularity - plain.modularity) <= 0.005
    assert ctx.count_disconnected(res.membership) == 0


@pytest.mark.parametrize("order", [gsp.ORDER_AUTO, gsp.ORDER_LOADED])
def test_whole_run_equals_oracle(big, order):
    g, w, S, moved, ctx = big
    with open(os.path.join(os.path.dirname(GOLDEN), "rmat26_oracle.json")) as f:
        ref = json.load(f)
    assert ref["nnz"] == g.nnz and ref["n"] == g.n
    res = ctx.louvain(tolerance=1e-2, max_passes=10, vertex_order=order)
    sha = hashlib.sha1(np.ascontiguousarray(res.membership, dtype=np.int32).tobytes()).hexdigest()
    assert res.stats["iterations"] == ref["iterations"]
    assert res.stats["communities"] == ref["communities"]
    assert sha == ref["membership_sha1"]
    assert abs(res.modularity - ref["modularity"]) <= 1e-9


def test_leiden_equals_oracle(big):
    g, w, S, moved, ctx = big
    path = os.path.join(os.path.dirname(GOLDEN), "leiden_oracle.json")
    with open(path) as f:
        ref = json.load(f)["rmat26"]
    assert ref["nnz"] == g.nnz and ref["n"] == g.n
    res = ctx.louvain(tolerance=1e-2, max_passes=10, leiden=1)
    sha = hashlib.sha1(np.ascontiguousarray(res.membership, dtype=np.int32).tobytes()).hexdigest()
    assert res.stats["iterations"] == ref["iterations"]
    assert res.stats["communities"] == ref["communities"]
    assert res.stats["refine_iterations"] == ref["refine_iterations"]
    assert res.stats["refined"] == ref["refined"]
    assert sha == ref["membership_sha1"]
    assert abs(res.modularity - ref["modularity"]) <= 1e-9
    assert ctx.count_disconnected(res.membership) == 0
