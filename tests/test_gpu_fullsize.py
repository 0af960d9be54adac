"""Full-size parity on the GPU: the 4M-vertex degree-corrected SBM (the
learned-pruning workload, held-out seed 1000) and the batch of 512 SBM graphs
(the batch workload), through the C ABI.

Bars:
  * 4M graph, whole runs: plain and learned-pruned (a seeded random network,
    see tests/golden/make_dcsbm4m.py) equal to the oracle's stored runs:
    membership digest, iterations and communities per pass, the pruning
    counters, Q within 1e-9; no disconnected community;
  * 4M graph, the shipped trained network at its threshold: Q within 0.005
    of the plain run's, no disconnected community;
  * batch: every 16th graph's membership bit-identical to the oracle's run of
    that graph alone, Q within 1e-9, passes equal; no graph with a
    disconnected community; with learned pruning (the trained network), every
    32nd graph equal to its single-graph GPU run;
  * GSP-Leiden, whole runs in the loaded order and in degree order: on the 4M
    graph equal to the oracle's stored run (tests/golden/make_leiden.py), on
    R-MAT 20 equal to the oracle's run made here: membership, per-pass
    local-moving and refinement statistics, Q within 1e-9; no disconnected
    community.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import gsp_inputs as gi
import oracle
import paper_2402_11454_amd as gsp
from golden import make_dcsbm4m as mk

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dcsbm4m_oracle.json")
LEIDEN = os.path.join(os.path.dirname(GOLDEN), "leiden_oracle.json")


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


@pytest.fixture(scope="module")
def g4m():
    return gi.dcsbm_4m(mk.SEED)


@pytest.fixture(scope="module")
def gold():
    with open(GOLDEN) as f:
        return json.load(f)


def _digest(m):
    return hashlib.sha1(np.ascontiguousarray(m, dtype=np.int32).tobytes()).hexdigest()


def test_dcsbm4m_plain_equals_oracle(ctx, g4m, gold):
    assert (g4m.n, g4m.nnz) == (gold["n"], gold["nnz"])
    ctx.load(g4m.offsets, g4m.cols, g4m.weights, n=g4m.n)
    res = ctx.louvain(tolerance=1e-2, max_passes=10)
    ref = gold["plain"]
    assert _digest(res.membership) == ref["membership_sha1"]
    assert res.stats["iterations"] == ref["iterations"]
    assert res.stats["communities"] == ref["communities"]
    assert abs(res.modularity - ref["modularity"]) <= 1e-9
    assert ctx.count_disconnected(res.membership) == 0
    # the asynchronous oracle's quality (stored): Q >= Q_async - 0.005
    asy = json.load(open(os.path.join(os.path.dirname(GOLDEN), "async_q.json")))["dcsbm4m_s1000"]
    assert asy["nnz"] == g4m.nnz and res.modularity >= asy["modularity"] - 0.005


def test_dcsbm4m_learned_equals_oracle(ctx, g4m, gold):
    ctx.load(g4m.offsets, g4m.cols, g4m.weights, n=g4m.n)
    ctx.pruner_set(mk.gate_params())
    res = ctx.louvain(tolerance=1e-2, max_passes=10, prune_mode=gsp.PRUNE_LEARNED, prune_threshold=gold["theta"])
    ref = gold["learned"]
    assert res.stats["iterations"] == ref["iterations"]
    for k in ("scanned_vertices", "scanned_entries", "pruned", "confirm_sweeps"):
        assert res.stats[k] == ref["counters"][k], k
    assert res.stats["communities"] == ref["communities"]
    assert _digest(res.membership) == ref["membership_sha1"]
    assert abs(res.modularity - ref["modularity"]) <= 1e-9
    assert ctx.count_disconnected(res.membership) == 0


def test_dcsbm4m_shipped_network_quality(ctx, g4m, gold):
    """The shipped trained network at its threshold on the measured 4M graph:
    modularity within 0.005 of the plain run's (stored oracle Q), no
    internally-disconnected community, and pruning really happened."""
    from paper_2402_11454_amd.train_pruner import DEFAULT_OUT, DEFAULT_THETA, load_params
    ctx.load(g4m.offsets, g4m.cols, g4m.weights, n=g4m.n)
    ctx.pruner_set(load_params(DEFAULT_OUT))
    res = ctx.louvain(tolerance=1e-2, max_passes=10, prune_mode=gsp.PRUNE_LEARNED, prune_threshold=DEFAULT_THETA)
    print(f"[fullsize] shipped gate theta={DEFAULT_THETA}: Q={res.modularity:.6f} plain {gold['plain']['modularity']:.6f} "
          f"iterations={res.stats['iterations']} pruned={res.stats['pruned']}", flush=True)
    assert res.stats["pruned"] > 0
    assert abs(res.modularity - gold["plain"]["modularity"]) <= 0.005
    assert ctx.count_disconnected(res.membership) == 0


@pytest.fixture(scope="module")
def batch():
    return gi.batch_sbm(512, master_seed=4, scale=1.0)


def test_batch512_plain_full_size(ctx, batch):
    ctx.load_batch(batch)
    ctx.run_batch(1e-2, 10)
    q = ctx.batch_modularity()
    passes = ctx.batch_passes()
    for k, g in enumerate(batch):
        m = ctx.batch_membership(k)
        if k % 16 == 0:
            ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8)
            assert np.array_equal(m, ref.membership), f"graph {k} (n={g.n})"
            assert abs(q[k] - ref.modularity) <= 1e-9
            assert passes[k] == ref.passes
        cnt, _ = oracle.disconnected(g, m)
        assert cnt == 0, k


def test_batch512_learned_equals_single_runs(ctx, batch):
    from paper_2402_11454_amd.train_pruner import DEFAULT_OUT, load_params
    ctx.pruner_set(load_params(DEFAULT_OUT))
    kw = dict(prune_mode=gsp.PRUNE_LEARNED, prune_threshold=0.5)
    ctx.load_batch(batch)
    ctx.run_batch(1e-2, 10, **kw)
    q = ctx.batch_modularity()
    got = {k: ctx.batch_membership(k) for k in range(0, len(batch), 32)}
    for k, m in got.items():
        g = batch[k]
        ctx.load(g.offsets, g.cols, g.weights, n=g.n)
        res = ctx.louvain(1e-2, 10, **kw)
        assert np.array_equal(m, res.membership), k
        assert abs(q[k] - res.modularity) <= 1e-12


def _leiden_matches(res, ref_stats, sha, q):
    assert res.stats["iterations"] == ref_stats["iterations"]
    assert res.stats["communities"] == ref_stats["communities"]
    assert res.stats["refine_iterations"] == ref_stats["refine_iterations"]
    assert res.stats["refined"] == ref_stats["refined"]
    assert hashlib.sha1(np.ascontiguousarray(res.membership, dtype=np.int32).tobytes()).hexdigest() == sha
    assert abs(res.modularity - q) <= 1e-9


@pytest.mark.parametrize("order", [gsp.ORDER_LOADED, gsp.ORDER_DEGREE])
def test_dcsbm4m_leiden_equals_oracle(ctx, g4m, order):
    with open(LEIDEN) as f:
        ref = json.load(f)["dcsbm4m"]
    assert ref["n"] == g4m.n and ref["nnz"] == g4m.nnz
    ctx.load_graph(g4m)
    print(f"[leiden] dcsbm4m order={order}", flush=True)
    res = ctx.louvain(1e-2, 10, leiden=1, vertex_order=order)
    _leiden_matches(res, ref, ref["membership_sha1"], ref["modularity"])
    assert ctx.count_disconnected(res.membership) == 0


@pytest.fixture(scope="module")
def rmat20_leiden():
    g = gi.rmat20()
    ref = oracle.louvain(g, tolerance=1e-2, max_passes=10, sync=True, rounds=8, leiden=True)
    sha = hashlib.sha1(np.ascontiguousarray(ref.membership, dtype=np.int32).tobytes()).hexdigest()
    stats = dict(iterations=ref.iterations, communities=ref.communities, refine_iterations=ref.refine_iterations,
                 refined=ref.refined)
    return g, stats, sha, ref.modularity


@pytest.mark.parametrize("order", [gsp.ORDER_LOADED, gsp.ORDER_DEGREE])
def test_rmat20_leiden_equals_oracle(ctx, rmat20_leiden, order):
    g, stats, sha, q = rmat20_leiden
    ctx.load_graph(g)
    print(f"[leiden] rmat20 order={order}", flush=True)
    res = ctx.louvain(1e-2, 10, leiden=1, vertex_order=order)
    _leiden_matches(res, stats, sha, q)
    assert ctx.count_disconnected(res.membership) == 0
