"""The seeded generators produce valid symmetric CSR graphs, deterministically."""
import numpy as np
import pytest

import gsp_inputs as gi


def _check_csr(g):
    assert g.offsets[0] == 0 and g.offsets[-1] == g.nnz
    assert np.all(np.diff(g.offsets) >= 0)
    assert np.all((g.cols >= 0) & (g.cols < g.n))
    rows = np.repeat(np.arange(g.n), g.degrees())
    assert not np.any(rows == g.cols)                      # no self-loops
    key = rows.astype(np.int64) * g.n + g.cols
    assert np.all(np.diff(key) > 0)                         # sorted, no duplicates
    rev = np.sort(g.cols.astype(np.int64) * g.n + rows)
    assert np.array_equal(rev, key)                         # symmetric
    if g.weights is not None:
        order = np.argsort(g.cols.astype(np.int64) * g.n + rows)
        assert np.array_equal(g.weights[order], g.weights)  # w_ij = w_ji


@pytest.mark.parametrize("make", [
    lambda: gi.planted_sbm_10k(),
    lambda: gi.rmat_small(12, 1),
    lambda: gi.rmat_small(12, 2, weights=(1.0, 10.0)),
    lambda: gi.sbm(3000, 7, 0.05, 0.001, 5, weights=(1.0, 4.0)),
    lambda: gi.dcsbm_small(5000, 3),
    lambda: gi.road_small(80, 5),
])
def test_valid_and_deterministic(make):
    a, b = make(), make()
    _check_csr(a)
    assert np.array_equal(a.offsets, b.offsets) and np.array_equal(a.cols, b.cols)
    if a.weights is not None:
        assert np.array_equal(a.weights, b.weights)
        assert a.weights.min() >= 1.0


def test_planted_sbm_shape():
    g = gi.planted_sbm_10k()
    assert g.n == 10_000
    assert 19.0 < g.nnz / g.n < 21.0                        # expected degree 20
    rows = np.repeat(np.arange(g.n), g.degrees())
    intra = (g.block[rows] == g.block[g.cols]).mean()
    assert 0.78 < intra < 0.82                              # 80% intra-block
    assert np.all(np.bincount(g.block) == 100)


def test_batch_params():
    ps = gi.batch_sbm_params(512)
    ns = np.array([p["n"] for p in ps])
    assert ns.min() >= 1000 and ns.max() <= 200_000


def test_dcsbm_shape():
    """Power-law degrees and community sizes, mixing mu: the planted
    communities hold about 1 - mu of the entries, community sizes respect
    the size law's bounds, the degree law's bounds hold, and every vertex
    sits in a community with room for its intra-community stubs."""
    mu = 0.3
    g = gi.dcsbm(30_000, 2.5, 5, 600, 1.5, 20, 3000, mu, 11)
    _check_csr(g)
    rows = np.repeat(np.arange(g.n), g.degrees())
    intra = (g.block[rows] == g.block[g.cols]).mean()
    assert abs(intra - (1 - mu)) < 0.03
    sizes = np.bincount(g.block)
    sizes = sizes[sizes > 0]
    assert sizes.min() >= 20 and sizes.sum() == g.n
    assert sizes.max() <= 3000 + 20                      # a merged remainder may exceed smax by < smin
    d = g.degrees()
    assert d.max() <= 600                                # duplicates only lower degrees
    assert 8.0 < d.mean() < 16.0                         # law mean ~ 12.6 before dedup
    # heavy tail: the top 1% of vertices hold far more than 1% of the entries
    top = np.sort(d)[::-1][: g.n // 100].sum() / g.nnz
    assert top > 0.05
    full = np.bincount(g.block)                          # room for the intra stubs: (1-mu) k <= s - 1
    assert np.all(full[g.block] - 1 >= (1 - mu) * d)


def test_dcsbm_seeds_differ():
    a, b = gi.dcsbm_small(4000, 0), gi.dcsbm_small(4000, 1)
    assert a.nnz != b.nnz or not np.array_equal(a.cols, b.cols)


def test_batch_sbm_shape():
    """The batch law at a tenth of its size: n >= 100, degree and mixing of
    each graph close to its parameters, deterministic."""
    ps = gi.batch_sbm_params(40, master_seed=4)
    gs = gi.batch_sbm(40, master_seed=4, scale=0.1)
    for p, g in zip(ps, gs):
        _check_csr(g)
        assert g.n == max(100, int(round(p["n"] * 0.1)))
        if g.n >= 2000:
            assert abs(g.nnz / g.n - p["degree"]) < 0.15 * p["degree"] + 1
            rows = np.repeat(np.arange(g.n), g.degrees())
            inter = (g.block[rows] != g.block[g.cols]).mean()
            assert abs(inter - p["mixing"]) < 0.06
    gs2 = gi.batch_sbm(40, master_seed=4, scale=0.1)
    assert all(np.array_equal(a.cols, b.cols) for a, b in zip(gs, gs2))


def test_road_shape():
    """The road-like law: degrees at most 4 (lattice junctions), mostly 2
    (chain vertices), average degree near the paper's road and k-mer graphs
    (about 2.1); the lattice edges kept and the chain lengths follow the
    parameters."""
    g = gi.road(200, 0.7, 8, 11, permute=False)
    d = g.degrees()
    assert d.max() <= 4 and 2.05 < g.nnz / g.n < 2.2
    assert np.mean(d == 2) > 0.85
    kept = 2 * 200 * 199 * 0.7
    inner = g.n - 200 * 200
    assert abs(inner / kept - 4.0) < 0.1                   # mean chain length (0..8 uniform)
    assert abs((g.nnz // 2 - inner) / kept - 1.0) < 0.02   # edges = kept lattice edges + inner vertices
