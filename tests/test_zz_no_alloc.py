"""gsp_count_disconnected_noalloc (the entry point for callers that cannot
allocate) against gsp_count_disconnected on a context, through the C ABI:
two calls in a row on one GPU, the second with a smaller input, so the
shared scratch holds the first call's contents when the second starts."""
import numpy as np
import pytest

import gsp_inputs as gi
import paper_2402_11454_amd as gsp

pytestmark = pytest.mark.gpu


def _count_ctx(g, memb):
    with gsp.Context(0) as c:
        c.load_graph(g)
        return c.count_disconnected(memb)


def _count_noalloc(g, memb):
    import torch
    dev = torch.device("cuda:0")
    off = torch.from_numpy(g.offsets.astype(np.int64)).to(dev)
    col = torch.from_numpy(g.cols.astype(np.int32)).to(dev)
    m = torch.from_numpy(np.ascontiguousarray(memb, dtype=np.int32)).to(dev)
    out = torch.full((1,), -7, dtype=torch.int64, device=dev)
    gsp.count_disconnected_noalloc(off, col, m, out)
    torch.cuda.synchronize()
    return int(out.item())


def test_noalloc_count_equals_context_count_twice():
    import torch
    if torch.cuda.device_count() == 0:
        pytest.skip("no GPU")
    big = gi.rmat_small(16, 3)                        # 65,536 vertices
    small = gi.rmat_small(12, 4)                      # 4,096 vertices
    cases = []
    for g, k, seed in ((big, 3000, 1), (small, 200, 2)):
        memb = gi.random_membership(g.n, k, seed)      # random communities: many disconnected
        cases.append((g, memb))
    want = [_count_ctx(g, m) for g, m in cases]
    assert want[0] > 0 and want[1] > 0
    got = [_count_noalloc(g, m) for g, m in cases]
    assert got == want
    # a connected membership (every vertex alone): none disconnected
    assert _count_noalloc(small, np.arange(small.n, dtype=np.int32)) == 0


def test_noalloc_limits_and_bad_labels():
    import torch
    if torch.cuda.device_count() == 0:
        pytest.skip("no GPU")
    assert gsp.lib().gsp_noalloc_max_vertices() == (64 * 2 ** 20 - 256) // 8
    g = gi.rmat_small(10, 5)
    memb = gi.random_membership(g.n, 50, 3)
    memb[7] = g.n + 5                                  # a label out of range: the count reads -1
    assert _count_noalloc(g, memb) == -1
    # no vertex: nothing is disconnected
    dev = torch.device("cuda:0")
    out = torch.full((1,), -7, dtype=torch.int64, device=dev)
    gsp.count_disconnected_noalloc(torch.zeros(1, dtype=torch.int64, device=dev),
                                   torch.zeros(0, dtype=torch.int32, device=dev),
                                   torch.zeros(0, dtype=torch.int32, device=dev), out)
    torch.cuda.synchronize()
    assert int(out.item()) == 0
    # more vertices than the scratch holds: refused before any launch
    st = gsp.lib().gsp_count_disconnected_noalloc(gsp.lib().gsp_noalloc_max_vertices() + 1, 0, 1, None, 1, 1, None)
    assert st == gsp.GSP_EINVAL
