"""Independent exact-arithmetic helpers for pinning the oracle.

Nothing here calls the oracle: modularity is evaluated from the all-pairs
form of Eq. 1 (Section 3.2) with Python fractions, so results are exact and
share no arithmetic with the oracle's community-form fp64 code.
"""
from fractions import Fraction
from itertools import combinations

import numpy as np


def dense(g):
    """Dense weighted adjacency as nested lists of Fractions (self-loop
    entries counted as stored, once)."""
    n = g.n
    A = [[Fraction(0)] * n for _ in range(n)]
    w = g.weights_f64() if hasattr(g, "weights_f64") else g.w
    off = g.offsets if hasattr(g, "offsets") else g.off
    col = g.cols if hasattr(g, "cols") else g.col
    for i in range(n):
        for e in range(int(off[i]), int(off[i + 1])):
            A[i][int(col[e])] += Fraction(float(w[e]))
    return A


def modularity_allpairs(A, memb):
    """Q = 1/2m sum_{i,j in V} [A_ij - K_i K_j / 2m] delta(C_i, C_j), exact."""
    n = len(A)
    K = [sum(row) for row in A]
    M2 = sum(K)
    if M2 == 0:
        return Fraction(0)
    q = Fraction(0)
    for i in range(n):
        for j in range(n):
            if memb[i] == memb[j]:
                q += A[i][j] - K[i] * K[j] / M2
    return q / M2


def set_partitions(n):
    """All set partitions of range(n) as restricted growth strings."""
    a = [0] * n

    def rec(i, m):
        if i == n:
            yield list(a)
            return
        for v in range(m + 1):
            a[i] = v
            yield from rec(i + 1, max(m, v + 1) if v == m else m)

    if n == 0:
        yield []
        return
    yield from rec(1, 1)


def max_modularity_bruteforce(A):
    """Max Q over every partition of a small graph (Bell(n) evaluations),
    vectorised over partitions with numpy in float64."""
    n = len(A)
    Af = np.array([[float(x) for x in row] for row in A])
    K = Af.sum(1)
    M2 = K.sum()
    B = Af - np.outer(K, K) / M2
    best, arg = -1.0, None
    parts = np.array(list(set_partitions(n)), dtype=np.int64)
    for s in range(0, parts.shape[0], 20000):
        P = parts[s:s + 20000]
        same = (P[:, :, None] == P[:, None, :])
        q = (same * B[None]).sum((1, 2)) / M2
        k = int(np.argmax(q))
        if q[k] > best:
            best, arg = float(q[k]), P[k]
    return best, arg


def components_union_find(n, off, col, memb):
    """Components of the same-community subgraph; label = smallest vertex."""
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for i in range(n):
        for e in range(int(off[i]), int(off[i + 1])):
            j = int(col[e])
            if memb[i] == memb[j]:
                a, b = find(i), find(j)
                if a != b:
                    parent[max(a, b)] = min(a, b)
    return np.array([find(i) for i in range(n)], dtype=np.int32)


def clique_edges(s, base=0):
    return [(base + a, base + b) for a, b in combinations(range(s), 2)]
