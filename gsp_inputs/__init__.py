"""Seeded synthetic graph inputs.

This module only draws random graphs (planted-partition SBM, R-MAT, batches of
SBMs and hand-built edge lists) and returns them as symmetric CSR arrays.  It
holds none of the community-detection arithmetic, so both the GPU library's
tests and the CPU oracle's tests can take their inputs from it.

The generators live in ``gen.c`` (compiled to ``libgsp_inputs.so`` by
:func:`build`); this file is argument marshalling plus the workload presets
whose shapes follow the graphs of the paper's evaluation (Section 5.1.3:
undirected graphs, reverse edges stored, unit weight by default).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libgsp_inputs.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compiles gen.c into libgsp_inputs.so (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, u64, dbl, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
    lib.gen_sbm.restype = vp
    lib.gen_sbm.argtypes = [i64, i64, dbl, dbl, u64, i32, i32, dbl, dbl]
    lib.gen_rmat.restype = vp
    lib.gen_rmat.argtypes = [i32, i64, dbl, dbl, dbl, u64, i32, i32, dbl, dbl]
    lib.gen_dcsbm.restype = vp
    lib.gen_dcsbm.argtypes = [i64, dbl, i64, i64, dbl, i64, i64, dbl, u64, i32, i32, dbl, dbl]
    lib.gen_road.restype = vp
    lib.gen_road.argtypes = [i64, dbl, i32, u64, i32]
    lib.gen_from_edges.restype = vp
    lib.gen_from_edges.argtypes = [i64, i64, vp, vp]
    lib.gen_free.argtypes = [vp]
    lib.gen_n.restype = i64
    lib.gen_n.argtypes = [vp]
    lib.gen_nnz.restype = i64
    lib.gen_nnz.argtypes = [vp]
    lib.gen_has_weights.restype = i32
    lib.gen_has_weights.argtypes = [vp]
    lib.gen_has_blocks.restype = i32
    lib.gen_has_blocks.argtypes = [vp]
    lib.gen_copy.argtypes = [vp, vp, vp, vp, vp]
    lib.gen_uniform.argtypes = [u64, i64, vp]
    lib.gen_set_verbose.argtypes = [i32]
    _lib = lib
    return lib


@dataclass
class Graph:
    """Symmetric CSR graph on the host.

    offsets: int64[n+1]; cols: int32[nnz]; weights: float32[nnz] or None
    (unit weights); block: planted block of each vertex or None.
    """

    n: int
    offsets: np.ndarray
    cols: np.ndarray
    weights: Optional[np.ndarray] = None
    block: Optional[np.ndarray] = None
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.cols.shape[0])

    def weights_f64(self) -> np.ndarray:
        if self.weights is None:
            return np.ones(self.nnz, dtype=np.float64)
        return self.weights.astype(np.float64)

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)


def _take(h, name: str) -> Graph:
    lib = _load()
    if not h:
        raise MemoryError(f"generator {name} failed")
    try:
        n, nnz = lib.gen_n(h), lib.gen_nnz(h)
        off = np.empty(n + 1, dtype=np.int64)
        col = np.empty(nnz, dtype=np.int32)
        w = np.empty(nnz, dtype=np.float32) if lib.gen_has_weights(h) else None
        blk = np.empty(n, dtype=np.int64) if lib.gen_has_blocks(h) else None
        lib.gen_copy(h, off.ctypes.data, col.ctypes.data,
                     w.ctypes.data if w is not None else None,
                     blk.ctypes.data if blk is not None else None)
    finally:
        lib.gen_free(h)
    return Graph(n=int(n), offsets=off, cols=col, weights=w, block=blk, name=name)


def sbm(n: int, blocks: int, p_in: float, p_out: float, seed: int, permute: bool = True,
        weights: Optional[tuple] = None, name: str = "sbm") -> Graph:
    """Planted-partition SBM (equal consecutive blocks, then relabelled)."""
    lo, hi = weights if weights is not None else (1.0, 1.0)
    h = _load().gen_sbm(n, blocks, p_in, p_out, seed, int(permute), int(weights is not None), lo, hi)
    return _take(h, name)


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int, permute: bool = True,
         weights: Optional[tuple] = None, name: str = "rmat") -> Graph:
    """R-MAT with edge_factor * 2^scale samples, symmetrised and deduplicated."""
    lo, hi = weights if weights is not None else (1.0, 1.0)
    samples = edge_factor << scale
    h = _load().gen_rmat(scale, samples, a, b, c, seed, int(permute), int(weights is not None), lo, hi)
    return _take(h, name)


def dcsbm(n: int, deg_alpha: float, kmin: int, kmax: int, size_alpha: float, smin: int, smax: int, mu: float,
          seed: int, permute: bool = True, weights: Optional[tuple] = (1.0, 4.0), name: str = "dcsbm") -> Graph:
    """Degree-corrected SBM with power-law degrees and community sizes (see
    gen.c): ``block`` holds each vertex's planted community."""
    lo, hi = weights if weights is not None else (1.0, 1.0)
    h = _load().gen_dcsbm(n, deg_alpha, kmin, kmax, size_alpha, smin, smax, mu, seed, int(permute),
                          int(weights is not None), lo, hi)
    return _take(h, name)


def road(side: int, keep: float, max_inner: int, seed: int, permute: bool = True, name: str = "road") -> Graph:
    """Road-like graph: a side x side lattice of intersections, each lattice
    edge kept with probability `keep` and subdivided into a chain of 0 ..
    max_inner degree-2 vertices (see gen.c); unit weights."""
    return _take(_load().gen_road(side, keep, max_inner, seed, int(permute)), name)


def from_edges(n: int, edges, weights=None, name: str = "edges") -> Graph:
    """Graph from an undirected edge list [(u, v), ...].

    Without ``weights`` the graph has unit weights.  ``weights`` maps each
    undirected edge (min, max) to a weight; self-loops given in ``edges`` are
    dropped by the CSR builder, so hand-built graphs with self-loops use
    :func:`with_self_loops`.
    """
    e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    eu = np.ascontiguousarray(e[:, 0])
    ev = np.ascontiguousarray(e[:, 1])
    h = _load().gen_from_edges(n, e.shape[0], eu.ctypes.data, ev.ctypes.data)
    g = _take(h, name)
    if weights is not None:
        w = np.empty(g.nnz, dtype=np.float32)
        for i in range(n):
            for k in range(g.offsets[i], g.offsets[i + 1]):
                j = int(g.cols[k])
                w[k] = weights[(min(i, j), max(i, j))]
        g.weights = w
    return g


def with_self_loops(g: Graph, loops: dict) -> Graph:
    """Returns a copy of g with a self-loop entry (i, i, w) added per item of
    ``loops`` ({i: w}); the entry is stored once in row i."""
    rows = []
    for i in range(g.n):
        s, e = g.offsets[i], g.offsets[i + 1]
        cols = list(g.cols[s:e])
        ws = list(g.weights_f64()[s:e])
        if i in loops:
            cols.append(i)
            ws.append(float(loops[i]))
        order = np.argsort(np.asarray(cols, dtype=np.int64), kind="stable")
        rows.append(([cols[k] for k in order], [ws[k] for k in order]))
    off = np.zeros(g.n + 1, dtype=np.int64)
    for i, (c, _) in enumerate(rows):
        off[i + 1] = off[i] + len(c)
    col = np.concatenate([np.asarray(c, dtype=np.int32) for c, _ in rows]) if off[-1] else np.zeros(0, np.int32)
    w = np.concatenate([np.asarray(x, dtype=np.float32) for _, x in rows]) if off[-1] else np.zeros(0, np.float32)
    return Graph(n=g.n, offsets=off, cols=col, weights=w, block=g.block, name=g.name + "+loops")


def set_verbose(on: bool) -> None:
    """Progress lines on stderr from the generators (for long generations)."""
    _load().gen_set_verbose(int(on))


def uniform(seed: int, count: int) -> np.ndarray:
    """Seeded uniform draws in [0, 1) (xoshiro256**)."""
    out = np.empty(count, dtype=np.float64)
    if count:
        _load().gen_uniform(seed, count, out.ctypes.data)
    return out


def random_membership(n: int, ncomm: int, seed: int) -> np.ndarray:
    """Seeded random labels in [0, ncomm) for n vertices."""
    u = uniform(seed, n)
    return np.minimum((u * ncomm).astype(np.int64), ncomm - 1).astype(np.int32)


# --------------------------------------------------------------------------
# Workload presets.  The paper's 13 SuiteSparse graphs are not available, so
# these seeded synthetic graphs stand in for them (same shape classes).
# --------------------------------------------------------------------------

RMAT_ABC = (0.57, 0.19, 0.19)


def planted_sbm_10k(seed: int = 1) -> Graph:
    """10,000 vertices, 100 equal blocks, expected degree 20 with 80% of the
    edges inside blocks: p_in = 16/99, p_out = 4/9900; unit weights."""
    return sbm(10_000, 100, 16.0 / 99.0, 4.0 / 9900.0, seed, name="sbm-10k")


def rmat20(seed: int = 20) -> Graph:
    """R-MAT scale 20, 16 samples per vertex, a/b/c/d = .57/.19/.19/.05,
    symmetrised, deduplicated, no self-loops, unit weights."""
    return rmat(20, 16, *RMAT_ABC, seed, name="rmat-20")


def rmat_small(scale: int, seed: int, edge_factor: int = 16, weights=None) -> Graph:
    """Smaller R-MAT of the same law, for parity tests."""
    return rmat(scale, edge_factor, *RMAT_ABC, seed, weights=weights, name=f"rmat-{scale}")


def dcsbm_4m(seed: int, n: int = 4_000_000) -> Graph:
    """The social-network-shaped workload: n vertices (4M), degrees power
    law 2.5 on [5, 5000], community sizes power law 1.5 on [20, 50000],
    mixing 0.3, weights uniform in [1, 4] (fp32).  Seeds 0-31 are the
    training graphs of the pruning network, 1000-1007 the held-out ones."""
    return dcsbm(n, 2.5, 5, 5000, 1.5, 20, 50_000, 0.3, seed, name=f"dcsbm-{n}-s{seed}")


def dcsbm_small(n: int, seed: int, mu: float = 0.3, kmax: int = 500, smax: int = 2000) -> Graph:
    """Smaller graph of the same law (tests, quick training)."""
    return dcsbm(n, 2.5, 5, kmax, 1.5, 20, smax, mu, seed, name=f"dcsbm-{n}-s{seed}")


def road_network(seed: int = 7, side: int = 3000) -> Graph:
    """The low-degree, high-diameter workload (the road / k-mer class of the
    paper's graphs, average degree about 2.1): a 3000 x 3000 lattice of
    intersections, 70 % of its edges kept, each subdivided into 0 .. 8
    degree-2 vertices: about 34 M vertices, 37 M undirected edges."""
    return road(side, 0.7, 8, seed, name=f"road-{side}-s{seed}")


def road_small(side: int, seed: int) -> Graph:
    """Smaller graph of the same law, for parity tests."""
    return road(side, 0.7, 8, seed, name=f"road-{side}-s{seed}")


def batch_sbm_params(count: int, master_seed: int = 4):
    """Per-graph parameters of a batch of planted-partition SBMs: n
    log-uniform in [1e3, 2e5], average degree uniform in [4, 40], mixing
    uniform in [0.1, 0.5], round(n / 100) equal blocks."""
    u = uniform(master_seed, 3 * count).reshape(count, 3)
    out = []
    for g in range(count):
        n = int(round(math.exp(math.log(1e3) + (math.log(2e5) - math.log(1e3)) * u[g, 0])))
        d = 4.0 + 36.0 * u[g, 1]
        mu = 0.1 + 0.4 * u[g, 2]
        k = max(1, int(round(n / 100)))
        s = n / k
        p_in = min(1.0, (1.0 - mu) * d / max(s - 1.0, 1.0))
        p_out = min(1.0, mu * d / max(n - s, 1.0)) if k > 1 else 0.0
        out.append(dict(n=n, blocks=k, p_in=p_in, p_out=p_out, seed=master_seed * 1_000_003 + g, degree=d,
                        mixing=mu))
    return out


def batch_sbm(count: int, master_seed: int = 4, scale: float = 1.0):
    """The batch's graphs (planted-partition SBMs, unit weights).  scale < 1
    shrinks every n (at least 100 vertices) keeping its average degree,
    mixing and block size of ~100 vertices."""
    gs = []
    for p in batch_sbm_params(count, master_seed):
        n = max(100, int(round(p["n"] * scale)))
        k = max(1, int(round(n / 100)))
        s = n / k
        d, mu = p["degree"], p["mixing"]
        p_in = min(1.0, (1.0 - mu) * d / max(s - 1.0, 1.0))
        p_out = min(1.0, mu * d / max(n - s, 1.0)) if k > 1 else 0.0
        gs.append(sbm(n, k, p_in, p_out, p["seed"], name=f"batch-{p['seed']}"))
    return gs
