"""TEST INFRASTRUCTURE ONLY: ctypes binding of the sequential CPU oracle.

The oracle (``oracle.c``) is a plain, slow, fp64 rendering of GSP-Louvain
(arXiv 2402.11454).  Only the tests, ``__graft_entry__.smoke()`` and the
bench's CPU-baseline leg may import this package; the GPU library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compiles oracle.c (always recompiles): -O2, no fast-math, no FMA."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Options(ctypes.Structure):
    _fields_ = [("tolerance", ctypes.c_double), ("max_passes", ctypes.c_int32),
                ("max_iterations", ctypes.c_int32), ("tolerance_drop", ctypes.c_double),
                ("aggregation_tolerance", ctypes.c_double), ("sync_moves", ctypes.c_int32),
                ("sync_rounds", ctypes.c_int32), ("split_mode", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("iterations", ctypes.c_int32 * 64),
                ("communities", ctypes.c_int64 * 64), ("vertices", ctypes.c_int64 * 64),
                ("modularity", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sig = {
        "orc_vertex_weights": (dbl, [i64, vp, vp, vp, vp]),
        "orc_modularity": (dbl, [i64, vp, vp, vp, vp]),
        "orc_delta_modularity": (dbl, [i64, vp, vp, vp, vp, i64, i32]),
        "orc_move_async": (i32, [i64, vp, vp, vp, dbl, vp, vp, vp, dbl, i32, vp]),
        "orc_move_sync_step": (i64, [i64, vp, vp, vp, dbl, vp, vp, vp, vp, vp, vp, vp]),
        "orc_move_sync": (i32, [i64, vp, vp, vp, dbl, vp, vp, dbl, i32, i32, vp, vp]),
        "orc_split_bfs": (i32, [i64, vp, vp, vp, vp]),
        "orc_split_lp": (i32, [i64, vp, vp, vp, i32, vp]),
        "orc_renumber": (i64, [i64, vp, vp]),
        "orc_aggregate": (i64, [i64, vp, vp, vp, vp, i64, vp, vp, vp, i64]),
        "orc_disconnected": (i64, [i64, vp, vp, vp, vp]),
        "orc_louvain": (i32, [i64, vp, vp, vp, ctypes.POINTER(_Options), vp, ctypes.POINTER(_Stats)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class CSR:
    """Host CSR in the oracle's types: int64 offsets, int32 cols, fp64 weights."""

    def __init__(self, n, offsets, cols, weights=None):
        self.n = int(n)
        self.off = np.ascontiguousarray(offsets, dtype=np.int64)
        self.col = np.ascontiguousarray(cols, dtype=np.int32)
        if weights is None:
            self.w = np.ones(self.col.shape[0], dtype=np.float64)
        else:
            self.w = np.ascontiguousarray(weights, dtype=np.float64)
        assert self.off.shape[0] == self.n + 1 and self.off[-1] == self.col.shape[0] == self.w.shape[0]

    @classmethod
    def of(cls, g) -> "CSR":
        if isinstance(g, CSR):
            return g
        return cls(g.n, g.offsets, g.cols, None if g.weights is None else g.weights.astype(np.float64))

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def args(self):
        return (self.n, _p(self.off), _p(self.col), _p(self.w))


def _memb(m, n) -> np.ndarray:
    m = np.ascontiguousarray(m, dtype=np.int32)
    assert m.shape[0] == n
    return m


def vertex_weights(g):
    g = CSR.of(g)
    K = np.empty(g.n, dtype=np.float64)
    M2 = _load().orc_vertex_weights(*g.args(), _p(K))
    return K, M2


def modularity(g, memb) -> float:
    g = CSR.of(g)
    return float(_load().orc_modularity(*g.args(), _p(_memb(memb, g.n))))


def delta_modularity(g, memb, i: int, c: int) -> float:
    g = CSR.of(g)
    return float(_load().orc_delta_modularity(*g.args(), _p(_memb(memb, g.n)), i, c))


def move_async(g, memb=None, tau: float = 0.0, max_iter: int = 20):
    """Returns (membership, l_i, per-iteration dQ)."""
    g = CSR.of(g)
    K, M2 = vertex_weights(g)
    m = np.arange(g.n, dtype=np.int32) if memb is None else _memb(memb, g.n).copy()
    sigma = np.zeros(g.n, dtype=np.float64)
    np.add.at(sigma, m, K)
    dq = np.zeros(max(max_iter, 1), dtype=np.float64)
    li = _load().orc_move_async(*g.args(), M2, _p(K), _p(m), _p(sigma), tau, max_iter, _p(dq))
    if li < 0:
        raise ValueError("orc_move_async failed")
    return m, li, dq[:li]


def move_sync_step(g, memb, active=None, K=None, M2=None):
    """One synchronous step from a snapshot; returns (dec, gain, moved)."""
    g = CSR.of(g)
    if K is None:
        K, M2 = vertex_weights(g)
    m = _memb(memb, g.n)
    sigma = np.zeros(g.n, dtype=np.float64)
    np.add.at(sigma, m, K)
    csize = np.bincount(m, minlength=g.n).astype(np.int32)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    dec = np.empty(g.n, dtype=np.int32)
    gain = np.empty(g.n, dtype=np.float64)
    moved = _load().orc_move_sync_step(*g.args(), M2, _p(K), _p(m), _p(sigma), _p(csize), _p(act), _p(dec), _p(gain))
    if moved < 0:
        raise ValueError("orc_move_sync_step failed")
    return dec, gain, int(moved)


def move_sync(g, memb=None, tau: float = 0.0, max_iter: int = 20, rounds: int = 8):
    """Returns (membership, l_i, per-iteration dQ, per-iteration movers)."""
    g = CSR.of(g)
    K, M2 = vertex_weights(g)
    m = np.arange(g.n, dtype=np.int32) if memb is None else _memb(memb, g.n).copy()
    dq = np.zeros(max(max_iter, 1), dtype=np.float64)
    mv = np.zeros(max(max_iter, 1), dtype=np.int64)
    li = _load().orc_move_sync(*g.args(), M2, _p(K), _p(m), tau, max_iter, rounds, _p(dq), _p(mv))
    if li < 0:
        raise ValueError("orc_move_sync failed")
    return m, li, dq[:li], mv[:li]


def split_bfs(g, memb) -> np.ndarray:
    g = CSR.of(g)
    lab = np.empty(g.n, dtype=np.int32)
    if _load().orc_split_bfs(g.n, _p(g.off), _p(g.col), _p(_memb(memb, g.n)), _p(lab)) < 0:
        raise ValueError("orc_split_bfs failed")
    return lab


def split_lp(g, memb, pruned: bool = True):
    g = CSR.of(g)
    lab = np.empty(g.n, dtype=np.int32)
    sweeps = _load().orc_split_lp(g.n, _p(g.off), _p(g.col), _p(_memb(memb, g.n)), int(pruned), _p(lab))
    if sweeps < 0:
        raise ValueError("orc_split_lp failed")
    return lab, int(sweeps)


def renumber(labels):
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.empty_like(labels)
    G = _load().orc_renumber(labels.shape[0], _p(labels), _p(out))
    if G < 0:
        raise ValueError("orc_renumber failed")
    return out, int(G)


def aggregate(g, memb, ncomm: int) -> CSR:
    g = CSR.of(g)
    m = _memb(memb, g.n)
    off2 = np.empty(ncomm + 1, dtype=np.int64)
    col2 = np.empty(max(g.nnz, 1), dtype=np.int32)
    w2 = np.empty(max(g.nnz, 1), dtype=np.float64)
    nnz = _load().orc_aggregate(*g.args(), _p(m), ncomm, _p(off2), _p(col2), _p(w2), g.nnz)
    if nnz < 0:
        raise ValueError("orc_aggregate failed")
    return CSR(ncomm, off2, col2[:nnz].copy(), w2[:nnz].copy())


def disconnected(g, memb):
    """Returns (count, per-community flags)."""
    g = CSR.of(g)
    flags = np.zeros(g.n, dtype=np.uint8)
    cnt = _load().orc_disconnected(g.n, _p(g.off), _p(g.col), _p(_memb(memb, g.n)), _p(flags))
    if cnt < 0:
        raise ValueError("orc_disconnected failed")
    return int(cnt), flags


@dataclass
class Result:
    membership: np.ndarray
    passes: int
    iterations: list = field(default_factory=list)
    communities: list = field(default_factory=list)
    vertices: list = field(default_factory=list)
    modularity: float = 0.0


def louvain(g, tolerance: float = 1e-2, max_passes: int = 10, max_iterations: int = 20,
            tolerance_drop: float = 10.0, aggregation_tolerance: float = 0.8,
            sync: bool = False, rounds: int = 8, split_mode: int = 0) -> Result:
    """The whole method; split_mode 0 = every pass, 1 = after the last, 2 = none."""
    g = CSR.of(g)
    opt = _Options(tolerance, max_passes, max_iterations, tolerance_drop, aggregation_tolerance,
                   int(sync), rounds, split_mode)
    st = _Stats()
    memb = np.empty(g.n, dtype=np.int32)
    passes = _load().orc_louvain(*g.args(), ctypes.byref(opt), _p(memb), ctypes.byref(st))
    if passes < 0:
        raise ValueError("orc_louvain failed")
    k = min(passes, 64)
    return Result(memb, passes, list(st.iterations[:k]), list(st.communities[:k]), list(st.vertices[:k]),
                  float(st.modularity))
