"""TEST INFRASTRUCTURE ONLY: ctypes binding of the sequential CPU oracle.

The oracle (``oracle.c``) is a plain, slow, fp64 rendering of GSP-Louvain
(arXiv 2402.11454); ``prune.c`` adds the learned pruning gate that runs
beside its local-moving phase (features, the 8-64-64-1 network, its loss,
gradients and Adam, and the gated synchronous phase).  Only the tests, ``__graft_entry__.smoke()`` and the
bench's CPU-baseline leg may import this package; the GPU library never does.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "prune.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compiles oracle.c and prune.c (always recompiles): -O2, no fast-math, no FMA."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", _LIB_PATH + ".tmp", *_SRCS, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Trace(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("threshold", ctypes.c_uint64), ("cap", ctypes.c_int64),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("vertex", ctypes.c_void_p),
                ("meta", ctypes.c_void_p), ("rows", ctypes.c_int64), ("seen", ctypes.c_int64)]


class _Options(ctypes.Structure):
    _fields_ = [("tolerance", ctypes.c_double), ("max_passes", ctypes.c_int32),
                ("max_iterations", ctypes.c_int32), ("tolerance_drop", ctypes.c_double),
                ("aggregation_tolerance", ctypes.c_double), ("sync_moves", ctypes.c_int32),
                ("sync_rounds", ctypes.c_int32), ("split_mode", ctypes.c_int32),
                ("prune_params", ctypes.c_void_p), ("prune_theta_logit", ctypes.c_double),
                ("trace", ctypes.POINTER(_Trace)), ("return_moves", ctypes.c_int32),
                ("confirm_final", ctypes.c_int32), ("leiden", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("iterations", ctypes.c_int32 * 64),
                ("communities", ctypes.c_int64 * 64), ("vertices", ctypes.c_int64 * 64),
                ("modularity", ctypes.c_double), ("counters", ctypes.c_int64 * 4),
                ("tau", ctypes.c_double * 64), ("final_iterations", ctypes.c_int32),
                ("refine_iterations", ctypes.c_int32 * 64), ("refined", ctypes.c_int64 * 64)]


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
        "orc_move_sync": (i32, [i64, vp, vp, vp, dbl, vp, vp, dbl, i32, i32, vp, vp, i32]),
        "orc_refine_sync": (i32, [i64, vp, vp, vp, dbl, vp, vp, vp, dbl, i32, i32, vp, vp]),
        "orc_split_bfs": (i32, [i64, vp, vp, vp, vp]),
        "orc_split_lp": (i32, [i64, vp, vp, vp, i32, vp]),
        "orc_renumber": (i64, [i64, vp, vp]),
        "orc_aggregate": (i64, [i64, vp, vp, vp, vp, i64, vp, vp, vp, i64]),
        "orc_disconnected": (i64, [i64, vp, vp, vp, vp]),
        "orc_louvain": (i32, [i64, vp, vp, vp, ctypes.POINTER(_Options), vp, ctypes.POINTER(_Stats)]),
        "orc_decide_row": (i32, [i64, i64, vp, vp, vp, vp, vp, dbl, dbl, vp, vp]),
        "orc_weight_grid": (i32, [i64, vp, vp]),
        "orc_set_verbose": (None, [i32]),
        "orc_gain_fixed": (i64, [dbl, dbl]),
        "orc_bf16": (ctypes.c_float, [ctypes.c_float]),
        "orc_plog2": (dbl, [dbl]),
        "orc_gate_features": (None, [i64, dbl, dbl, ctypes.c_float, ctypes.c_float, ctypes.c_uint8, dbl, i32, i32,
                                     vp]),
        "orc_mlp_logits": (None, [vp, vp, i64, i32, vp]),
        "orc_mlp_loss_grad": (dbl, [vp, vp, vp, i64, dbl, vp]),
        "orc_mlp_loss_grad_f64": (dbl, [vp, vp, vp, i64, dbl, vp]),
        "orc_mlp_loss_grad_f32": (ctypes.c_float, [vp, vp, vp, i64, ctypes.c_float, vp]),
        "orc_mlp_train_adam": (i64, [vp, vp, vp, i64, i64, i32, dbl, dbl, vp]),
        "orc_trace_keep": (i32, [ctypes.c_uint64, i32, i32, i64, ctypes.c_uint64]),
        "orc_move_sync_gated": (i32, [i64, vp, vp, vp, dbl, vp, vp, dbl, i32, i32, vp, dbl, i32,
                                      ctypes.POINTER(_Trace), vp, vp, vp, i32, i32]),
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
        """A generator graph in the oracle's types, its weights taken on the
        grid of exact sums (:func:`weight_grid`; a no-op for unit weights and
        for every workload but the largest)."""
        if isinstance(g, CSR):
            return g
        if g.weights is None:
            return cls(g.n, g.offsets, g.cols, None)
        w = g.weights.astype(np.float64)
        weight_grid(w)
        return cls(g.n, g.offsets, g.cols, w)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def args(self):
        return (self.n, _p(self.off), _p(self.col), _p(self.w))


def _memb(m, n) -> np.ndarray:
    m = np.ascontiguousarray(m, dtype=np.int32)
    assert m.shape[0] == n
    return m


def set_verbose(on: bool) -> None:
    """Progress lines on stderr from long oracle runs."""
    _load().orc_set_verbose(int(on))


def weight_grid(w: np.ndarray):
    """Takes fp64 weights (in place) on the grid of multiples of 2^-S that
    makes every sum of them exact; returns (S, weights that moved)."""
    assert w.dtype == np.float64 and w.flags.c_contiguous
    ch = ctypes.c_int64()
    S = _load().orc_weight_grid(w.shape[0], _p(w), ctypes.byref(ch))
    return int(S), int(ch.value)


def gain_fixed(gain: float, M2: float) -> int:
    """A mover's share of the iteration's gain total, in units of 2^-61."""
    return int(_load().orc_gain_fixed(float(gain), float(M2)))


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
    sigma = np.bincount(m, weights=K, minlength=g.n).astype(np.float64)
    csize = np.bincount(m, minlength=g.n).astype(np.int32)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    dec = np.empty(g.n, dtype=np.int32)
    gain = np.empty(g.n, dtype=np.float64)
    moved = _load().orc_move_sync_step(*g.args(), M2, _p(K), _p(m), _p(sigma), _p(csize), _p(act), _p(dec), _p(gain))
    if moved < 0:
        raise ValueError("orc_move_sync_step failed")
    return dec, gain, int(moved)


def move_sync(g, memb=None, tau: float = 0.0, max_iter: int = 20, rounds: int = 8, returns: bool = False):
    """Returns (membership, l_i, per-iteration dQ, per-iteration movers);
    returns=True leaves return moves out of the gain totals."""
    g = CSR.of(g)
    K, M2 = vertex_weights(g)
    m = np.arange(g.n, dtype=np.int32) if memb is None else _memb(memb, g.n).copy()
    dq = np.zeros(max(max_iter, 1), dtype=np.float64)
    mv = np.zeros(max(max_iter, 1), dtype=np.int64)
    li = _load().orc_move_sync(*g.args(), M2, _p(K), _p(m), tau, max_iter, rounds, _p(dq), _p(mv), int(returns))
    if li < 0:
        raise ValueError("orc_move_sync failed")
    return m, li, dq[:li], mv[:li]


def refine_sync(g, bound, memb=None, tau: float = 0.0, max_iter: int = 20, rounds: int = 8):
    """GSP-Leiden's refinement within the communities `bound`, from memb
    (default: every vertex alone); returns (sub-communities, iterations,
    per-iteration dQ, per-iteration movers)."""
    g = CSR.of(g)
    K, M2 = vertex_weights(g)
    b = _memb(bound, g.n)
    m = np.arange(g.n, dtype=np.int32) if memb is None else _memb(memb, g.n).copy()
    dq = np.zeros(max(max_iter, 1), dtype=np.float64)
    mv = np.zeros(max(max_iter, 1), dtype=np.int64)
    li = _load().orc_refine_sync(*g.args(), M2, _p(K), _p(b), _p(m), tau, max_iter, rounds, _p(dq), _p(mv))
    if li < 0:
        raise ValueError("orc_refine_sync failed")
    return m, li, dq[:li], mv[:li]


def decide_row(i, cols, weights, memb, sigma, csize, ki, M2):
    """Synchronous decision of vertex i from its row alone: (community,
    gain numerator, [best, second, stay] scores)."""
    c = np.ascontiguousarray(cols, dtype=np.int32)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    gain = ctypes.c_double()
    sc = np.empty(3, dtype=np.float64)
    d = _load().orc_decide_row(int(i), c.shape[0], _p(c), _p(w), _p(memb), _p(sigma), _p(csize), float(ki),
                               float(M2), ctypes.byref(gain), _p(sc))
    return int(d), gain.value, sc


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


MLP_PARAMS = 4801


def _params(params):
    if params is None:
        return None
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.shape == (MLP_PARAMS,)
    return p


def logit_of(theta: float) -> float:
    """Gate threshold on the probability -> threshold on the logit."""
    return math.log(theta / (1.0 - theta))


def bf16(x) -> np.ndarray:
    """bf16 rounding (to nearest even) of fp32 values, elementwise."""
    x = np.asarray(x, dtype=np.float32).ravel()
    f = _load().orc_bf16
    return np.array([f(float(v)) for v in x], dtype=np.float32)


def plog2(x: float) -> float:
    return float(_load().orc_plog2(float(x)))


def gate_features(deg, ki, sig_d, hfrac, hgain, hbits, dmoved, pass_index, iteration) -> np.ndarray:
    x = np.empty(8, dtype=np.float32)
    _load().orc_gate_features(int(deg), float(ki), float(sig_d), float(hfrac), float(hgain), int(hbits),
                              float(dmoved), int(pass_index), int(iteration), _p(x))
    return x


def mlp_logits(params, x, bf16_formats: bool = False) -> np.ndarray:
    p = _params(params)
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 8)
    out = np.empty(x.shape[0], dtype=np.float64)
    _load().orc_mlp_logits(_p(p), _p(x), x.shape[0], int(bf16_formats), _p(out))
    return out


def mlp_loss_grad(params, x, y, pos_weight: float = 1.0, fp32: bool = False):
    """(loss, gradient[4801]) of the mean pos-weighted BCE."""
    p = _params(params)
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 8)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    if fp32:
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        loss = _load().orc_mlp_loss_grad_f32(_p(p), _p(x), _p(y), x.shape[0], pos_weight, _p(g))
    else:
        g = np.empty(MLP_PARAMS, dtype=np.float64)
        loss = _load().orc_mlp_loss_grad(_p(p), _p(x), _p(y), x.shape[0], pos_weight, _p(g))
    return float(loss), g


def mlp_loss_grad_f64(params, x, y, pos_weight: float = 1.0):
    """Loss and gradient at fp64 parameters (for finite differences)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    assert p.shape == (MLP_PARAMS,)
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 8)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    g = np.empty(MLP_PARAMS, dtype=np.float64)
    loss = _load().orc_mlp_loss_grad_f64(_p(p), _p(x), _p(y), x.shape[0], pos_weight, _p(g))
    return float(loss), g


def mlp_train_adam(params, x, y, batch: int, epochs: int, lr: float, pos_weight: float = 1.0):
    """Returns (trained params fp32, per-epoch mean batch loss)."""
    p = _params(params).copy()
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 8)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    el = np.zeros(max(epochs, 1), dtype=np.float64)
    t = _load().orc_mlp_train_adam(_p(p), _p(x), _p(y), x.shape[0], batch, epochs, lr, pos_weight, _p(el))
    if t < 0:
        raise ValueError("orc_mlp_train_adam failed")
    return p, el[:epochs]


def trace_keep(seed: int, pass_index: int, sweep: int, i: int, threshold: int) -> bool:
    return bool(_load().orc_trace_keep(seed, pass_index, sweep, i, threshold))


class Trace:
    """Trace buffers: rows of (features, moved, vertex, pass * 256 + sweep)."""

    def __init__(self, cap: int, seed: int = 0, rate: float = 1.0):
        self.cap = int(cap)
        self.x = np.zeros((self.cap, 8), dtype=np.float32)
        self.y = np.zeros(self.cap, dtype=np.uint8)
        self.vertex = np.zeros(self.cap, dtype=np.int32)
        self.meta = np.zeros(self.cap, dtype=np.int32)
        thr = 2 ** 64 - 1 if rate >= 1.0 else int(rate * 2 ** 64)
        self.c = _Trace(seed, thr, self.cap, _p(self.x), _p(self.y), _p(self.vertex), _p(self.meta), 0, 0)

    @property
    def rows(self) -> int:
        return int(self.c.rows)

    @property
    def seen(self) -> int:
        return int(self.c.seen)

    def arrays(self):
        r = self.rows
        return self.x[:r], self.y[:r], self.vertex[:r], self.meta[:r]


def move_sync_gated(g, params=None, theta: float = 0.5, pass_index: int = 0, memb=None, tau: float = 0.0,
                    max_iter: int = 20, rounds: int = 8, trace: Optional[Trace] = None, theta_logit=None,
                    returns: bool = False, confirm: bool = True):
    """Returns (membership, l_i, dQ per counted iteration, movers per counted
    iteration, counters dict)."""
    g = CSR.of(g)
    K, M2 = vertex_weights(g)
    m = np.arange(g.n, dtype=np.int32) if memb is None else _memb(memb, g.n).copy()
    dq = np.zeros(max(max_iter, 1), dtype=np.float64)
    mv = np.zeros(max(max_iter, 1), dtype=np.int64)
    c4 = np.zeros(4, dtype=np.int64)
    p = _params(params)
    tl = theta_logit if theta_logit is not None else logit_of(theta)
    li = _load().orc_move_sync_gated(*g.args(), M2, _p(K), _p(m), tau, max_iter, rounds, _p(p), tl, pass_index,
                                     ctypes.byref(trace.c) if trace is not None else None, _p(dq), _p(mv), _p(c4),
                                     int(returns), int(confirm))
    if li < 0:
        raise ValueError("orc_move_sync_gated failed")
    cnt = dict(scanned_vertices=int(c4[0]), scanned_entries=int(c4[1]), pruned=int(c4[2]), confirm_sweeps=int(c4[3]))
    return m, li, dq[:li], mv[:li], cnt


def louvain(g, tolerance: float = 1e-2, max_passes: int = 10, max_iterations: int = 20,
            tolerance_drop: float = 10.0, aggregation_tolerance: float = 0.8,
            sync: bool = False, rounds: int = 8, split_mode: int = 0, prune_params=None, theta: float = 0.5,
            trace: Optional[Trace] = None, theta_logit=None, return_moves: bool = False,
            confirm_final: bool = False, leiden: bool = False) -> Result:
    """The whole method; split_mode 0 = every pass, 1 = after the last, 2 = none.
    prune_params / trace / return_moves need sync=True; leiden=True runs
    GSP-Leiden (sync=True, no gate or trace)."""
    g = CSR.of(g)
    p = _params(prune_params)
    tl = theta_logit if theta_logit is not None else logit_of(theta)
    opt = _Options(tolerance, max_passes, max_iterations, tolerance_drop, aggregation_tolerance,
                   int(sync), rounds, split_mode, _p(p), tl,
                   ctypes.pointer(trace.c) if trace is not None else None, int(return_moves), int(confirm_final),
                   int(leiden))
    st = _Stats()
    memb = np.empty(g.n, dtype=np.int32)
    passes = _load().orc_louvain(*g.args(), ctypes.byref(opt), _p(memb), ctypes.byref(st))
    if passes < 0:
        raise ValueError("orc_louvain failed")
    k = min(passes, 64)
    r = Result(memb, passes, list(st.iterations[:k]), list(st.communities[:k]), list(st.vertices[:k]),
               float(st.modularity))
    r.counters = dict(scanned_vertices=int(st.counters[0]), scanned_entries=int(st.counters[1]),
                      pruned=int(st.counters[2]), confirm_sweeps=int(st.counters[3]))
    r.tau = list(st.tau[:k])
    r.final_iterations = int(st.final_iterations)
    r.refine_iterations = list(st.refine_iterations[:k])
    r.refined = list(st.refined[:k])
    return r
