"""GSP-Louvain on AMD Instinct MI355X: Python binding of libgsp.so.

This module only marshals arguments to the C ABI declared in
``include/gsp.h``; every step of the method runs in the library's HIP
kernels.  Arrays may be numpy arrays (host memory) or torch tensors (host or
device memory on the context's GPU); torch is used only for device memory
and streams.  If libgsp.so has not been built, importing works but creating a
:class:`Context` raises, naming the build step: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsp.so")
HEADER = os.path.join(_HERE, "..", "include", "gsp.h")

GSP_OK, GSP_EINVAL, GSP_ENOMEM, GSP_EHIP, GSP_ESTATE, GSP_EGRAPH = 0, -1, -2, -3, -4, -5
HOST, DEVICE = 0, 1
SPLIT_PASS, SPLIT_LAST, SPLIT_NONE = 0, 1, 2
MAX_PASSES_STATS = 64
KERNEL_CLASSES = ("move_small", "move_wave", "move_block", "move_hub", "move_hub_finish", "move_apply", "frontier",
                  "split", "aggregate", "gate", "move_hub_gather")
PRUNE_PLAIN, PRUNE_LEARNED = 0, 1
SPLIT_UF, SPLIT_LPP = 0, 1
ORDER_AUTO, ORDER_LOADED, ORDER_DEGREE = 0, 1, 2
GATE_PARAMS = 4801  # (8*64 + 64) + (64*64 + 64) + (64 + 1)

_STATUS = {GSP_EINVAL: "GSP_EINVAL", GSP_ENOMEM: "GSP_ENOMEM", GSP_EHIP: "GSP_EHIP",
           GSP_ESTATE: "GSP_ESTATE", GSP_EGRAPH: "GSP_EGRAPH"}


class GspError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("max_iterations", ctypes.c_int32), ("sub_rounds", ctypes.c_int32),
                ("tolerance_drop", ctypes.c_double), ("aggregation_tolerance", ctypes.c_double),
                ("split_mode", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("mem_limit_bytes", ctypes.c_uint64), ("prune_mode", ctypes.c_int32),
                ("prune_threshold", ctypes.c_float), ("use_graphs", ctypes.c_int32),
                ("timing_mask", ctypes.c_uint32), ("hub_global", ctypes.c_int32),
                ("hub_max_parts", ctypes.c_int32), ("return_moves", ctypes.c_int32),
                ("split_algo", ctypes.c_int32), ("grid_cap", ctypes.c_int32),
                ("vertex_order", ctypes.c_int32), ("leiden", ctypes.c_int32)]


class KernelStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("items", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("iterations", ctypes.c_int32 * MAX_PASSES_STATS),
                ("vertices", ctypes.c_int64 * MAX_PASSES_STATS),
                ("communities", ctypes.c_int64 * MAX_PASSES_STATS),
                ("moves", ctypes.c_int64), ("scanned_entries", ctypes.c_int64),
                ("ms_move", ctypes.c_double), ("ms_split", ctypes.c_double), ("ms_aggregate", ctypes.c_double),
                ("ms_other", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("kernels", KernelStat * len(KERNEL_CLASSES)),
                ("scanned_vertices", ctypes.c_int64), ("pruned", ctypes.c_int64),
                ("confirm_sweeps", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("split_rounds", ctypes.c_int32),
                ("refine_iterations", ctypes.c_int32 * MAX_PASSES_STATS),
                ("refined", ctypes.c_int64 * MAX_PASSES_STATS), ("ms_refine", ctypes.c_double)]

    def as_dict(self) -> dict:
        k = self.passes
        return dict(passes=k, iterations=list(self.iterations[:k]), vertices=list(self.vertices[:k]),
                    communities=list(self.communities[:k]), moves=self.moves,
                    scanned_entries=self.scanned_entries, ms_move=self.ms_move, ms_split=self.ms_split,
                    ms_aggregate=self.ms_aggregate, ms_other=self.ms_other, ms_total=self.ms_total,
                    scanned_vertices=self.scanned_vertices, pruned=self.pruned,
                    confirm_sweeps=self.confirm_sweeps, sweeps=self.sweeps, split_rounds=self.split_rounds,
                    refine_iterations=list(self.refine_iterations[:k]), refined=list(self.refined[:k]),
                    ms_refine=self.ms_refine,
                    kernels={name: dict(launches=s.launches, ms=s.ms, bytes=s.bytes, items=s.items)
                             for name, s in zip(KERNEL_CLASSES, self.kernels)})


_lib = None


def lib():
    """The loaded libgsp.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                          "(the HIP library is required; there is no CPU path)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int
    sigs = {
        "gsp_default_options": [ctypes.POINTER(Options)],
        "gsp_create": [ctypes.c_int, vp, ctypes.POINTER(vp)],
        "gsp_destroy": [vp],
        "gsp_load_csr": [vp, i64, i64, vp, vp, vp, ctypes.c_int],
        "gsp_load_csr32": [vp, i32, i32, vp, vp, vp, ctypes.c_int],
        "gsp_load_csr_f64": [vp, i64, i64, vp, vp, vp, ctypes.c_int],
        "gsp_run": [vp, dbl, i32, ctypes.POINTER(Options)],
        "gsp_get_membership": [vp, vp, ctypes.c_int],
        "gsp_get_modularity": [vp, ctypes.POINTER(dbl)],
        "gsp_get_stats": [vp, ctypes.POINTER(Stats)],
        "gsp_modularity": [vp, vp, ctypes.c_int, ctypes.POINTER(dbl)],
        "gsp_count_disconnected": [vp, vp, ctypes.c_int, ctypes.POINTER(i64)],
        "gsp_step_move": [vp, vp, vp, ctypes.c_int, vp, vp, ctypes.POINTER(i64)],
        "gsp_move_phase": [vp, vp, ctypes.c_int, dbl, i32, i32, ctypes.POINTER(i32), vp, vp],
        "gsp_step_split": [vp, vp, ctypes.c_int, vp],
        "gsp_step_aggregate": [vp, vp, ctypes.c_int, ctypes.POINTER(i64), ctypes.POINTER(i64), vp, vp, vp],
        "gsp_move_phase_ex": [vp, vp, ctypes.c_int, dbl, i32, ctypes.POINTER(Options), ctypes.POINTER(i32), vp, vp,
                              vp],
        "gsp_pruner_set": [vp, vp, i64, ctypes.c_int],
        "gsp_gate_logits": [vp, vp, i64, vp, ctypes.c_int],
        "gsp_pruner_grad": [vp, vp, vp, vp, i64, ctypes.c_float, vp, ctypes.POINTER(dbl), ctypes.c_int],
        "gsp_pruner_train": [vp, vp, vp, i64, i64, i32, ctypes.c_float, ctypes.c_float, vp, vp, ctypes.c_int],
        "gsp_load_batch": [vp, i32, vp, vp, vp, vp, vp],
        "gsp_run_batch": [vp, dbl, i32, ctypes.POINTER(Options)],
        "gsp_get_batch_membership": [vp, i32, vp, ctypes.c_int],
        "gsp_get_batch_modularity": [vp, vp],
        "gsp_get_batch_passes": [vp, vp],
        "gsp_capture_traces": [vp, i64, dbl, ctypes.c_uint64],
        "gsp_get_traces": [vp, vp, vp, vp, vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.c_int],
        "gsp_get_weight_grid": [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)],
        "gsp_count_disconnected_noalloc": [i64, i64, vp, vp, vp, vp, vp],
        "gsp_step_split_lp": [vp, vp, ctypes.c_int, vp, ctypes.POINTER(i32)],
        "gsp_refine_phase": [vp, vp, vp, ctypes.c_int, dbl, ctypes.POINTER(Options), ctypes.POINTER(i32), vp, vp],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    L.gsp_last_error.argtypes = [vp]
    L.gsp_last_error.restype = ctypes.c_char_p
    L.gsp_noalloc_max_vertices.argtypes = []
    L.gsp_noalloc_max_vertices.restype = i64
    _lib = L
    return L


def count_disconnected_noalloc(offsets, cols, membership, out, stream=None) -> None:
    """gsp_count_disconnected_noalloc on torch device tensors (int64
    offsets, int32 cols and membership, one-element int64 out); enqueued on
    `stream` (a torch stream, default: the current one), no allocation."""
    import torch
    n = int(membership.numel())
    st = stream if stream is not None else torch.cuda.current_stream()
    for t, dt in ((offsets, torch.int64), (cols, torch.int32), (membership, torch.int32), (out, torch.int64)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError("device tensors: int64 offsets, int32 cols and membership, int64 out")
    if offsets.numel() != n + 1 or out.numel() < 1:
        raise ValueError("offsets must hold n + 1 values and out one")
    status = lib().gsp_count_disconnected_noalloc(n, int(cols.numel()), offsets.data_ptr(), cols.data_ptr(),
                                                  membership.data_ptr(), out.data_ptr(),
                                                  ctypes.c_void_p(st.cuda_stream))
    if status != GSP_OK:
        raise GspError(status, "gsp_count_disconnected_noalloc failed")


def default_options(**kw) -> Options:
    o = Options()
    lib().gsp_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, where, keepalive) for a numpy array or torch tensor."""
    if x is None:
        return None, HOST, None
    if _is_torch(x):
        import torch
        want = {np.int32: torch.int32, np.int64: torch.int64, np.float32: torch.float32,
                np.float64: torch.float64, np.uint8: torch.uint8}[dtype]
        if x.dtype != want:
            raise TypeError(f"expected a {want} tensor, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr(), (DEVICE if x.is_cuda else HOST), x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data, HOST, a


@dataclass
class RunResult:
    membership: np.ndarray
    modularity: float
    stats: dict


class Context:
    """One library context on one GPU (owns every device buffer it uses)."""

    def __init__(self, device: int = 0, stream=None):
        self._h = ctypes.c_void_p()
        s = None
        if stream is not None:
            s = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        self._check(lib().gsp_create(device, s, ctypes.byref(self._h)), "gsp_create")
        self.n = 0
        self.nnz = 0

    def close(self):
        if self._h:
            lib().gsp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, status: int, what: str):
        if status != GSP_OK:
            msg = lib().gsp_last_error(self._h) if self._h else b""
            raise GspError(status, f"{what}: {(msg or b'').decode()}")

    def last_error(self) -> str:
        return lib().gsp_last_error(self._h).decode()

    # ---------------------------------------------------------------- graph
    def load(self, offsets, cols, weights=None, n: Optional[int] = None) -> None:
        """Loads a symmetric CSR (int64 or int32 offsets; fp32/fp64/None weights)."""
        n = int((offsets.shape[0] if hasattr(offsets, "shape") else len(offsets)) - 1) if n is None else n
        nnz = int(cols.shape[0])
        off_dtype = np.int32 if str(getattr(offsets, "dtype", "")) in ("int32", "torch.int32") else np.int64
        po, wo, k1 = _ptr(offsets, off_dtype)
        pc, wc, k2 = _ptr(cols, np.int32)
        wdt = None
        if weights is not None:
            wdt = np.float64 if str(weights.dtype) in ("float64", "torch.float64") else np.float32
        pw, ww, k3 = _ptr(weights, wdt) if weights is not None else (None, wo, None)
        if len({wo, wc, ww}) != 1:
            raise ValueError("offsets, cols and weights must all be on the host or all on the device")
        if off_dtype == np.int32:
            if wdt == np.float64:
                raise TypeError("fp64 weights need int64 offsets")
            st = lib().gsp_load_csr32(self._h, n, nnz, po, pc, pw, wo)
        elif wdt == np.float64:
            st = lib().gsp_load_csr_f64(self._h, n, nnz, po, pc, pw, wo)
        else:
            st = lib().gsp_load_csr(self._h, n, nnz, po, pc, pw, wo)
        self._check(st, "gsp_load_csr")
        self.n, self.nnz = n, nnz

    def load_graph(self, g) -> None:
        """Loads a gsp_inputs.Graph (host arrays)."""
        self.load(g.offsets, g.cols, g.weights, n=g.n)

    # ------------------------------------------------------------------ run
    def run(self, tolerance: float = 1e-2, max_passes: int = 10, options: Optional[Options] = None,
            **kw) -> None:
        opt = options if options is not None else default_options(**kw)
        self._check(lib().gsp_run(self._h, tolerance, max_passes, ctypes.byref(opt)), "gsp_run")

    def membership(self, out=None):
        if out is None:
            out = np.empty(self.n, dtype=np.int32)
        p, w, _ = _ptr(out, np.int32)
        self._check(lib().gsp_get_membership(self._h, p, w), "gsp_get_membership")
        return out

    def result_modularity(self) -> float:
        q = ctypes.c_double()
        self._check(lib().gsp_get_modularity(self._h, ctypes.byref(q)), "gsp_get_modularity")
        return q.value

    def stats(self) -> dict:
        s = Stats()
        self._check(lib().gsp_get_stats(self._h, ctypes.byref(s)), "gsp_get_stats")
        return s.as_dict()

    def weight_grid(self):
        """(S, moved): the loaded weights are multiples of 2^-S; `moved` of
        them were rounded onto that grid at load."""
        S, mv = ctypes.c_int32(), ctypes.c_int64()
        self._check(lib().gsp_get_weight_grid(self._h, ctypes.byref(S), ctypes.byref(mv)), "gsp_get_weight_grid")
        return S.value, mv.value

    def louvain(self, tolerance: float = 1e-2, max_passes: int = 10, **kw) -> RunResult:
        self.run(tolerance, max_passes, **kw)
        return RunResult(self.membership(), self.result_modularity(), self.stats())

    # ---------------------------------------------------------- evaluation
    def modularity(self, membership) -> float:
        p, w, keep = _ptr(membership, np.int32)
        q = ctypes.c_double()
        self._check(lib().gsp_modularity(self._h, p, w, ctypes.byref(q)), "gsp_modularity")
        return q.value

    def count_disconnected(self, membership) -> int:
        p, w, keep = _ptr(membership, np.int32)
        c = ctypes.c_int64()
        self._check(lib().gsp_count_disconnected(self._h, p, w, ctypes.byref(c)), "gsp_count_disconnected")
        return c.value

    # --------------------------------------------------------------- hooks
    def step_move(self, membership, active=None):
        """One synchronous step; returns (dec, gain, moved)."""
        p, w, keep = _ptr(membership, np.int32)
        pa, wa, keep2 = _ptr(active, np.uint8)
        if active is not None and wa != w:
            raise ValueError("membership and active must live in the same place")
        dev = w == DEVICE
        if dev:
            import torch
            dec = torch.empty(self.n, dtype=torch.int32, device=membership.device)
            gain = torch.empty(self.n, dtype=torch.float64, device=membership.device)
        else:
            dec = np.empty(self.n, dtype=np.int32)
            gain = np.empty(self.n, dtype=np.float64)
        pd, _, _ = _ptr(dec, np.int32)
        pg, _, _ = _ptr(gain, np.float64)
        moved = ctypes.c_int64()
        self._check(lib().gsp_step_move(self._h, p, pa, w, pd, pg, ctypes.byref(moved)), "gsp_step_move")
        return dec, gain, moved.value

    def move_phase(self, membership=None, tolerance: float = 0.0, max_iterations: int = 20, sub_rounds: int = 8,
                   return_moves: int = 0):
        """The local-moving phase; returns (membership, l_i, dq per iteration, movers per iteration).
        return_moves = 1 goes through gsp_move_phase_ex with that option."""
        if return_moves:
            return self.move_phase_ex(membership, tolerance, max_iterations=max_iterations, sub_rounds=sub_rounds,
                                      return_moves=return_moves)[:4]
        m = np.arange(self.n, dtype=np.int32) if membership is None else np.array(membership, dtype=np.int32)
        li = ctypes.c_int32()
        dq = np.zeros(max(max_iterations, 1), dtype=np.float64)
        mv = np.zeros(max(max_iterations, 1), dtype=np.int64)
        self._check(lib().gsp_move_phase(self._h, m.ctypes.data, HOST, tolerance, max_iterations, sub_rounds,
                                         ctypes.byref(li), dq.ctypes.data, mv.ctypes.data), "gsp_move_phase")
        return m, li.value, dq[:li.value], mv[:li.value]

    def move_phase_ex(self, membership=None, tolerance: float = 0.0, pass_index: int = 0,
                      options: Optional[Options] = None, **kw):
        """The local-moving phase with the run's options (learned gate
        included); returns (membership, l_i, dq per counted iteration,
        movers per counted iteration, counters dict)."""
        opt = options if options is not None else default_options(**kw)
        m = np.arange(self.n, dtype=np.int32) if membership is None else np.array(membership, dtype=np.int32)
        li = ctypes.c_int32()
        mi = max(opt.max_iterations, 1)
        dq = np.zeros(mi, dtype=np.float64)
        mv = np.zeros(mi, dtype=np.int64)
        c4 = np.zeros(4, dtype=np.int64)
        self._check(lib().gsp_move_phase_ex(self._h, m.ctypes.data, HOST, tolerance, pass_index, ctypes.byref(opt),
                                            ctypes.byref(li), dq.ctypes.data, mv.ctypes.data, c4.ctypes.data),
                    "gsp_move_phase_ex")
        cnt = dict(scanned_vertices=int(c4[0]), scanned_entries=int(c4[1]), pruned=int(c4[2]),
                   confirm_sweeps=int(c4[3]))
        return m, li.value, dq[:li.value], mv[:li.value], cnt

    def refine_phase(self, bound, membership=None, tolerance: float = 0.0, options: Optional[Options] = None,
                     **kw):
        """GSP-Leiden's refinement within the communities `bound`, from
        `membership` (default: every vertex alone); returns (sub-community
        labels, iterations, dq per iteration, movers per iteration)."""
        opt = options if options is not None else default_options(**kw)
        b = np.ascontiguousarray(bound, dtype=np.int32)
        m = np.arange(self.n, dtype=np.int32) if membership is None else np.array(membership, dtype=np.int32)
        li = ctypes.c_int32()
        mi = max(opt.max_iterations, 1)
        dq = np.zeros(mi, dtype=np.float64)
        mv = np.zeros(mi, dtype=np.int64)
        self._check(lib().gsp_refine_phase(self._h, b.ctypes.data, m.ctypes.data, HOST, tolerance, ctypes.byref(opt),
                                           ctypes.byref(li), dq.ctypes.data, mv.ctypes.data), "gsp_refine_phase")
        return m, li.value, dq[:li.value], mv[:li.value]

    # -------------------------------------------------------------- batches
    def load_batch(self, graphs) -> None:
        """Loads a list of graphs (objects with n, offsets, cols, weights) as
        one batch."""
        G = len(graphs)
        keep = []
        n = np.array([g.n for g in graphs], dtype=np.int64)
        nnz = np.array([int(g.cols.shape[0]) for g in graphs], dtype=np.int64)
        offs = (ctypes.c_void_p * G)()
        cols = (ctypes.c_void_p * G)()
        any_w = any(g.weights is not None for g in graphs)
        ws = (ctypes.c_void_p * G)() if any_w else None
        for k, g in enumerate(graphs):
            o = np.ascontiguousarray(g.offsets, dtype=np.int64)
            c = np.ascontiguousarray(g.cols, dtype=np.int32)
            keep += [o, c]
            offs[k] = o.ctypes.data
            cols[k] = c.ctypes.data
            if any_w and g.weights is not None:
                w = np.ascontiguousarray(g.weights, dtype=np.float32)
                keep.append(w)
                ws[k] = w.ctypes.data
        self._check(lib().gsp_load_batch(self._h, G, n.ctypes.data, nnz.ctypes.data, offs, cols, ws),
                    "gsp_load_batch")
        self.batch_n = [int(x) for x in n]
        self.n = int(n.sum())
        self.nnz = int(nnz.sum())

    def run_batch(self, tolerance: float = 1e-2, max_passes: int = 10, options: Optional[Options] = None,
                  **kw) -> None:
        opt = options if options is not None else default_options(**kw)
        self._check(lib().gsp_run_batch(self._h, tolerance, max_passes, ctypes.byref(opt)), "gsp_run_batch")

    def batch_membership(self, k: int) -> np.ndarray:
        out = np.empty(self.batch_n[k], dtype=np.int32)
        self._check(lib().gsp_get_batch_membership(self._h, k, out.ctypes.data, HOST), "gsp_get_batch_membership")
        return out

    def batch_modularity(self) -> np.ndarray:
        q = np.empty(len(self.batch_n), dtype=np.float64)
        self._check(lib().gsp_get_batch_modularity(self._h, q.ctypes.data), "gsp_get_batch_modularity")
        return q

    def batch_passes(self) -> np.ndarray:
        p = np.empty(len(self.batch_n), dtype=np.int32)
        self._check(lib().gsp_get_batch_passes(self._h, p.ctypes.data), "gsp_get_batch_passes")
        return p

    # ---------------------------------------------------- learned pruning
    def pruner_set(self, params) -> None:
        """Sets the gate's network (4801 fp32 parameters, see gsp.h)."""
        p, w, keep = _ptr(params, np.float32)
        self._check(lib().gsp_pruner_set(self._h, p, GATE_PARAMS, w), "gsp_pruner_set")

    def gate_logits(self, x) -> np.ndarray:
        """Logits of feature rows x[rows][8] by the inference kernel."""
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 8)
        out = np.empty(x.shape[0], dtype=np.float32)
        self._check(lib().gsp_gate_logits(self._h, x.ctypes.data, x.shape[0], out.ctypes.data, HOST),
                    "gsp_gate_logits")
        return out

    def pruner_grad(self, params, x, y, pos_weight: float = 1.0):
        """(loss, gradient[4801]) of the mean pos-weighted BCE, by the fp32
        training kernels."""
        p = np.ascontiguousarray(params, dtype=np.float32)
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 8)
        y = np.ascontiguousarray(y, dtype=np.uint8)
        g = np.empty(GATE_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        self._check(lib().gsp_pruner_grad(self._h, p.ctypes.data, x.ctypes.data, y.ctypes.data, x.shape[0],
                                          pos_weight, g.ctypes.data, ctypes.byref(loss), HOST), "gsp_pruner_grad")
        return loss.value, g

    def pruner_train(self, params, x, y, batch: int, epochs: int, lr: float, pos_weight: float = 1.0):
        """Adam training on the GPU; returns (params fp32, per-epoch loss).
        x, y may be numpy arrays or device tensors (float32 [rows, 8], uint8)."""
        p = np.array(params, dtype=np.float32)
        px, wx, kx = _ptr(x, np.float32)
        py, wy, ky = _ptr(y, np.uint8)
        if wx != wy:
            raise ValueError("x and y must live in the same place")
        rows = int(y.shape[0])
        el = np.zeros(max(epochs, 1), dtype=np.float64)
        self._check(lib().gsp_pruner_train(self._h, px, py, rows, batch, epochs, lr, pos_weight, p.ctypes.data,
                                           el.ctypes.data, wx), "gsp_pruner_train")
        return p, el[:epochs]

    def capture_traces(self, capacity: int, rate: float = 1.0, seed: int = 0) -> None:
        """Starts (capacity > 0, clearing earlier rows) or stops (0) recording
        sampled scans of later runs."""
        self._check(lib().gsp_capture_traces(self._h, capacity, rate, seed), "gsp_capture_traces")

    def traces(self, max_rows: Optional[int] = None):
        """(x float32[rows, 8], moved uint8, vertex int32, meta int32, seen)."""
        rows, seen = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().gsp_get_traces(self._h, None, None, None, None, 0, ctypes.byref(rows),
                                         ctypes.byref(seen), HOST), "gsp_get_traces")
        k = rows.value if max_rows is None else min(rows.value, max_rows)
        x = np.empty((k, 8), dtype=np.float32)
        y = np.empty(k, dtype=np.uint8)
        v = np.empty(k, dtype=np.int32)
        m = np.empty(k, dtype=np.int32)
        self._check(lib().gsp_get_traces(self._h, x.ctypes.data, y.ctypes.data, v.ctypes.data, m.ctypes.data, k,
                                         ctypes.byref(rows), ctypes.byref(seen), HOST), "gsp_get_traces")
        return x[:rows.value], y[:rows.value], v[:rows.value], m[:rows.value], seen.value

    def step_split(self, membership):
        p, w, keep = _ptr(membership, np.int32)
        out = np.empty(self.n, dtype=np.int32)
        if w == DEVICE:
            import torch
            out = torch.empty(self.n, dtype=torch.int32, device=membership.device)
        po, _, _ = _ptr(out, np.int32)
        self._check(lib().gsp_step_split(self._h, p, w, po), "gsp_step_split")
        return out

    def step_split_lp(self, membership):
        """The split by label propagation; returns (labels, rounds)."""
        p, w, keep = _ptr(membership, np.int32)
        lab = np.empty(self.n, dtype=np.int32)
        r = ctypes.c_int32()
        self._check(lib().gsp_step_split_lp(self._h, p, w, lab.ctypes.data, ctypes.byref(r)), "gsp_step_split_lp")
        return lab, r.value

    def step_aggregate(self, membership):
        """Returns (n2, offsets int64, cols int32, weights fp64) on the host."""
        p, w, keep = _ptr(membership, np.int32)
        if w != HOST:
            raise ValueError("step_aggregate takes a host membership")
        n2, nnz2 = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().gsp_step_aggregate(self._h, p, w, ctypes.byref(n2), ctypes.byref(nnz2), None, None,
                                             None), "gsp_step_aggregate")
        off = np.empty(n2.value + 1, dtype=np.int64)
        col = np.empty(max(nnz2.value, 1), dtype=np.int32)
        wt = np.empty(max(nnz2.value, 1), dtype=np.float64)
        self._check(lib().gsp_step_aggregate(self._h, p, w, ctypes.byref(n2), ctypes.byref(nnz2), off.ctypes.data,
                                             col.ctypes.data, wt.ctypes.data), "gsp_step_aggregate")
        return n2.value, off, col[:nnz2.value], wt[:nnz2.value]
