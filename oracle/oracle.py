"""ctypes front end of the FP64 C oracle (apex_oracle.c).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU-baseline
leg call it. It shares no code with the HIP library.

Semantics (see apex_oracle.c for the paper passages): the compound embedding is
the sum of its per-slot table rows (eq. "factorizer"); heads come from the
decoder applied to that sum (eq. "surrogate", generalised to an MLP); the query
keeps the k best feasible compounds by w . heads, bounds inclusive, ties by
lower id (eq. "apex_topk").
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import List, Optional

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_DIR, "liboracle.so")
_lib = None


def build() -> str:
    src = os.path.join(_DIR, "apex_oracle.c")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           src, "-o", _SO, "-lm"])
    return _SO


class _Lib(ctypes.Structure):
    _fields_ = [("n_reactions", ctypes.c_uint32), ("n_slots", ctypes.c_void_p),
                ("slot_sizes", ctypes.c_void_p), ("d", ctypes.c_uint32), ("tables", ctypes.c_void_p)]


class _Dec(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_uint32), ("dims", ctypes.c_void_p), ("act", ctypes.c_uint32),
                ("W", ctypes.c_void_p), ("b", ctypes.c_void_p)]


class _Query(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("n_con", ctypes.c_uint32), ("con_head", ctypes.c_void_p),
                ("con_lo", ctypes.c_void_p), ("con_hi", ctypes.c_void_p), ("k", ctypes.c_uint64),
                ("subset", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [("n_feasible", ctypes.c_uint64), ("n_out", ctypes.c_uint64),
                ("min_slack_selected", ctypes.c_double), ("min_violation_near", ctypes.c_double),
                ("n_near", ctypes.c_uint64)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        lib.orc_num_compounds.argtypes = [P]
        lib.orc_num_compounds.restype = ctypes.c_uint64
        lib.orc_decode.argtypes = [P, P, ctypes.c_uint64, P, P]
        lib.orc_decode.restype = ctypes.c_int
        lib.orc_heads.argtypes = [P, P, P, ctypes.c_uint64, P]
        lib.orc_heads.restype = ctypes.c_int
        lib.orc_topk.argtypes = [P, P, P, ctypes.c_int, ctypes.c_uint64, ctypes.c_double, P, P, P, P]
        lib.orc_topk.restype = ctypes.c_int
        lib.orc_topk_lex.argtypes = [P, P, P, ctypes.c_int, P, P, P, P]
        lib.orc_topk_lex.restype = ctypes.c_int
        lib.orc_assoc_embeddings.argtypes = [ctypes.c_uint32, P, P, ctypes.c_uint32, ctypes.c_uint32, P, P, P]
        lib.orc_assoc_embeddings.restype = ctypes.c_int
        lib.orc_max_threads.argtypes = []
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


class _Keep:
    """Holds numpy buffers alive while ctypes structs point into them."""

    def __init__(self):
        self.bufs = []

    def ptr(self, a: np.ndarray) -> int:
        self.bufs.append(a)
        return a.ctypes.data


def _lib_struct(lib, keep: _Keep) -> _Lib:
    ns = np.ascontiguousarray(lib.n_slots, dtype=np.uint32)
    ss = np.ascontiguousarray(lib.slot_sizes, dtype=np.uint32)
    tb = np.ascontiguousarray(lib.tables, dtype=np.float32)
    return _Lib(len(ns), keep.ptr(ns), keep.ptr(ss), int(lib.d), keep.ptr(tb))


def _dec_struct(dec, keep: _Keep) -> _Dec:
    dims = np.asarray(dec.dims, dtype=np.uint32)
    Ws = [np.ascontiguousarray(w, dtype=np.float32) for w in dec.W]
    bs = [np.ascontiguousarray(b, dtype=np.float32) for b in dec.b]
    wp = np.array([keep.ptr(w) for w in Ws], dtype=np.uint64)
    bp = np.array([keep.ptr(b) for b in bs], dtype=np.uint64)
    return _Dec(len(Ws), keep.ptr(dims), int(dec.act), keep.ptr(wp), keep.ptr(bp))


def _query_struct(q, n_reactions: int, keep: _Keep) -> _Query:
    w = np.ascontiguousarray(q.w, dtype=np.float32)
    heads = np.array([c.head for c in q.constraints] or [0], dtype=np.uint32)
    lo = np.array([c.lo for c in q.constraints] or [0], dtype=np.float32)
    hi = np.array([c.hi for c in q.constraints] or [0], dtype=np.float32)
    subset = None
    if q.reactions is not None:
        m = np.zeros(n_reactions, dtype=np.uint8)
        m[np.asarray(list(q.reactions), dtype=np.int64)] = 1
        subset = keep.ptr(m)
    return _Query(keep.ptr(w), len(q.constraints), keep.ptr(heads), keep.ptr(lo), keep.ptr(hi),
                  int(q.k), subset)


def max_threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(_load().orc_max_threads())


def num_compounds(lib) -> int:
    keep = _Keep()
    L = _lib_struct(lib, keep)
    return int(_load().orc_num_compounds(ctypes.byref(L)))


def decode(lib, ids):
    """ids -> (reaction uint32 [n], synthon uint32 [n, 3])."""
    keep = _Keep()
    L = _lib_struct(lib, keep)
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    n = ids.size
    r = np.zeros(max(n, 1), dtype=np.uint32)
    s = np.zeros((max(n, 1), 3), dtype=np.uint32)
    rc = _load().orc_decode(ctypes.byref(L), ids.ctypes.data, n, r.ctypes.data, s.ctypes.data)
    if rc != 0:
        raise ValueError("compound id out of range")
    return r[:n], s[:n]


def heads(lib, dec, ids) -> np.ndarray:
    """FP64 heads of the given compounds, [n, H]."""
    keep = _Keep()
    L = _lib_struct(lib, keep)
    D = _dec_struct(dec, keep)
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    out = np.zeros((max(ids.size, 1), dec.n_heads), dtype=np.float64)
    rc = _load().orc_heads(ctypes.byref(L), ctypes.byref(D), ids.ctypes.data, ids.size, out.ctypes.data)
    if rc != 0:
        raise ValueError("compound id out of range")
    return out[:ids.size]


@dataclasses.dataclass
class TopK:
    ids: np.ndarray  # uint64 [n] (first min(k, n_feasible) are the answer)
    objective: np.ndarray  # float64 [n]
    heads: np.ndarray  # float64 [n, H]
    n_feasible: int
    k: int
    min_slack_selected: float
    min_violation_near: float
    n_near: int

    @property
    def answer_ids(self) -> np.ndarray:
        return self.ids[:min(self.k, len(self.ids))]

    @property
    def gap_k(self) -> float:
        """o_(k) - o_(k+1) among feasible compounds (inf if fewer than k+1)."""
        if len(self.objective) <= self.k:
            return math.inf
        return float(self.objective[self.k - 1] - self.objective[self.k])


def topk(lib, dec, q, extra: int = 1, near_tol: float = 0.0, nthreads: int = 0) -> TopK:
    keep = _Keep()
    L = _lib_struct(lib, keep)
    D = _dec_struct(dec, keep)
    Q = _query_struct(q, len(lib.n_slots), keep)
    cap = int(q.k) + int(extra)
    ids = np.zeros(max(cap, 1), dtype=np.uint64)
    o = np.zeros(max(cap, 1), dtype=np.float64)
    h = np.zeros((max(cap, 1), dec.n_heads), dtype=np.float64)
    info = _Info()
    rc = _load().orc_topk(ctypes.byref(L), ctypes.byref(D), ctypes.byref(Q), int(nthreads), int(extra),
                          float(near_tol), ids.ctypes.data, o.ctypes.data, h.ctypes.data,
                          ctypes.byref(info))
    if rc != 0:
        raise ValueError("oracle rejected the inputs")
    n = int(info.n_out)
    return TopK(ids=ids[:n].copy(), objective=o[:n].copy(), heads=h[:n].copy(),
                n_feasible=int(info.n_feasible), k=int(q.k),
                min_slack_selected=float(info.min_slack_selected),
                min_violation_near=float(info.min_violation_near), n_near=int(info.n_near))


def topk_lex(lib, dec, q, keep_violators: bool = False, with_violation: bool = False):
    """The paper's lexicographic priority-queue form; returns (ids, objective),
    plus each entry's violation (<= 0) when with_violation. keep_violators
    returns the queue without the final removal of violating compounds (the
    violation-ranked fallback)."""
    keep = _Keep()
    L = _lib_struct(lib, keep)
    D = _dec_struct(dec, keep)
    Q = _query_struct(q, len(lib.n_slots), keep)
    ids = np.zeros(max(int(q.k), 1), dtype=np.uint64)
    o = np.zeros(max(int(q.k), 1), dtype=np.float64)
    c = np.zeros(max(int(q.k), 1), dtype=np.float64)
    n = ctypes.c_uint64(0)
    _load().orc_topk_lex(ctypes.byref(L), ctypes.byref(D), ctypes.byref(Q), int(bool(keep_violators)),
                         ids.ctypes.data, o.ctypes.data, c.ctypes.data, ctypes.byref(n))
    out = (ids[:n.value].copy(), o[:n.value].copy())
    return out + (c[:n.value].copy(),) if with_violation else out


def assoc_embeddings(n_slots, slot_sizes, keys, values) -> np.ndarray:
    """u_{r,s} = K_r v_s for every (reaction, slot, synthon) row, FP64
    (Section 4.2, eq. "assoc_embeds"). keys: [n_slot_total, d, dU] float32,
    values: [rows, dU] float32; returns [rows, d] float64."""
    ns = np.ascontiguousarray(n_slots, dtype=np.uint32)
    ss = np.ascontiguousarray(slot_sizes, dtype=np.uint32)
    K = np.ascontiguousarray(keys, dtype=np.float32)
    V = np.ascontiguousarray(values, dtype=np.float32)
    assert K.ndim == 3 and K.shape[0] == ss.size and V.shape == (int(ss.sum()), K.shape[2])
    out = np.zeros((V.shape[0], K.shape[1]), dtype=np.float64)
    _load().orc_assoc_embeddings(ns.size, ns.ctypes.data, ss.ctypes.data, K.shape[1], K.shape[2], K.ctypes.data,
                                 V.ctypes.data, out.ctypes.data)
    return out
