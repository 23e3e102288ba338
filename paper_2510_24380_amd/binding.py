"""ctypes binding of libapex.so (include/apex.h). Argument marshalling only:
every step of the search runs in the library's HIP kernels. torch provides the
device memory (engine and query workspaces, tables, weights) and the stream.

Raises if the library is not built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libapex.so")

APEX_OK = 0
STATUS = {0: "APEX_OK", -1: "APEX_E_INVALID", -2: "APEX_E_NOMEM", -3: "APEX_E_DEVICE",
          -4: "APEX_E_UNSUPPORTED", -5: "APEX_E_PENDING", -6: "APEX_E_CANCELLED"}
ACT = {"none": 0, "relu": 1, "silu": 2}
APEX_QUERY_KEEP_VIOLATORS = 1
PREC = {"fp32": 0, "bf16": 1, "fp8": 2}

P = ctypes.c_void_p
U32 = ctypes.c_uint32
U64 = ctypes.c_uint64


class ApexError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class LibraryDesc(ctypes.Structure):
    _fields_ = [("n_reactions", U32), ("n_slots", P), ("slot_sizes", P), ("d", U32), ("tables", P)]


class DecoderDesc(ctypes.Structure):
    _fields_ = [("n_layers", U32), ("dims", P), ("act", U32), ("W", P), ("b", P)]


class ConstraintC(ctypes.Structure):
    _fields_ = [("head", U32), ("lo", ctypes.c_float), ("hi", ctypes.c_float)]


class QueryC(ctypes.Structure):
    _fields_ = [("objective_w", P), ("n_constraints", U32), ("constraints", P), ("k", U64),
                ("precision", U32), ("pool_factor", U32), ("n_subset", U32), ("subset", P), ("flags", U32)]


class ResultC(ctypes.Structure):
    _fields_ = [("capacity", U64), ("ids", P), ("objective", P), ("heads", P), ("reaction", P),
                ("synthon", P), ("n_found", U64), ("n_scored", U64), ("n_candidates", U64),
                ("n_reruns", U32), ("violation", P)]


class ServerConfigC(ctypes.Structure):
    _fields_ = [("pool", P), ("pool_bytes", ctypes.c_size_t), ("max_active", U32), ("stream", P),
                ("chunk_compounds", U64)]


class ServerStatsC(ctypes.Structure):
    _fields_ = [("submitted", U64), ("completed", U64), ("cancelled", U64), ("failed", U64),
                ("active", U64), ("waiting", U64), ("p50_latency_ms", ctypes.c_double),
                ("p99_latency_ms", ctypes.c_double), ("max_latency_ms", ctypes.c_double),
                ("compounds_per_s", ctypes.c_double), ("compounds_scored", U64)]


_lib = None

_SIGS = {
    "apex_library_create": [P, P],
    "apex_library_destroy": [P],
    "apex_library_num_compounds": [P, P],
    "apex_assoc_workspace_size": [P, P],
    "apex_assoc_embeddings": [P, U32, P, P, P, P, ctypes.c_size_t, P],
    "apex_decode_ids": [P, P, ctypes.c_size_t, P, P],
    "apex_decoder_create": [P, P],
    "apex_decoder_destroy": [P],
    "apex_engine_workspace_size": [P, P, U32, P],
    "apex_engine_create": [P, P, U32, P, ctypes.c_size_t, P, P],
    "apex_engine_destroy": [P],
    "apex_query_workspace_size": [P, P, P],
    "apex_search": [P, P, P, ctypes.c_size_t, P, P],
    "apex_search_noalloc": [P, P, P, P],
    "apex_batch_workspace_size": [P, P, U32, P],
    "apex_search_batch": [P, P, U32, P, ctypes.c_size_t, P, P],
    "apex_engine_profile": [P, ctypes.c_int, P, P, P],
    "apex_engine_heads": [P, P, U32, U32, P, P],
    "apex_engine_head_quantiles": [P, P, U32, P, U32, P, P],
    "apex_server_create": [P, P, P],
    "apex_server_submit": [P, P, P],
    "apex_server_poll": [P, U64, P, ctypes.c_int],
    "apex_server_cancel": [P, U64],
    "apex_server_stats_get": [P, P],
    "apex_server_destroy": [P],
}


def lib() -> ctypes.CDLL:
    """The loaded library; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(f"{SO_PATH} is missing: build it with paper_2510_24380_amd.build.build()")
        L = ctypes.CDLL(SO_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.apex_status_string.argtypes = [ctypes.c_int]
        L.apex_status_string.restype = ctypes.c_char_p
        L.apex_last_error.argtypes = []
        L.apex_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != APEX_OK:
        raise ApexError(status, lib().apex_last_error().decode())


def _stream_ptr(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_ptr(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return int(t.data_ptr())


class Library:
    """Reactions, slot sizes and the FP32 synthon table (device, rows in
    (reaction, slot, synthon) order). Keeps the table tensor alive."""

    def __init__(self, n_slots: Sequence[int], slot_sizes: Sequence[int], tables: torch.Tensor):
        if tables.dtype != torch.float32 or tables.dim() != 2 or not tables.is_contiguous():
            raise ValueError("tables must be a contiguous 2-D float32 tensor")
        self.tables = tables
        self._ns = np.ascontiguousarray(n_slots, dtype=np.uint32)
        self._ss = np.ascontiguousarray(slot_sizes, dtype=np.uint32)
        desc = LibraryDesc(len(self._ns), self._ns.ctypes.data, self._ss.ctypes.data, tables.shape[1],
                           _dev_ptr(tables))
        h = P()
        _check(lib().apex_library_create(ctypes.byref(desc), ctypes.byref(h)))
        self.handle = h
        self.n_reactions = len(self._ns)

    @property
    def num_compounds(self) -> int:
        n = U64()
        _check(lib().apex_library_num_compounds(self.handle, ctypes.byref(n)))
        return int(n.value)

    def assoc_embeddings(self, keys: torch.Tensor, values: torch.Tensor, out: Optional[torch.Tensor] = None,
                         stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """u_{r,s} = K_r v_s for every table row (apex_assoc_embeddings): keys
        [n_slots_total, d, dU], values [rows, dU] (device FP32). Writes `out`
        (default: this library's own tables) and returns it."""
        for t in (keys, values):
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("keys and values must be contiguous float32 device tensors")
        out = self.tables if out is None else out
        n = ctypes.c_size_t()
        _check(lib().apex_assoc_workspace_size(self.handle, ctypes.byref(n)))
        ws = torch.empty(max(int(n.value), 256), dtype=torch.uint8, device=keys.device)
        _check(lib().apex_assoc_embeddings(self.handle, int(keys.shape[2]), keys.data_ptr(), values.data_ptr(),
                                           out.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
        return out

    def decode(self, ids):
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        r = np.zeros(max(ids.size, 1), np.uint32)
        s = np.zeros((max(ids.size, 1), 3), np.uint32)
        _check(lib().apex_decode_ids(self.handle, ids.ctypes.data, ids.size, r.ctypes.data, s.ctypes.data))
        return r[:ids.size], s[:ids.size]

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.apex_library_destroy(self.handle)
            self.handle = None


class Decoder:
    """Decoder weights (device FP32): W[l] is dims[l+1] x dims[l]."""

    def __init__(self, dims: Sequence[int], act: str, W: Sequence[torch.Tensor], b: Sequence[torch.Tensor]):
        self.W = [w.contiguous() for w in W]
        self.b = [x.contiguous() for x in b]
        self._dims = np.ascontiguousarray(dims, dtype=np.uint32)
        self._wp = (ctypes.c_void_p * len(self.W))(*[_dev_ptr(w) for w in self.W])
        self._bp = (ctypes.c_void_p * len(self.b))(*[_dev_ptr(x) for x in self.b])
        desc = DecoderDesc(len(self.W), self._dims.ctypes.data, ACT[act] if isinstance(act, str) else int(act),
                           ctypes.cast(self._wp, P), ctypes.cast(self._bp, P))
        h = P()
        _check(lib().apex_decoder_create(ctypes.byref(desc), ctypes.byref(h)))
        self.handle = h
        self.dims = [int(x) for x in dims]

    @property
    def n_heads(self) -> int:
        return self.dims[-1]

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.apex_decoder_destroy(self.handle)
            self.handle = None


@dataclasses.dataclass
class SearchResult:
    ids: np.ndarray
    objective: np.ndarray
    heads: np.ndarray
    reaction: np.ndarray
    synthon: np.ndarray
    n_scored: int
    n_candidates: int
    n_reruns: int
    violation: Optional[np.ndarray] = None  # c(x) per entry (keep-violators queries)


class _QueryMarshal:
    """Keeps the ctypes arrays of one query alive."""

    def __init__(self, q, n_heads: int, precision: str, pool_factor: int):
        w = np.zeros(n_heads, np.float32)
        w[:len(q.w)] = np.asarray(q.w, np.float32)[:n_heads]
        self.w = w
        cons = list(q.constraints)
        self.cons = (ConstraintC * max(len(cons), 1))()
        for i, c in enumerate(cons):
            lo = -math.inf if c.lo is None else float(c.lo)
            hi = math.inf if c.hi is None else float(c.hi)
            self.cons[i] = ConstraintC(int(c.head), lo, hi)
        subset = getattr(q, "reactions", None)
        self.subset = np.ascontiguousarray(list(subset) if subset is not None else [0], dtype=np.uint32)
        flags = APEX_QUERY_KEEP_VIOLATORS if getattr(q, "keep_violators", False) else 0
        self.c = QueryC(self.w.ctypes.data, len(cons), ctypes.cast(self.cons, P), int(q.k), PREC[precision],
                        int(pool_factor), len(subset) if subset is not None else 0,
                        self.subset.ctypes.data if subset is not None else None, flags)


class ResultBuffers:
    """Result arrays for answers of up to `capacity` entries, in pinned host
    memory, for reuse across searches (`Engine.search(..., out=buffers)`): the
    library copies long answers into them straight from the device, and no
    fresh host memory is touched per search. A result returned through them
    views these arrays and is overwritten by the next search that uses them."""

    def __init__(self, capacity: int, n_heads: int):
        def pinned(shape, dtype):
            return torch.empty(shape, dtype=dtype, pin_memory=True)
        self.capacity = int(capacity)
        self.n_heads = int(n_heads)
        # torch has no unsigned 64/32-bit dtypes for pinned tensors: int64/int32
        # storage viewed as uint64/uint32
        self._t = [pinned((capacity,), torch.int64), pinned((capacity,), torch.float32),
                   pinned((capacity, n_heads), torch.float32), pinned((capacity,), torch.int32),
                   pinned((capacity, 3), torch.int32), pinned((capacity,), torch.float32)]
        self.ids = self._t[0].numpy().view(np.uint64)
        self.obj = self._t[1].numpy()
        self.heads = self._t[2].numpy()
        self.reaction = self._t[3].numpy().view(np.uint32)
        self.synthon = self._t[4].numpy().view(np.uint32)
        self.viol = self._t[5].numpy()


class _ResultMarshal:
    def __init__(self, k: int, n_heads: int, out: Optional[ResultBuffers] = None):
        if out is not None:
            if out.capacity < k or out.n_heads != n_heads:
                raise ValueError(f"result buffers hold {out.capacity} x {out.n_heads} heads, "
                                 f"the query needs {k} x {n_heads}")
            self.ids, self.obj, self.heads = out.ids, out.obj, out.heads
            self.reaction, self.synthon, self.viol = out.reaction, out.synthon, out.viol
        else:
            self.ids = np.empty(k, np.uint64)
            self.obj = np.empty(k, np.float32)
            self.heads = np.empty((k, n_heads), np.float32)
            self.reaction = np.empty(k, np.uint32)
            self.synthon = np.empty((k, 3), np.uint32)
            self.viol = np.empty(k, np.float32)
        self.c = ResultC(k, self.ids.ctypes.data, self.obj.ctypes.data, self.heads.ctypes.data,
                         self.reaction.ctypes.data, self.synthon.ctypes.data, 0, 0, 0, 0, self.viol.ctypes.data)

    def result(self) -> SearchResult:
        # the arrays belong to this one result: views, no copies
        n = int(self.c.n_found)
        return SearchResult(self.ids[:n], self.obj[:n], self.heads[:n], self.reaction[:n], self.synthon[:n],
                            int(self.c.n_scored), int(self.c.n_candidates), int(self.c.n_reruns), self.viol[:n])


class Engine:
    """Resident hoisted tables and decoder layouts for one (library, decoder)."""

    def __init__(self, library: Library, decoder: Decoder, precisions=("fp32", "bf16", "fp8"),
                 stream: Optional[torch.cuda.Stream] = None):
        mask = 0
        for p in precisions:
            mask |= 1 << PREC[p]
        n = ctypes.c_size_t()
        _check(lib().apex_engine_workspace_size(library.handle, decoder.handle, mask, ctypes.byref(n)))
        self.workspace = torch.empty(max(int(n.value), 256), dtype=torch.uint8, device="cuda")
        h = P()
        _check(lib().apex_engine_create(library.handle, decoder.handle, mask, self.workspace.data_ptr(),
                                        self.workspace.numel(), _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        self.library = library
        self.decoder = decoder
        self.n_heads = decoder.n_heads
        self._qws = None

    def _workspace(self, nbytes: int) -> torch.Tensor:
        if self._qws is None or self._qws.numel() < nbytes:
            self._qws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
        return self._qws

    def query_workspace_size(self, q, precision="fp32", pool_factor=0) -> int:
        m = _QueryMarshal(q, self.n_heads, precision, pool_factor)
        n = ctypes.c_size_t()
        _check(lib().apex_query_workspace_size(self.handle, ctypes.byref(m.c), ctypes.byref(n)))
        return int(n.value)

    def search(self, q, precision: str = "fp32", pool_factor: int = 0,
               stream: Optional[torch.cuda.Stream] = None, out: Optional[ResultBuffers] = None) -> SearchResult:
        """One query. With `out`, the result views those reusable pinned arrays
        (see ResultBuffers); otherwise it owns freshly allocated ones."""
        return self.search_batch([q], precision, pool_factor, stream, outs=None if out is None else [out])[0]

    def search_batch(self, qs, precision: str = "fp32", pool_factor: int = 0,
                     stream: Optional[torch.cuda.Stream] = None,
                     outs: Optional[List[ResultBuffers]] = None) -> List[SearchResult]:
        ms = [_QueryMarshal(q, self.n_heads, precision, pool_factor) for q in qs]
        arr = (QueryC * len(ms))(*[m.c for m in ms])
        n = ctypes.c_size_t()
        _check(lib().apex_batch_workspace_size(self.handle, arr, len(ms), ctypes.byref(n)))
        ws = self._workspace(int(n.value))
        rs = [_ResultMarshal(int(q.k), self.n_heads, None if outs is None else outs[i]) for i, q in enumerate(qs)]
        rarr = (ResultC * len(rs))(*[r.c for r in rs])
        if len(ms) == 1:
            st = lib().apex_search(self.handle, arr, ws.data_ptr(), ws.numel(), _stream_ptr(stream), rarr)
        else:
            st = lib().apex_search_batch(self.handle, arr, len(ms), ws.data_ptr(), ws.numel(),
                                         _stream_ptr(stream), rarr)
        _check(st)
        out = []
        for r, rc in zip(rs, rarr):
            r.c = rc
            out.append(r.result())
        return out

    def search_noalloc(self, q, precision: str = "fp32", pool_factor: int = 0,
                       stream: Optional[torch.cuda.Stream] = None) -> SearchResult:
        """apex_search_noalloc: the same search with the library's static device
        scratch instead of a workspace (nothing is allocated by the call)."""
        m = _QueryMarshal(q, self.n_heads, precision, pool_factor)
        r = _ResultMarshal(int(q.k), self.n_heads)
        _check(lib().apex_search_noalloc(self.handle, ctypes.byref(m.c), _stream_ptr(stream), ctypes.byref(r.c)))
        return r.result()

    def heads(self, ids, precision: str = "fp32", stream: Optional[torch.cuda.Stream] = None) -> np.ndarray:
        """Heads of the listed compounds in one precision's enumeration arithmetic."""
        ids_d = torch.from_numpy(np.ascontiguousarray(ids, dtype=np.int64)).cuda()
        stride = 16 if self.n_heads <= 16 else 32  # row stride of apex_engine_heads
        out = torch.empty((max(len(ids), 1), stride), dtype=torch.float32, device="cuda")
        _check(lib().apex_engine_heads(self.handle, ids_d.data_ptr(), len(ids), PREC[precision], out.data_ptr(),
                                       _stream_ptr(stream)))
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        return out[:len(ids), :self.n_heads].cpu().numpy()

    def head_quantiles(self, levels, n: int = 8192, ids=None,
                       stream: Optional[torch.cuda.Stream] = None) -> np.ndarray:
        """[len(levels), H] quantiles of the FP32 heads over n compounds drawn by
        the engine (or the listed ids): percentile thresholds for queries."""
        lv = np.ascontiguousarray(levels, dtype=np.float32)
        out = np.empty((lv.size, self.n_heads), np.float32)
        ids_d = None
        if ids is not None:
            ids_d = torch.from_numpy(np.ascontiguousarray(ids, dtype=np.int64)).cuda()
            n = len(ids)
        _check(lib().apex_engine_head_quantiles(self.handle, ids_d.data_ptr() if ids_d is not None else None, int(n),
                                                lv.ctypes.data, lv.size, out.ctypes.data, _stream_ptr(stream)))
        return out

    def profile(self, enable: bool):
        """Returns (ms, launches, compounds) timed since the last call, then
        switches timing of the fused kernel on or off."""
        ms = ctypes.c_double()
        nl = U64()
        nc = U64()
        _check(lib().apex_engine_profile(self.handle, int(enable), ctypes.byref(ms), ctypes.byref(nl),
                                         ctypes.byref(nc)))
        return float(ms.value), int(nl.value), int(nc.value)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.apex_engine_destroy(self.handle)
            self.handle = None


class Server:
    """Continuous-batching server over one engine (apex_server_*): a library
    thread admits queries by workspace memory and fuses those that are active
    into chunk-by-chunk passes. The pool is device memory owned by this object."""

    def __init__(self, engine: Engine, pool_bytes: int, max_active: int = 8, chunk_compounds: int = 0,
                 stream: Optional[torch.cuda.Stream] = None):
        self.engine = engine
        self.pool = torch.empty(max(int(pool_bytes), 256), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        cfg = ServerConfigC(self.pool.data_ptr(), self.pool.numel(), int(max_active), int(self.stream.cuda_stream),
                            int(chunk_compounds))
        h = P()
        _check(lib().apex_server_create(engine.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._k = {}

    def submit(self, q, precision: str = "fp32", pool_factor: int = 0) -> int:
        m = _QueryMarshal(q, self.engine.n_heads, precision, pool_factor)
        t = U64()
        _check(lib().apex_server_submit(self.handle, ctypes.byref(m.c), ctypes.byref(t)))
        self._k[int(t.value)] = int(q.k)
        return int(t.value)

    def poll(self, ticket: int, timeout_ms: int = -1) -> Optional[SearchResult]:
        """The result, or None while the query is still pending."""
        r = _ResultMarshal(self._k[ticket], self.engine.n_heads)
        st = lib().apex_server_poll(self.handle, ticket, ctypes.byref(r.c), int(timeout_ms))
        if st == -5:
            return None
        self._k.pop(ticket, None)
        _check(st)
        return r.result()

    def cancel(self, ticket: int) -> None:
        _check(lib().apex_server_cancel(self.handle, ticket))

    def stats(self) -> dict:
        s = ServerStatsC()
        _check(lib().apex_server_stats_get(self.handle, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in ServerStatsC._fields_}

    def close(self) -> None:
        if getattr(self, "handle", None) and _lib is not None:
            _lib.apex_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()
