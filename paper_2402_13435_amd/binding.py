"""ctypes binding of the C ABI in include/fr.h (argument marshalling only).

Every step of retrieval runs in the HIP library ``libfr.so``; this module
only converts NumPy arrays / PyTorch device tensors to pointers and back.
There is no fallback: if the library is not built, or no GPU is present,
calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Any, Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfr.so")

FR_OK, FR_EINVAL, FR_ENOMEM, FR_ECAPACITY, FR_EDUPID = 0, -1, -2, -3, -4
FR_ENOTFOUND, FR_EUNSUPPORTED, FR_EDEVICE, FR_EBUSY = -5, -6, -7, -8
STATUS_NAMES = {0: "FR_OK", -1: "FR_EINVAL", -2: "FR_ENOMEM", -3: "FR_ECAPACITY",
                -4: "FR_EDUPID", -5: "FR_ENOTFOUND", -6: "FR_EUNSUPPORTED",
                -7: "FR_EDEVICE", -8: "FR_EBUSY"}
FR_DEVICE_PTRS, FR_NOWAIT, FR_GRAPH, FR_ASYNC, FR_PRESELECT = 1, 2, 4, 8, 16
FR_STRAT_NO_SPECULATION, FR_STRAT_NO_REFRESH = 1, 2


FR_STRAT_SPARSE_MASK = 0xF0


def FR_STRAT_SPARSE(level: int) -> int:
    """Sparse routing level 1..7 (see include/fr.h)."""
    return int(level) << 4
DTYPES = {"f32": 0, "bf16": 1, "fp8": 2}

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_f32p = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p


class FrConfig(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_uint64), ("dim", ctypes.c_uint32),
                ("vocab", ctypes.c_uint32), ("k_max", ctypes.c_uint32),
                ("rescore_r", ctypes.c_uint32), ("rescore_min", ctypes.c_uint32),
                ("dtype", ctypes.c_int), ("max_batch", ctypes.c_uint32),
                ("max_clauses", ctypes.c_uint32), ("max_literals", ctypes.c_uint32),
                ("n_workspaces", ctypes.c_uint32), ("cand_cap", ctypes.c_uint32),
                ("device", ctypes.c_int), ("quant_bits", ctypes.c_uint32),
                ("quant_factor", ctypes.c_uint32), ("list_terms", ctypes.c_uint32),
                ("batch_terms", ctypes.c_uint32)]


class FrCnfBatch(ctypes.Structure):
    _fields_ = [("n_queries", ctypes.c_uint32), ("clause_off", _u32p),
                ("literal_off", _u32p), ("terms", _u32p)]


class FrStats(ctypes.Structure):
    _fields_ = [("n_queries", ctypes.c_uint32), ("n_passes", ctypes.c_uint32),
                ("candidates", ctypes.c_uint64), ("n_live", ctypes.c_uint64),
                ("n_terms_batch", ctypes.c_uint64), ("alg_bytes", ctypes.c_double),
                ("alg_flops", ctypes.c_double), ("ms_scan", ctypes.c_float),
                ("ms_total", ctypes.c_float), ("n_sparse", ctypes.c_uint32),
                ("ms_call", ctypes.c_float)]


class FrServerConfig(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32),
                ("max_wait_us", ctypes.c_uint32)]


class FrServerStats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_uint64), ("queries", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("max_batch_seen", ctypes.c_uint32),
                ("pending", ctypes.c_uint32)]


class FrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


_LIB = None

SYMBOLS = {
    "fr_create": (ctypes.c_int, [ctypes.POINTER(FrConfig), ctypes.POINTER(_vp)]),
    "fr_destroy": (ctypes.c_int, [_vp]),
    "fr_load_corpus": (ctypes.c_int, [_vp, ctypes.c_uint64, _vp, _vp, _vp, _vp, ctypes.c_uint32]),
    "fr_update_docs": (ctypes.c_int, [_vp, ctypes.c_uint64, _vp, ctypes.c_uint64, _vp, _vp,
                                      _vp, _vp, _u64p]),
    "fr_search": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, ctypes.POINTER(FrCnfBatch), _vp,
                                 _vp, _vp, _vp, _vp, _vp, ctypes.c_uint32]),
    "fr_search_noalloc": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, ctypes.POINTER(FrCnfBatch),
                                         _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_uint32]),
    "fr_last_error": (ctypes.c_char_p, []),
    "fr_stats": (ctypes.c_int, [_vp, ctypes.POINTER(FrStats)]),
    "fr_info": (ctypes.c_int, [_vp, _u64p, _u64p, _u64p]),
    "fr_timings": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp, _u32p]),
    "fr_debug_masks": (ctypes.c_int, [_vp, ctypes.POINTER(FrCnfBatch), _vp, ctypes.c_uint64]),
    "fr_debug_rows": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_uint64, _vp, _vp]),
    "fr_debug_slots": (ctypes.c_int, [_vp, _vp, ctypes.c_uint64]),
    "fr_debug_candidates": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp, _vp]),
    "fr_set_tiling": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]),
    "fr_autotune": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, ctypes.POINTER(FrCnfBatch), _vp,
                                   ctypes.c_uint32, _u32p, _u32p, _u32p, _u32p]),
    "fr_set_strategy": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.c_int]),
    "fr_tuning_save": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "fr_tuning_choice": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _u32p, _u32p, _u32p, _u32p,
                                        _u32p]),
    "fr_tuning_load": (ctypes.c_int, [_vp, ctypes.c_char_p, _u32p]),
    "fr_set_quantizer": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "fr_debug_codes": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_uint64, _vp]),
    "fr_server_create": (ctypes.c_int, [_vp, ctypes.POINTER(FrServerConfig),
                                        ctypes.POINTER(_vp)]),
    "fr_server_submit": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, ctypes.POINTER(FrCnfBatch),
                                        _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _u64p]),
    "fr_server_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_uint32]),
    "fr_server_get_stats": (ctypes.c_int, [_vp, ctypes.POINTER(FrServerStats)]),
    "fr_server_destroy": (ctypes.c_int, [_vp]),
    "fr_clock_ns": (ctypes.c_uint64, []),
}


def lib() -> ctypes.CDLL:
    """Load libfr.so (raises if it is not built)."""
    global _LIB
    if _LIB is None:
        # Use the HIP runtime PyTorch ships when PyTorch is present: loading it
        # first makes libfr.so bind to that same runtime (one runtime per
        # process, so device pointers and streams are shared).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (python -m paper_2402_13435_amd.build)")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SYMBOLS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _LIB = h
    return _LIB


def _check(status: int) -> None:
    if status != FR_OK:
        raise FrError(status, lib().fr_last_error().decode(errors="replace"))


def _is_dev(x: Any) -> bool:
    return hasattr(x, "data_ptr") and getattr(x, "is_cuda", False)


def _host(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if _is_dev(a):
        return a.data_ptr()
    return a.ctypes.data


class Cnf:
    """A CNF batch in CSR-of-CSR form (see fr_cnf_batch)."""

    def __init__(self, clause_off, literal_off, terms):
        self.clause_off = _host(clause_off, np.uint32)
        self.literal_off = _host(literal_off if len(literal_off) else [0], np.uint32)
        self.terms = _host(terms if len(terms) else np.zeros(0), np.uint32)

    @classmethod
    def of(cls, obj) -> "Cnf":
        if isinstance(obj, Cnf):
            return obj
        return cls(obj.clause_off, obj.literal_off, obj.terms)

    @classmethod
    def from_lists(cls, cnfs) -> "Cnf":
        co, lo, tt = [0], [0], []
        for cnf in cnfs:
            for clause in cnf:
                tt.extend(int(t) for t in clause)
                lo.append(len(tt))
            co.append(len(lo) - 1)
        return cls(co, lo, tt)

    @property
    def n_queries(self) -> int:
        return len(self.clause_off) - 1

    def struct(self) -> FrCnfBatch:
        def p(a):
            return a.ctypes.data_as(_u32p) if a.size else ctypes.cast(None, _u32p)
        return FrCnfBatch(self.n_queries, p(self.clause_off), p(self.literal_off), p(self.terms))


FAILED_COUNT = 0xFFFFFFFF   # out_count of a query the library could not answer


@dataclass
class SearchResult:
    ids: Any        # u32 [n_q, k_max]
    scores: Any     # f32 [n_q, k_max]
    count: Any      # u32 [n_q]
    n_match: Any    # u64 [n_q]

    def failed(self) -> np.ndarray:
        """Indices of the queries marked failed (count 0xFFFFFFFF).  For an
        asynchronous search, call once its stream has passed the search."""
        c = self.count
        if hasattr(c, "cpu"):
            c = c.cpu().numpy()
        return np.flatnonzero(np.asarray(c).view(np.uint32) == FAILED_COUNT)

    def raise_if_failed(self) -> None:
        bad = self.failed()
        if len(bad):
            raise FrError(FR_EUNSUPPORTED, f"queries {bad[:8].tolist()} could not be answered "
                                           "(more tied candidates than the candidate buffer holds)")


class Index:
    """One pre-allocated retrieval index on one GPU (fr_create)."""

    def __init__(self, capacity: int, dim: int, vocab: int, k_max: int, dtype: str = "f32",
                 rescore_r: int = 0, rescore_min: int = 0, max_batch: int = 1024,
                 max_clauses: int = 0, max_literals: int = 0, n_workspaces: int = 1,
                 cand_cap: int = 0, device: int = 0, quant_bits: int = 0,
                 quant_factor: int = 0, list_terms: int = 0, batch_terms: int = 0):
        self._h = None
        cfg = FrConfig(capacity, dim, vocab, k_max, rescore_r, rescore_min, DTYPES[dtype],
                       max_batch, max_clauses, max_literals, n_workspaces, cand_cap, device,
                       quant_bits, quant_factor, list_terms, batch_terms)
        h = _vp()
        _check(lib().fr_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.dim, self.vocab, self.k_max, self.dtype = dim, vocab, k_max, dtype
        self.rescore_r = (rescore_r or 4096) if dtype != "f32" else 0
        self.max_batch = max_batch
        self.n_workspaces = max(1, n_workspaces)
        self.quant_bits = quant_bits
        self.list_terms = list_terms
        self.batch_terms = (batch_terms or 1024) if list_terms else 0
        self.quant_factor = quant_factor or 200

    # ----------------------------------------------------------- lifecycle
    def close(self) -> None:
        if self._h is not None:
            lib().fr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --------------------------------------------------------------- corpus
    def load_corpus(self, emb, ids, term_off, terms) -> None:
        dev = _is_dev(emb)
        if dev != _is_dev(ids):
            raise ValueError("emb and ids must both be host arrays or both device tensors")
        if not dev:
            emb = _host(emb, np.float32)
            ids = _host(ids, np.uint32)
        n = int(emb.shape[0])
        term_off = _host(term_off, np.uint64)
        terms = _host(terms, np.uint32)
        _check(lib().fr_load_corpus(self._h, n, _ptr(emb), _ptr(ids), _ptr(term_off),
                                    _ptr(terms), FR_DEVICE_PTRS if dev else 0))

    def update_docs(self, del_ids, ins_ids, ins_emb, ins_term_off, ins_terms) -> int:
        del_ids = _host(del_ids, np.uint32)
        ins_ids = _host(ins_ids, np.uint32)
        ins_emb = _host(ins_emb, np.float32).reshape(len(ins_ids), self.dim)
        ins_term_off = _host(ins_term_off if len(ins_term_off) else [0], np.uint64)
        ins_terms = _host(ins_terms, np.uint32)
        ep = ctypes.c_uint64(0)
        _check(lib().fr_update_docs(self._h, len(del_ids), _ptr(del_ids), len(ins_ids),
                                    _ptr(ins_ids), _ptr(ins_emb), _ptr(ins_term_off),
                                    _ptr(ins_terms), ctypes.byref(ep)))
        return int(ep.value)

    def info(self) -> Tuple[int, int, int]:
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().fr_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return int(a.value), int(b.value), int(c.value)

    # --------------------------------------------------------------- search
    def search(self, queries, cnf, k, out: Optional[SearchResult] = None, stream=None,
               nowait: bool = False, graph: bool = False,
               preselect: bool = False) -> SearchResult:
        """Filtered top-K of a query batch.

        Host NumPy queries -> host NumPy results (synchronous).  Device
        tensors -> results in ``out`` (device tensors, allocated with torch
        if not given), optionally asynchronous on ``stream`` (a
        ``torch.cuda.Stream`` or a raw hipStream_t integer)."""
        cnf = Cnf.of(cnf)
        n_q = cnf.n_queries
        k = _host(np.broadcast_to(np.asarray(k, dtype=np.uint32), (n_q,)), np.uint32)
        dev = _is_dev(queries)
        flags = ((FR_DEVICE_PTRS if dev else 0) | (FR_NOWAIT if nowait else 0) |
                 (FR_GRAPH if graph else 0) | (FR_ASYNC if dev and stream is not None else 0) |
                 (FR_PRESELECT if preselect else 0))
        if dev:
            if out is None:
                import torch
                d = queries.device
                out = SearchResult(torch.empty((n_q, self.k_max), dtype=torch.int32, device=d),
                                   torch.empty((n_q, self.k_max), dtype=torch.float32, device=d),
                                   torch.empty(n_q, dtype=torch.int32, device=d),
                                   torch.empty(n_q, dtype=torch.int64, device=d))
            s = getattr(stream, "cuda_stream", stream)
        else:
            queries = _host(queries, np.float32).reshape(n_q, self.dim)
            if out is None:
                out = SearchResult(np.empty((n_q, self.k_max), np.uint32),
                                   np.empty((n_q, self.k_max), np.float32),
                                   np.empty(n_q, np.uint32), np.empty(n_q, np.uint64))
            s = None
        st = cnf.struct()
        _check(lib().fr_search(self._h, n_q, _ptr(queries), ctypes.byref(st), _ptr(k),
                               _ptr(out.ids), _ptr(out.scores), _ptr(out.count),
                               _ptr(out.n_match), s, flags))
        return out

    def search_noalloc(self, queries, cnf, k, out: SearchResult, stream=None) -> SearchResult:
        """fr_search_noalloc: device ``queries`` and device outputs ``out``
        (the caller allocates them); the search itself allocates nothing.
        Asynchronous on ``stream`` when one is given."""
        cnf = Cnf.of(cnf)
        n_q = cnf.n_queries
        k = _host(np.broadcast_to(np.asarray(k, dtype=np.uint32), (n_q,)), np.uint32)
        flags = FR_DEVICE_PTRS | (FR_ASYNC if stream is not None else 0)
        st = cnf.struct()
        _check(lib().fr_search_noalloc(self._h, n_q, _ptr(queries), ctypes.byref(st), _ptr(k),
                                       _ptr(out.ids), _ptr(out.scores), _ptr(out.count),
                                       _ptr(out.n_match), getattr(stream, "cuda_stream", stream),
                                       flags))
        return out

    def set_quantizer(self, bin_off, bin_dim, bin_sign) -> None:
        """fr_set_quantizer: the sign-code table (see datagen.sign_projection
        for the tests' draws); re-encodes the stored corpus."""
        bin_off = _host(bin_off, np.uint32)
        bin_dim = _host(bin_dim, np.uint32)
        bin_sign = _host(bin_sign, np.float32)
        _check(lib().fr_set_quantizer(self._h, _ptr(bin_off), _ptr(bin_dim), _ptr(bin_sign)))

    def debug_codes(self, slot0: int, n: int) -> np.ndarray:
        out = np.zeros((n, max(1, self.quant_bits // 64)), np.uint64)
        _check(lib().fr_debug_codes(self._h, slot0, n, _ptr(out)))
        return out

    def stats(self) -> FrStats:
        s = FrStats()
        _check(lib().fr_stats(self._h, ctypes.byref(s)))
        return s

    def timings(self, max_calls: int = 64):
        """(scan_ms, total_ms) arrays of the most recent searches."""
        a = np.zeros(max_calls, np.float32)
        b = np.zeros(max_calls, np.float32)
        n = ctypes.c_uint32()
        _check(lib().fr_timings(self._h, max_calls, _ptr(a), _ptr(b), ctypes.byref(n)))
        return a[:n.value], b[:n.value]

    # ------------------------------------------------------------ testing
    def debug_masks(self, cnf) -> np.ndarray:
        cnf = Cnf.of(cnf)
        _, _, n_slots = self.info()
        words = max(1, (n_slots + 63) // 64)
        out = np.zeros((cnf.n_queries, words), dtype=np.uint64)
        st = cnf.struct()
        _check(lib().fr_debug_masks(self._h, ctypes.byref(st), _ptr(out), words))
        return out

    def debug_rows(self, slot0: int, n: int):
        dpad = (self.dim + 63) // 64 * 64
        dt = {"f32": np.float32, "bf16": np.uint16, "fp8": np.uint8}[self.dtype]
        codes = np.zeros((n, dpad), dtype=dt)
        scales = np.zeros(n, dtype=np.float32)
        _check(lib().fr_debug_rows(self._h, slot0, n, _ptr(codes), _ptr(scales)))
        return codes, scales

    def debug_slots(self, n: Optional[int] = None) -> np.ndarray:
        if n is None:
            n = self.info()[2]
        out = np.zeros(n, dtype=np.uint32)
        _check(lib().fr_debug_slots(self._h, _ptr(out), n))
        return out

    def debug_candidates(self, n_q: int):
        r = max(self.rescore_r, self.k_max)
        ids = np.zeros((n_q, r), np.uint32)
        sc = np.zeros((n_q, r), np.float32)
        cnt = np.zeros(n_q, np.uint32)
        _check(lib().fr_debug_candidates(self._h, n_q, _ptr(ids), _ptr(sc), _ptr(cnt)))
        return ids, sc, cnt

    def set_tiling(self, query_blocks: int = 0, waves: int = 0, groups_per_item: int = 0) -> None:
        _check(lib().fr_set_tiling(self._h, query_blocks, waves, groups_per_item))

    def set_strategy(self, strategy: int = 0, pinned: bool = True) -> None:
        _check(lib().fr_set_strategy(self._h, strategy, 1 if pinned else 0))

    def autotune(self, queries, cnf, k) -> Tuple[int, int, int, int]:
        """Tune the scan tiling and search strategy for this batch's shape;
        the choice goes into the index's tuning table (used by later searches
        without a pinned tiling).  Returns (query_blocks, waves,
        groups_per_item, strategy)."""
        cnf = Cnf.of(cnf)
        n_q = cnf.n_queries
        q = _host(queries, np.float32).reshape(n_q, self.dim)
        k = _host(np.broadcast_to(np.asarray(k, dtype=np.uint32), (n_q,)), np.uint32)
        a, b, c, d = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        st = cnf.struct()
        _check(lib().fr_autotune(self._h, n_q, _ptr(q), ctypes.byref(st), _ptr(k), 0,
                                 ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                 ctypes.byref(d)))
        return int(a.value), int(b.value), int(c.value), int(d.value)

    def tuning_choice(self, n_q: int, k):
        """(query_blocks, waves, groups_per_item, strategy, source) a search of
        n_q queries with these K would use; source 0 defaults, 1 pinned, 2
        the tuning table."""
        k = _host(np.broadcast_to(np.asarray(k, dtype=np.uint32), (n_q,)), np.uint32)
        out = [ctypes.c_uint32() for _ in range(5)]
        _check(lib().fr_tuning_choice(self._h, n_q, _ptr(k), *[ctypes.byref(o) for o in out]))
        return tuple(int(o.value) for o in out)

    def tuning_save(self, path: str) -> None:
        _check(lib().fr_tuning_save(self._h, os.fsencode(path)))

    def tuning_load(self, path: str) -> int:
        n = ctypes.c_uint32()
        _check(lib().fr_tuning_load(self._h, os.fsencode(path), ctypes.byref(n)))
        return int(n.value)
