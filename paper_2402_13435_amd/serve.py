"""Continuous batching over one retrieval index (the library's fr_server).

The request loop itself is native (fr_server_* in the C ABI): a dispatcher
thread forms a batch of everything pending whenever fewer than
``max_inflight`` batches are on the device, so the batch size follows the
arrival rate, and enqueues it on the server's stream; a completion thread
copies each finished batch's rows to the requests' buffers.  This module
gives it two Python faces:

* ``Server.submit`` -> ``Future`` of a ``Reply`` (one request at a time, for
  applications and tests);
* ``Server.submit_many`` / ``Server.wait`` (many requests per call, results
  written into caller arrays, for load generators that must reach rates a
  per-request Python path cannot).

This is the serving form of the paper's batch inference (appendix "Batch
Inference": requests bundled so the corpus is scanned once per batch, a
trade of latency for throughput).  Document inserts and deletes go through
``update`` (fr_update_docs), which the index orders between batches on the
device without waiting for the batches in flight.
"""
from __future__ import annotations

import collections
import ctypes
import threading
from concurrent.futures import Future
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from .binding import (FR_EUNSUPPORTED, Cnf, FrError, FrServerConfig, FrServerStats, Index,
                      _check, _host, _ptr, _vp, lib)

FAILED = 0xFFFFFFFF     # count of a query the library could not answer
WAIT_FOREVER = 0xFFFFFFFF


def clock_ns() -> int:
    """The server's clock (monotonic, ns): arrival and completion times."""
    return int(lib().fr_clock_ns())


@dataclass
class Reply:
    ids: np.ndarray
    scores: np.ndarray
    n_match: int
    t_arrival: float      # seconds on the server's clock
    t_done: float

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class ResultRows:
    """Result rows for n requests, in the layout fr_server_submit writes."""

    def __init__(self, n: int, k_max: int):
        self.ids = np.empty((n, k_max), np.uint32)
        self.scores = np.empty((n, k_max), np.float32)
        self.count = np.empty(n, np.uint32)
        self.n_match = np.empty(n, np.uint64)
        self.done_ns = np.empty(n, np.uint64)
        self.status = np.empty(n, np.int32)


class Server:
    """Continuous batching over ``index``.  ``max_inflight`` batches may be
    on the device at once (at most the index's ``n_workspaces``; 2 keeps the
    device busy while the next batch is formed); ``max_wait_s`` lets an idle
    device wait that long after the oldest request for a fuller batch."""

    def __init__(self, index: Index, max_inflight: int = 2, max_batch: Optional[int] = None,
                 max_wait_s: float = 0.0):
        self.ix = index
        # a batch never exceeds what one workspace of the index holds
        self.max_batch = min(int(max_batch or index.max_batch), int(index.max_batch))
        self.max_inflight = max(1, min(int(max_inflight), index.n_workspaces))
        cfg = FrServerConfig(self.max_batch, self.max_inflight, int(round(max_wait_s * 1e6)))
        h = _vp()
        _check(lib().fr_server_create(index._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._lock = threading.Lock()      # ticket order == order of self._waiting
        self._cv = threading.Condition(self._lock)
        self._waiting: collections.deque = collections.deque()
        self._closing = False
        self._resolver = threading.Thread(target=self._resolve, daemon=True)
        self._resolver.start()

    # ------------------------------------------------------------- clients
    def _validate(self, emb, cnf, k) -> np.ndarray:
        emb = np.ascontiguousarray(emb, dtype=np.float32).reshape(-1)
        if emb.shape[0] != self.ix.dim:
            raise ValueError(f"query has {emb.shape[0]} dimensions, the index {self.ix.dim}")
        if not 0 <= int(k) <= self.ix.k_max:
            raise ValueError(f"K={k} outside 0..{self.ix.k_max}")
        for clause in cnf:
            for t in clause:
                if not 0 <= int(t) < self.ix.vocab:
                    raise ValueError(f"term {t} outside the vocabulary (0..{self.ix.vocab - 1})")
        return emb

    def submit(self, emb, cnf, k: int) -> Future:
        """Queue one request; raises ValueError at once for a request the
        index cannot take.  The future resolves to a ``Reply``, or raises
        ``FrError`` for a query the library could not answer."""
        emb = self._validate(emb, cnf, k)
        rows = ResultRows(1, self.ix.k_max)
        fut: Future = Future()
        c = Cnf.from_lists([cnf])
        t_arr = np.array([clock_ns()], np.uint64)
        with self._cv:
            ticket = self._submit(emb, c, np.array([k], np.uint32), t_arr, rows, 0)
            self._waiting.append((ticket, rows, int(t_arr[0]), fut))
            self._cv.notify()
        return fut

    def submit_many(self, emb, cnf: Cnf, k, t_arrival_ns, rows: ResultRows, row0: int) -> int:
        """Queue n requests (emb n x dim, their Cnf, k, arrival times on the
        server's clock); their results go to rows[row0 : row0 + n], which
        must stay alive until ``wait`` has returned for the last ticket.
        Returns the first ticket."""
        with self._cv:
            return self._submit(emb, cnf, k, t_arrival_ns, rows, row0)

    def _submit(self, emb, cnf: Cnf, k, t_arrival_ns, rows: ResultRows, row0: int) -> int:
        n = cnf.n_queries
        emb = _host(emb, np.float32).reshape(n, self.ix.dim)
        k = _host(k, np.uint32)
        t = _host(t_arrival_ns, np.uint64)
        st = cnf.struct()
        first = ctypes.c_uint64(0)
        _check(lib().fr_server_submit(
            self._h, n, _ptr(emb), ctypes.byref(st), _ptr(k), _ptr(t),
            rows.ids[row0:].ctypes.data, rows.scores[row0:].ctypes.data,
            rows.count[row0:].ctypes.data, rows.n_match[row0:].ctypes.data,
            rows.done_ns[row0:].ctypes.data, rows.status[row0:].ctypes.data,
            ctypes.byref(first)))
        return int(first.value)

    def wait(self, ticket: int, timeout_s: Optional[float] = None) -> None:
        """Return once every request up to ``ticket`` has completed."""
        ms = WAIT_FOREVER if timeout_s is None else max(0, int(timeout_s * 1e3))
        _check(lib().fr_server_wait(self._h, int(ticket), ms))

    def stats(self) -> dict:
        s = FrServerStats()
        _check(lib().fr_server_get_stats(self._h, ctypes.byref(s)))
        return {"batches": int(s.batches), "queries": int(s.queries), "failed": int(s.failed),
                "max_batch_seen": int(s.max_batch_seen), "pending": int(s.pending),
                "mean_batch": float(s.queries) / max(1, int(s.batches))}

    def update(self, del_ids, ins_ids, ins_emb, ins_term_off, ins_terms) -> int:
        return self.ix.update_docs(del_ids, ins_ids, ins_emb, ins_term_off, ins_terms)

    def close(self) -> None:
        """Serve what is queued, then stop."""
        if self._h is None:
            return
        with self._cv:
            self._closing = True
            self._cv.notify_all()
        self._resolver.join()
        lib().fr_server_destroy(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------- resolver
    def _resolve(self) -> None:
        while True:
            with self._cv:
                while not self._waiting and not self._closing:
                    self._cv.wait()
                if not self._waiting:
                    return
                ticket, rows, t_arr, fut = self._waiting.popleft()
            try:
                self.wait(ticket)
            except FrError as e:
                fut.set_exception(e)
                continue
            st = int(rows.status[0])
            if st != 0:
                msg = ("more tied candidates than the candidate buffer holds"
                       if st == FR_EUNSUPPORTED else "the batch could not be enqueued")
                fut.set_exception(FrError(st, msg))
                continue
            c = int(rows.count[0])
            fut.set_result(Reply(rows.ids[0, :c].copy(), rows.scores[0, :c].copy(),
                                 int(rows.n_match[0]), t_arr * 1e-9,
                                 int(rows.done_ns[0]) * 1e-9))


def latency_summary(replies: Sequence[Reply]) -> dict:
    lat = np.array([r.latency for r in replies]) * 1e3
    if not len(lat):
        return {}
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "n": int(len(lat))}
