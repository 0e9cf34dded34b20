"""Continuous-batching request loop over one retrieval index.

Requests (query embedding, CNF predicate, K) arrive at any time.  A
dispatcher thread groups whatever is pending into a batch as soon as one of
the index's workspaces is free (admission by pre-allocated memory: one
workspace = one batch of at most ``max_batch`` queries in flight) and issues
it asynchronously on that workspace's stream, so batches admitted while
others are on the device overlap with them.  A completion thread waits for
each batch's event, copies its results to the host and resolves the
requests' futures, recording latency = completion - arrival.

This is the serving form of the paper's batch inference (appendix "Batch
Inference": requests bundled so the corpus is scanned once per batch, a
trade of latency for throughput).  Document inserts and deletes go through
``update`` and are ordered between batches by the library (an update waits
for every batch in flight; later batches see it).
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

from .binding import FR_EUNSUPPORTED, Cnf, FrError, Index, SearchResult

FAILED = 0xFFFFFFFF     # count of a query the library could not answer


@dataclass
class Request:
    emb: np.ndarray
    cnf: Sequence[Sequence[int]]
    k: int
    t_arrival: float
    future: Future = field(default_factory=Future)


@dataclass
class Reply:
    ids: np.ndarray
    scores: np.ndarray
    n_match: int
    t_arrival: float
    t_done: float
    batch_size: int

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Server:
    """Continuous batching over ``index`` (created with ``n_workspaces`` >=
    ``slots``).  Every slot owns a CUDA stream at the default priority and
    device buffers for one batch."""

    def __init__(self, index: Index, slots: int = 2, max_batch: Optional[int] = None,
                 max_wait_s: float = 0.0):
        import torch
        self.torch = torch
        self.ix = index
        # a batch never exceeds what one workspace of the index holds
        self.max_batch = min(int(max_batch or index.max_batch), int(index.max_batch))
        self.max_wait_s = max_wait_s
        dev = torch.device("cuda", torch.cuda.current_device())
        self.dev = dev
        self.slots = []
        for _ in range(slots):
            s = torch.cuda.Stream(device=dev)
            out = SearchResult(
                torch.empty((self.max_batch, index.k_max), dtype=torch.int32, device=dev),
                torch.empty((self.max_batch, index.k_max), dtype=torch.float32, device=dev),
                torch.empty(self.max_batch, dtype=torch.int32, device=dev),
                torch.empty(self.max_batch, dtype=torch.int64, device=dev))
            qbuf = torch.empty((self.max_batch, index.dim), dtype=torch.float32, device=dev)
            self.slots.append({"stream": s, "out": out, "q": qbuf, "busy": False})
        self._pending: collections.deque = collections.deque()
        self._cv = threading.Condition()
        self._inflight: collections.deque = collections.deque()
        self._done_cv = threading.Condition()
        self._stop = False
        self._lock = threading.Lock()        # serialises library calls from this object
        self.batches: List[int] = []
        self._disp = threading.Thread(target=self._dispatch, daemon=True)
        self._comp = threading.Thread(target=self._complete, daemon=True)
        self._disp.start()
        self._comp.start()

    # ------------------------------------------------------------- clients
    def submit(self, emb, cnf, k: int) -> Future:
        """Queue one request; raises ValueError at once for a request the
        index cannot take (so that it never reaches, and stalls, a batch)."""
        emb = np.ascontiguousarray(emb, dtype=np.float32).reshape(-1)
        if emb.shape[0] != self.ix.dim:
            raise ValueError(f"query has {emb.shape[0]} dimensions, the index {self.ix.dim}")
        if not 0 <= int(k) <= self.ix.k_max:
            raise ValueError(f"K={k} outside 0..{self.ix.k_max}")
        for clause in cnf:
            for t in clause:
                if not 0 <= int(t) < self.ix.vocab:
                    raise ValueError(f"term {t} outside the vocabulary (0..{self.ix.vocab - 1})")
        r = Request(emb, cnf, int(k), time.perf_counter())
        with self._cv:
            self._pending.append(r)
            self._cv.notify()
        return r.future

    def update(self, del_ids, ins_ids, ins_emb, ins_term_off, ins_terms) -> int:
        with self._lock:
            return self.ix.update_docs(del_ids, ins_ids, ins_emb, ins_term_off, ins_terms)

    def close(self) -> None:
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        self._disp.join()
        with self._done_cv:
            self._done_cv.notify_all()
        self._comp.join()

    # ------------------------------------------------------------- threads
    def _free_slot(self):
        for s in self.slots:
            if not s["busy"]:
                return s
        return None

    def _dispatch(self) -> None:
        torch = self.torch
        torch.cuda.set_device(self.dev)
        while True:
            with self._cv:
                while not self._stop and (not self._pending or self._free_slot() is None):
                    self._cv.wait(timeout=0.01)
                if self._stop and not self._pending:
                    return
                if self.max_wait_s and len(self._pending) < self.max_batch:
                    deadline = self._pending[0].t_arrival + self.max_wait_s
                    while (len(self._pending) < self.max_batch and not self._stop and
                           time.perf_counter() < deadline):
                        self._cv.wait(timeout=max(0.0, deadline - time.perf_counter()))
                slot = self._free_slot()
                if slot is None:
                    continue
                reqs = [self._pending.popleft()
                        for _ in range(min(self.max_batch, len(self._pending)))]
                slot["busy"] = True
            n = len(reqs)
            emb = np.stack([r.emb for r in reqs])
            cnf = Cnf.from_lists([r.cnf for r in reqs])
            k = np.array([r.k for r in reqs], dtype=np.uint32)
            s = slot["stream"]
            try:
                with torch.cuda.stream(s):
                    slot["q"][:n].copy_(torch.from_numpy(emb).pin_memory(), non_blocking=True)
                    out = SearchResult(slot["out"].ids[:n], slot["out"].scores[:n],
                                       slot["out"].count[:n], slot["out"].n_match[:n])
                    with self._lock:
                        self.ix.search(slot["q"][:n], cnf, k, out=out, stream=s)
                    ev = torch.cuda.Event()
                    ev.record(s)
            except Exception as e:   # the batch fails, the server keeps serving
                s.synchronize()
                with self._cv:
                    slot["busy"] = False
                    self._cv.notify()
                for r in reqs:
                    r.future.set_exception(e)
                continue
            self.batches.append(n)
            with self._done_cv:
                self._inflight.append((slot, reqs, ev, n))
                self._done_cv.notify()

    def _complete(self) -> None:
        torch = self.torch
        torch.cuda.set_device(self.dev)
        while True:
            with self._done_cv:
                while not self._inflight and not (self._stop and not self._disp.is_alive()):
                    self._done_cv.wait(timeout=0.01)
                if not self._inflight:
                    return
                slot, reqs, ev, n = self._inflight.popleft()
            ev.synchronize()
            out = slot["out"]
            ids = out.ids[:n].cpu().numpy().view(np.uint32)
            sc = out.scores[:n].cpu().numpy()
            cnt = out.count[:n].cpu().numpy().view(np.uint32)
            nm = out.n_match[:n].cpu().numpy()
            t = time.perf_counter()
            with self._cv:
                slot["busy"] = False
                self._cv.notify()
            for i, r in enumerate(reqs):
                c = int(cnt[i])
                if c == FAILED:
                    r.future.set_exception(FrError(
                        FR_EUNSUPPORTED, "more tied candidates than the candidate buffer holds"))
                    continue
                r.future.set_result(Reply(ids[i, :c].copy(), sc[i, :c].copy(), int(nm[i]),
                                          r.t_arrival, t, n))


def latency_summary(replies: Sequence[Reply]) -> dict:
    lat = np.array([r.latency for r in replies]) * 1e3
    if not len(lat):
        return {}
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "n": int(len(lat))}
