"""The FP64 oracle: plain CNF match + FP64 dot + full sort.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Each step cites the
passage of the paper it follows.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence

import numpy as np

U32_MAX = 0xFFFFFFFF


def tolerance(dim: int) -> float:
    """Score tolerance for an FP32 dot product of two unit vectors.

    The paper fixes no accumulation order or rounding (Sec. 5.3 and the
    appendix "EBR" only say "inner product").  Any FP32 summation order obeys
    the order-free forward bound |s_hat - s| <= gamma_d * sum|q_i x_i| with
    gamma_d = d u / (1 - d u), u = 2^-24; for unit vectors sum|q_i x_i| <= 1.
    The tolerance is twice that bound, which also covers the matrix cores'
    internal rounding.
    """
    u = 2.0 ** -24
    return 2.0 * dim * u / (1.0 - dim * u)


@dataclasses.dataclass
class OracleResult:
    ids: np.ndarray        # u32 [count]
    scores: np.ndarray     # f64 [count]
    count: int
    n_match: int


class OracleIndex:
    """Live corpus state: id -> (FP32 embedding, term set).

    Rows are kept in insertion order; deleting marks a row dead.  Updates
    follow the reading that one call applies all its deletes, then all its
    inserts, and is rejected as a whole on any error (the paper only says the
    job corpus changes daily, Sec. 2).
    """

    def __init__(self, dim: int, vocab: int):
        self.dim = int(dim)
        self.vocab = int(vocab)
        self.emb = np.zeros((0, dim), dtype=np.float32)
        self.ids = np.zeros(0, dtype=np.uint32)
        self.live = np.zeros(0, dtype=bool)
        # term sets as CSR: row r holds terms[off[r]:off[r+1]] (sorted, distinct)
        self.off = np.zeros(1, dtype=np.int64)
        self.terms = np.zeros(0, dtype=np.int64)
        self._row_of: Optional[Dict[int, int]] = None
        self._postings: Optional[List[np.ndarray]] = None

    # ------------------------------------------------------------------ state
    @property
    def n_rows(self) -> int:
        return len(self.ids)

    @property
    def n_live(self) -> int:
        return int(self.live.sum())

    @staticmethod
    def _csr_sets(n: int, term_off, terms):
        """Per-row distinct sorted term sets of a CSR list (duplicates dropped)."""
        term_off = np.asarray(term_off, dtype=np.int64)
        terms = np.asarray(terms, dtype=np.int64)[term_off[0]:term_off[n]] if n else \
            np.zeros(0, dtype=np.int64)
        lens = np.diff(term_off[:n + 1])
        rows = np.repeat(np.arange(n, dtype=np.int64), lens)
        key = rows * (int(terms.max()) + 1 if len(terms) else 1) + terms
        if len(key) > 1 and not np.all(key[1:] > key[:-1]):
            key = np.unique(key)                      # sort within rows, drop duplicates
        width = int(terms.max()) + 1 if len(terms) else 1
        rows = key // width
        off = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(np.bincount(rows, minlength=n), out=off[1:])
        return off, key - rows * width

    @property
    def row_of(self) -> Dict[int, int]:
        if self._row_of is None:
            self._row_of = {int(x): i for i, x in enumerate(self.ids)}
        return self._row_of

    def term_set(self, r: int) -> np.ndarray:
        return self.terms[self.off[r]:self.off[r + 1]]

    def load(self, emb, ids, term_off, terms) -> None:
        emb = np.ascontiguousarray(emb, dtype=np.float32)
        ids = np.asarray(ids, dtype=np.uint32)
        terms = np.asarray(terms, dtype=np.uint32)
        if emb.shape != (len(ids), self.dim):
            raise ValueError("embedding shape")
        if len(np.unique(ids)) != len(ids) or (ids == U32_MAX).any():
            raise ValueError("ids must be unique and < 2^32-1")
        if len(terms) and int(terms.max()) >= self.vocab:
            raise ValueError("term id out of range")
        self.emb = emb.copy()
        self.ids = ids.copy()
        self.live = np.ones(len(ids), dtype=bool)
        self.off, self.terms = self._csr_sets(len(ids), term_off, terms)
        self._row_of = None
        self._postings = None

    def update(self, del_ids, ins_ids, ins_emb, ins_term_off, ins_terms) -> None:
        del_ids = [int(x) for x in np.asarray(del_ids, dtype=np.uint32)]
        ins_ids = [int(x) for x in np.asarray(ins_ids, dtype=np.uint32)]
        # validate the whole call first (all-or-nothing)
        if len(set(del_ids)) != len(del_ids):
            raise KeyError("duplicate delete id")
        for x in del_ids:
            r = self.row_of.get(x)
            if r is None or not self.live[r]:
                raise KeyError(f"unknown id {x}")
        dset = set(del_ids)
        if len(set(ins_ids)) != len(ins_ids):
            raise KeyError("duplicate insert id")
        for x in ins_ids:
            r = self.row_of.get(x)
            if x == U32_MAX or (r is not None and self.live[r] and x not in dset):
                raise KeyError(f"id {x} already live")
        for x in del_ids:
            self.live[self.row_of[x]] = False
        if ins_ids:
            ins_emb = np.ascontiguousarray(ins_emb, dtype=np.float32).reshape(-1, self.dim)
            base = self.n_rows
            self.emb = np.concatenate([self.emb, ins_emb])
            self.ids = np.concatenate([self.ids, np.asarray(ins_ids, dtype=np.uint32)])
            self.live = np.concatenate([self.live, np.ones(len(ins_ids), dtype=bool)])
            off, terms = self._csr_sets(len(ins_ids), ins_term_off, ins_terms)
            self.terms = np.concatenate([self.terms, terms])
            self.off = np.concatenate([self.off, self.off[-1] + off[1:]])
            rmap = self.row_of
            for j, x in enumerate(ins_ids):
                rmap[x] = base + j
        self._postings = None

    # --------------------------------------------------------------- F-TBR
    def _posting_lists(self) -> List[np.ndarray]:
        """term -> sorted rows holding it (the transpose of the term lists)."""
        if self._postings is None:
            lens = np.diff(self.off)
            rows = np.repeat(np.arange(self.n_rows, dtype=np.int64), lens)
            flat = self.terms
            order = np.argsort(flat, kind="stable")
            bounds = np.searchsorted(flat[order], np.arange(self.vocab + 1))
            srt = rows[order]
            self._postings = [srt[bounds[t]:bounds[t + 1]] for t in range(self.vocab)]
        return self._postings

    def term_bitmap(self, t: int) -> np.ndarray:
        """Packed bitmap over rows (bit r of byte r//8, little bit order)."""
        ind = np.zeros(self.n_rows, dtype=bool)
        ind[self._posting_lists()[int(t)]] = True
        return np.packbits(ind, bitorder="little")

    def live_bitmap(self) -> np.ndarray:
        return np.packbits(self.live, bitorder="little")

    def match_bitmap(self, cnf: Sequence[Sequence[int]]) -> np.ndarray:
        """CNF match over rows: live AND (AND over clauses of OR over terms).

        Sec. 5.3 turns each TBR query into conjunctive normal form and checks
        each clause against the document's attributes; the appendix "TBR"
        counts a clause as met when the query's values for it overlap the
        document's.  No clause -> every live row; an empty clause -> none.
        """
        m = self.live_bitmap()
        for clause in cnf:
            c = np.zeros_like(m)
            for t in clause:
                c |= self.term_bitmap(t)
            m &= c
        return m

    def match_rows(self, cnf) -> np.ndarray:
        bits = np.unpackbits(self.match_bitmap(cnf), bitorder="little",
                             count=self.n_rows).astype(bool)
        return np.flatnonzero(bits)

    # --------------------------------------------------------------- F-EBR
    def scores(self, q: np.ndarray, rows: np.ndarray, chunk: int = 1 << 16) -> np.ndarray:
        """Inner products (appendix, "EBR") in FP64.

        Each product of two FP32 values is exact in FP64; the row sum is
        NumPy's fixed pairwise summation along the contiguous axis, so equal
        rows give equal scores whatever the thread count.
        """
        q64 = np.asarray(q, dtype=np.float32).astype(np.float64)
        out = np.empty(len(rows), dtype=np.float64)
        for a in range(0, len(rows), chunk):
            x = self.emb[rows[a:a + chunk]].astype(np.float64)
            out[a:a + chunk] = (x * q64).sum(axis=1)
        return out

    def score_ids(self, q: np.ndarray, ids) -> np.ndarray:
        rows = np.array([self.row_of[int(x)] for x in ids], dtype=np.int64)
        return self.scores(q, rows)

    # -------------------------------------------------------------- select
    def search_one(self, q: np.ndarray, cnf, k: int) -> OracleResult:
        """Top-k matches by (score desc, id asc) via a full sort."""
        rows = self.match_rows(cnf)
        s = self.scores(q, rows)
        order = np.lexsort((self.ids[rows], -s))
        take = order[:min(int(k), len(rows))]
        return OracleResult(self.ids[rows[take]].copy(), s[take].copy(),
                            len(take), len(rows))

    def search(self, qb, k: Optional[Sequence[int]] = None) -> List[OracleResult]:
        ks = qb.k if k is None else k
        return [self.search_one(qb.emb[i], qb.cnf(i), int(ks[i])) for i in range(qb.n)]

    # --------------------------------------------- reduced-precision forms
    def approx_scores(self, q: np.ndarray, rows: np.ndarray, storage: str) -> np.ndarray:
        """First-pass scores of the reduced-precision forms, in FP64.

        Both operands are quantised (corpus rows at load, the query per
        search) by the CPU emulation in ``oracle.quant``; the products of the
        dequantised values are then summed exactly in FP64 and multiplied by
        the scales.  The GPU accumulates in FP32, so it agrees with this to
        within the FP32 accumulation bound.
        """
        from . import quant
        x = self.emb[rows]
        if storage == "bf16":
            qd = quant.bf16_round(np.asarray(q, dtype=np.float32)).astype(np.float64)
            xd = quant.bf16_round(x).astype(np.float64)
            return (xd * qd).sum(axis=1)
        if storage == "fp8":
            qv, qs = quant.fp8_rows(np.asarray(q, dtype=np.float32)[None, :])
            xv, xs = quant.fp8_rows(x)
            dot = (xv.astype(np.float64) * qv[0].astype(np.float64)).sum(axis=1)
            return dot * float(qs[0]) * xs.astype(np.float64)
        raise ValueError(storage)

    def search_rescored_one(self, q, cnf, k: int, r: int, storage: str) -> OracleResult:
        """Reduced-precision pipeline: approximate top-r by (approx desc, id
        asc), then exact rescoring of those r and top-k by (exact desc, id
        asc).  This mirrors the paper's use of a cheap, approximate
        pre-selection ahead of exact scoring (appendix, "Quantization"), with
        the cut-off r playing the role of quantK."""
        rows = self.match_rows(cnf)
        a = self.approx_scores(q, rows, storage)
        pre = np.lexsort((self.ids[rows], -a))[:min(int(r), len(rows))]
        rows_r = rows[pre]
        s = self.scores(q, rows_r)
        order = np.lexsort((self.ids[rows_r], -s))[:min(int(k), len(rows_r))]
        return OracleResult(self.ids[rows_r[order]].copy(), s[order].copy(),
                            len(order), len(rows))
