"""Shared test helpers: build a GPU index and an oracle on the same seeded
inputs, and compare their results query by query with the checker."""
from __future__ import annotations

import numpy as np

import datagen
from oracle import OracleIndex, check_result, tolerance


def oracle_for(c: datagen.Corpus) -> OracleIndex:
    o = OracleIndex(c.cfg.dim, c.cfg.vocab)
    o.load(c.emb, c.ids, c.term_off, c.terms)
    return o


def gpu_index(c: datagen.Corpus, k_max: int, dtype: str = "f32", capacity=None, **kw):
    from paper_2402_13435_amd import Index
    ix = Index(capacity or max(c.n, 1), c.cfg.dim, c.cfg.vocab, k_max, dtype=dtype, **kw)
    ix.load_corpus(c.emb, c.ids, c.term_off, c.terms)
    return ix


def check_query(o: OracleIndex, qb, q: int, res, k: int, tol=None, score_tol=None):
    """Check GPU row q of ``res`` against the oracle with the tie rule."""
    tol = tolerance(o.dim) if tol is None else tol
    a = o.search_one(qb.emb[q], qb.cnf(q), k)
    match_ids = set(int(o.ids[r]) for r in o.match_rows(qb.cnf(q)))
    check_result(res.ids[q], res.scores[q], int(res.count[q]), int(res.n_match[q]),
                 a.ids, a.scores, a.n_match, k,
                 lambda ids: o.score_ids(qb.emb[q], ids), lambda i: i in match_ids,
                 tol, score_tol)
    return a


def masks_as_bytes(words: np.ndarray, n: int) -> np.ndarray:
    """GPU mask words (u64, bit s = slot s) as little-bit-order bytes."""
    b = np.ascontiguousarray(words).astype("<u8").view(np.uint8)
    nbytes = (n + 7) // 8
    out = b[:nbytes].copy()
    if n % 8:
        out[-1] &= (1 << (n % 8)) - 1
    return out
