"""Seeded synthetic inputs for filtered top-K retrieval.

This module only *draws* inputs.  It holds none of the retrieval arithmetic:
it never evaluates a term predicate, never scores a document and never
selects.  Both the FP64 oracle (``oracle/``) and the GPU library's tests and
benchmark consume what it produces, and neither shares any other code.

The paper's own corpus (LinkedIn job postings with field-structured terms and
learned two-tower embeddings; Sections 4.2, 4.3 and the appendix on GPU
optimisation) is proprietary, so every workload here is a synthetic stand-in
with the same structure:

* document embeddings: i.i.d. N(0,1) in FP64, L2-normalised per row in FP64,
  then rounded to FP32 (RNE).  The FP32 values are the truth downstream.
* document term sets: ``n_i ~ U{lo..hi}`` draws with replacement from a
  finite Zipf law ``P(r) ~ r^-s`` over ranks ``1..V`` (term id = rank-1);
  the term set is the set of distinct draws.  Terms stand for the field
  values (geo, skill, ...) of the appendix's TBR example; a field is a
  disjoint id range, so one global id space has the same semantics.
* queries: normalised Gaussian embeddings plus a CNF predicate (an AND of
  clauses, each an OR of terms), drawn either freely (tiny config) or tuned
  towards a target selectivity drawn log-uniformly from a range.  Tuning uses
  only per-term document frequencies under an independence assumption; the
  achieved selectivity is measured later by the oracle.
* per-query K (fixed, or drawn from a set), Poisson arrival times and an
  insert/delete update log for the serving workload.

Everything derives from ``numpy.random.SeedSequence([240213435, config])``
with children spawned in a fixed order, and corpus rows are drawn in
independent 1M-row chunks so that any chunk can be regenerated alone.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Sequence, Tuple

import numpy as np

ROOT_SEED = 240213435
CHUNK_ROWS = 1 << 20

# child stream indices (fixed order)
_S_EMB, _S_TERMS, _S_QEMB, _S_PRED, _S_K, _S_ARR, _S_UPD = range(7)


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    index: int
    n_docs: int
    dim: int
    vocab: int
    terms_lo: int
    terms_hi: int
    zipf_s: float
    n_queries: int
    k_choices: Tuple[int, ...]
    sel_range: Optional[Tuple[float, float]]  # None -> untuned CNF (tiny config)
    clauses: Tuple[int, int] = (1, 3)
    literals: Tuple[int, int] = (1, 4)
    storage: str = "f32"
    rescore_r: int = 0


CONFIGS = {
    # 10k docs, d=64, V=1024, 8-32 terms, 16 untuned queries, K=10
    "tiny": Config("tiny", 0, 10_000, 64, 1024, 8, 32, 1.1, 16, (10,), None),
    # 1M docs, d=128 FP32, V=4096, 16-48 terms, 256 queries, sel 0.1%-50%, K=100
    "fp32": Config("fp32", 1, 1_000_000, 128, 4096, 16, 48, 1.1, 256, (100,),
                   (1e-3, 0.5)),
    # 10M docs, d=256, BF16/FP8 storage, 1024 queries, sel 1%-50%, K=100, R=4096
    "precision": Config("precision", 2, 10_000_000, 256, 4096, 16, 48, 1.1, 1024,
                        (100,), (1e-2, 0.5), storage="bf16", rescore_r=4096),
    # 10M docs, d=128 BF16, V=16384, 4096 queries, sel 1e-5-0.5, K in {10,100,1000}
    "batching": Config("batching", 3, 10_000_000, 128, 16384, 16, 48, 1.1, 4096,
                       (10, 100, 1000), (1e-5, 0.5), storage="bf16", rescore_r=4096),
    # 40M docs, d=128 BF16, V=16384; Poisson arrivals, sel 1e-4-0.3, K in {10,100}
    "serving": Config("serving", 4, 40_000_000, 128, 16384, 16, 48, 1.1, 4096,
                      (10, 100), (1e-4, 0.3), storage="bf16", rescore_r=1024),
}


def scaled(cfg: Config, n_docs: int, n_queries: Optional[int] = None) -> Config:
    """Same recipe at a different corpus / batch size (parity-sized cases)."""
    return dataclasses.replace(cfg, n_docs=int(n_docs),
                               n_queries=int(n_queries or cfg.n_queries))


def _children(cfg: Config) -> List[np.random.SeedSequence]:
    return np.random.SeedSequence([ROOT_SEED, cfg.index]).spawn(7)


def zipf_probs(vocab: int, s: float) -> np.ndarray:
    r = np.arange(1, vocab + 1, dtype=np.float64)
    p = r ** (-s)
    return p / p.sum()


# --------------------------------------------------------------------------
# corpus
# --------------------------------------------------------------------------

def _normal_rows(seed: np.random.SeedSequence, n: int, d: int) -> np.ndarray:
    g = np.random.Generator(np.random.PCG64(seed))
    x = g.standard_normal((n, d))                    # FP64
    nrm = np.sqrt(np.einsum("ij,ij->i", x, x))
    nrm[nrm == 0] = 1.0
    return (x / nrm[:, None]).astype(np.float32)     # RNE to FP32


def _term_rows(seed: np.random.SeedSequence, n: int, cfg: Config,
               cdf: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    g = np.random.Generator(np.random.PCG64(seed))
    cnt = g.integers(cfg.terms_lo, cfg.terms_hi + 1, size=n)
    draws = np.searchsorted(cdf, g.random(int(cnt.sum())), side="right")
    draws = np.minimum(draws, cfg.vocab - 1).astype(np.int64)
    owner = np.repeat(np.arange(n, dtype=np.int64), cnt)
    uniq = np.unique(owner * cfg.vocab + draws)      # sorted, de-duplicated
    doc = uniq // cfg.vocab
    terms = (uniq - doc * cfg.vocab).astype(np.uint32)
    lens = np.bincount(doc, minlength=n)
    return lens, terms


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunk_rows(cfg: Config, c: int) -> int:
    return min(CHUNK_ROWS, cfg.n_docs - c * CHUNK_ROWS)


def _chunks(cfg: Config, start: int, n: int) -> range:
    if start < 0 or start + n > cfg.n_docs:
        raise ValueError("rows outside the corpus")
    return range(start // CHUNK_ROWS, (start + n + CHUNK_ROWS - 1) // CHUNK_ROWS)


def embeddings(cfg: Config, n: Optional[int] = None, start: int = 0) -> np.ndarray:
    """Rows [start, start+n) of the document embedding matrix (FP32, n x d)."""
    n = cfg.n_docs - start if n is None else n
    chunks = _chunks(cfg, start, n)
    chunk_seeds = _children(cfg)[_S_EMB].spawn(max(chunks.stop, 1))
    out = np.empty((n, cfg.dim), dtype=np.float32)

    def work(c):
        lo = c * CHUNK_ROWS
        rows = _normal_rows(chunk_seeds[c], _chunk_rows(cfg, c), cfg.dim)
        a, b = max(lo, start), min(lo + len(rows), start + n)
        out[a - start:b - start] = rows[a - lo:b - lo]

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(work, chunks))
    return out


def doc_terms(cfg: Config, n: Optional[int] = None,
              start: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """CSR term lists of docs [start, start+n): (offsets u64[n+1], terms u32)."""
    n = cfg.n_docs - start if n is None else n
    chunks = _chunks(cfg, start, n)
    cdf = np.cumsum(zipf_probs(cfg.vocab, cfg.zipf_s))
    chunk_seeds = _children(cfg)[_S_TERMS].spawn(max(chunks.stop, 1))
    parts = {}

    def work(c):
        lo, m = c * CHUNK_ROWS, _chunk_rows(cfg, c)
        lens, terms = _term_rows(chunk_seeds[c], m, cfg, cdf)
        offs = np.zeros(m + 1, dtype=np.int64)
        np.cumsum(lens, out=offs[1:])
        a, b = max(lo, start), min(lo + m, start + n)
        parts[c] = (lens[a - lo:b - lo], terms[offs[a - lo]:offs[b - lo]])

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(work, chunks))
    lens = np.concatenate([parts[c][0] for c in chunks])
    terms = np.concatenate([parts[c][1] for c in chunks])
    off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens, out=off[1:])
    return off, terms


def doc_ids(cfg: Config, n: Optional[int] = None, start: int = 0) -> np.ndarray:
    """External ids: a fixed odd-multiplier scramble of the row index, so ids
    are unique, < 2^32-1 and not in row order (tie-breaks must use the id)."""
    n = cfg.n_docs - start if n is None else n
    r = np.arange(start, start + n, dtype=np.uint64)
    return ((r * np.uint64(2654435761)) % np.uint64(4294967291)).astype(np.uint32)


def doc_frequency(cfg: Config, off: np.ndarray, terms: np.ndarray) -> np.ndarray:
    """Fraction of docs holding each term (a count, not a predicate)."""
    n = len(off) - 1
    return np.bincount(terms, minlength=cfg.vocab).astype(np.float64) / max(n, 1)


# --------------------------------------------------------------------------
# queries
# --------------------------------------------------------------------------

@dataclasses.dataclass
class QueryBatch:
    emb: np.ndarray               # f32 [Q, d]
    clause_off: np.ndarray        # u32 [Q+1]   clauses of query q
    literal_off: np.ndarray       # u32 [C+1]   literals of clause c
    terms: np.ndarray             # u32 [L]
    k: np.ndarray                 # u32 [Q]
    target_sel: np.ndarray        # f64 [Q] (nan for untuned)
    est_sel: np.ndarray           # f64 [Q] independence estimate (nan for untuned)

    @property
    def n(self) -> int:
        return len(self.k)

    def cnf(self, q: int) -> List[List[int]]:
        out = []
        for c in range(int(self.clause_off[q]), int(self.clause_off[q + 1])):
            a, b = int(self.literal_off[c]), int(self.literal_off[c + 1])
            out.append([int(t) for t in self.terms[a:b]])
        return out

    def subset(self, idx: Sequence[int]) -> "QueryBatch":
        return from_cnf_lists(self.emb[list(idx)], [self.cnf(q) for q in idx],
                              self.k[list(idx)], self.target_sel[list(idx)],
                              self.est_sel[list(idx)])


def from_cnf_lists(emb: np.ndarray, cnfs: Sequence[Sequence[Sequence[int]]],
                   k: Sequence[int], target: Optional[Sequence[float]] = None,
                   est: Optional[Sequence[float]] = None) -> QueryBatch:
    co, lo, tt = [0], [0], []
    for cnf in cnfs:
        for clause in cnf:
            tt.extend(int(t) for t in clause)
            lo.append(len(tt))
        co.append(len(lo) - 1)
    q = len(cnfs)
    nan = np.full(q, np.nan)
    return QueryBatch(np.ascontiguousarray(emb, dtype=np.float32),
                      np.asarray(co, dtype=np.uint32), np.asarray(lo, dtype=np.uint32),
                      np.asarray(tt, dtype=np.uint32), np.asarray(k, dtype=np.uint32),
                      nan.copy() if target is None else np.asarray(target, dtype=np.float64),
                      nan.copy() if est is None else np.asarray(est, dtype=np.float64))


def _clause_est(df: np.ndarray, clause: Sequence[int]) -> float:
    return 1.0 - float(np.prod(1.0 - df[list(clause)]))


def _tune_cnf(g: np.random.Generator, df: np.ndarray, order: np.ndarray,
              target: float, cfg: Config) -> Tuple[List[List[int]], float]:
    """Pick a CNF whose independence-estimated selectivity is near target."""
    dfs = df[order]                                 # descending df
    m_lo, m_hi = cfg.clauses
    if target >= 0.05:
        m = int(g.integers(m_lo, min(2, m_hi) + 1))
    elif target >= 1e-3:
        m = int(g.integers(max(2, m_lo), m_hi + 1))
    else:
        m = m_hi
    best, best_err = None, np.inf
    for _attempt in range(24):
        cnf = []
        per_clause = target ** (1.0 / m)
        for _c in range(m):
            n_lit = int(g.integers(cfg.literals[0], cfg.literals[1] + 1))
            p = 1.0 - (1.0 - per_clause) ** (1.0 / n_lit)
            pos = int(np.searchsorted(-dfs, -p))          # first df <= p
            lo = max(0, pos - 8)
            hi = min(len(order), pos + 8)
            pool = order[lo:hi]
            take = g.choice(pool, size=min(n_lit, len(pool)), replace=False)
            cnf.append(sorted(int(t) for t in take))
        est = float(np.prod([_clause_est(df, c) for c in cnf]))
        err = abs(math.log(max(est, 1e-300) / target))
        if err < best_err:
            best, best_err = cnf, err
        if err <= math.log(1.25):
            break
    est = float(np.prod([_clause_est(df, c) for c in best]))
    return best, est


def queries(cfg: Config, df: Optional[np.ndarray] = None,
            n_queries: Optional[int] = None) -> QueryBatch:
    """Query embeddings, CNF predicates and per-query K for ``cfg``.

    ``df`` (per-term document frequency of the corpus) is required for tuned
    configs; the tiny config draws its CNFs freely from the Zipf law.
    """
    q = cfg.n_queries if n_queries is None else n_queries
    ch = _children(cfg)
    emb = _normal_rows(ch[_S_QEMB], q, cfg.dim)
    g = np.random.Generator(np.random.PCG64(ch[_S_PRED]))
    gk = np.random.Generator(np.random.PCG64(ch[_S_K]))
    k = gk.choice(np.asarray(cfg.k_choices, dtype=np.uint32), size=q)
    cnfs, target, est = [], np.full(q, np.nan), np.full(q, np.nan)
    if cfg.sel_range is None:
        p = zipf_probs(cfg.vocab, cfg.zipf_s)
        for i in range(q):
            m = int(g.integers(cfg.clauses[0], cfg.clauses[1] + 1))
            cnf = []
            for _c in range(m):
                n_lit = int(g.integers(cfg.literals[0], cfg.literals[1] + 1))
                cnf.append(sorted(int(t) for t in g.choice(cfg.vocab, size=n_lit, p=p)))
            cnfs.append(cnf)
    else:
        if df is None:
            raise ValueError("tuned predicates need the corpus document frequencies")
        order = np.argsort(-df, kind="stable")
        lo, hi = cfg.sel_range
        for i in range(q):
            t = math.exp(g.uniform(math.log(lo), math.log(hi)))
            cnf, e = _tune_cnf(g, df, order, t, cfg)
            cnfs.append(cnf)
            target[i], est[i] = t, e
    return from_cnf_lists(emb, cnfs, k, target, est)


# --------------------------------------------------------------------------
# serving workload
# --------------------------------------------------------------------------

@dataclasses.dataclass
class SignProjection:
    """Random draws of a sign-code quantiser: bit j sums the positions
    bin_off[j] .. bin_off[j+1] of (bin_dim, bin_sign)."""
    bin_off: np.ndarray           # u32 [n_bits + 1]
    bin_dim: np.ndarray           # u32 [entries]
    bin_sign: np.ndarray          # f32 [entries], each +1 or -1

    @property
    def n_bits(self) -> int:
        return len(self.bin_off) - 1


def sign_projection(dim: int, n_bits: int = 512, seed: int = 0,
                    bin_size: Optional[int] = None) -> SignProjection:
    """Independent random permutations of the ``dim`` coordinates,
    concatenated and cut into ``n_bits`` bins of ``bin_size`` consecutive
    positions, with a random sign per position.  Default bin size:
    dim // n_bits when that is at least 2 (one permutation, equal bins),
    else 2 (several permutations)."""
    s = bin_size or (dim // n_bits if dim >= 2 * n_bits else 2)
    need = n_bits * s
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, 1000, seed])))
    perms = [g.permutation(dim) for _ in range(-(-need // dim))]
    dims = np.concatenate(perms)[:need].astype(np.uint32)
    signs = np.where(g.random(need) < 0.5, -1.0, 1.0).astype(np.float32)
    off = (np.arange(n_bits + 1, dtype=np.uint64) * s).astype(np.uint32)
    return SignProjection(off, dims, signs)


def arrivals(cfg: Config, rate_qps: float, n: int, level: int = 0) -> np.ndarray:
    """Poisson arrival times (seconds from 0) at ``rate_qps``."""
    seq = _children(cfg)[_S_ARR].spawn(level + 1)[level]
    g = np.random.Generator(np.random.PCG64(seq))
    return np.cumsum(g.exponential(1.0 / rate_qps, size=n))


@dataclasses.dataclass
class UpdateBatch:
    del_ids: np.ndarray           # u32
    ins_ids: np.ndarray           # u32
    ins_emb: np.ndarray           # f32 [n_ins, d]
    ins_term_off: np.ndarray      # u64 [n_ins+1]
    ins_terms: np.ndarray         # u32


def update_log(cfg: Config, live_ids: np.ndarray, n_batches: int,
               per_batch: int) -> List[UpdateBatch]:
    """Batches of half deletes (of currently live ids) and half inserts of
    fresh documents drawn by the corpus recipe, with ids that never collide
    with the initial corpus (rows numbered from ``cfg.n_docs`` upward)."""
    seeds = _children(cfg)[_S_UPD].spawn(2 * n_batches + 1)
    g = np.random.Generator(np.random.PCG64(seeds[0]))
    cdf = np.cumsum(zipf_probs(cfg.vocab, cfg.zipf_s))
    live = list(int(i) for i in live_ids)
    row = cfg.n_docs
    out = []
    for b in range(n_batches):
        n_del = min(per_batch // 2, len(live))
        n_ins = per_batch - per_batch // 2
        pick = g.choice(len(live), size=n_del, replace=False)
        dels = np.asarray(sorted(live[i] for i in pick), dtype=np.uint32)
        dset = set(int(x) for x in dels)
        live = [x for x in live if x not in dset]
        emb = _normal_rows(seeds[1 + 2 * b], n_ins, cfg.dim)
        lens, terms = _term_rows(seeds[2 + 2 * b], n_ins, cfg, cdf)
        off = np.zeros(n_ins + 1, dtype=np.uint64)
        np.cumsum(lens, out=off[1:])
        r = np.arange(row, row + n_ins, dtype=np.uint64)
        ids = ((r * np.uint64(2654435761)) % np.uint64(4294967291)).astype(np.uint32)
        row += n_ins
        live.extend(int(i) for i in ids)
        out.append(UpdateBatch(dels, ids, emb, off, terms))
    return out


@dataclasses.dataclass
class Corpus:
    cfg: Config
    emb: np.ndarray
    ids: np.ndarray
    term_off: np.ndarray
    terms: np.ndarray

    @property
    def n(self) -> int:
        return len(self.ids)


def corpus(cfg: Config) -> Corpus:
    return Corpus(cfg, embeddings(cfg), doc_ids(cfg), *doc_terms(cfg))


def workload(name: str, n_docs: Optional[int] = None,
             n_queries: Optional[int] = None) -> Tuple[Corpus, QueryBatch]:
    """Corpus + query batch of a named config, optionally resized."""
    cfg = CONFIGS[name]
    if n_docs is not None or n_queries is not None:
        cfg = scaled(cfg, n_docs or cfg.n_docs, n_queries or cfg.n_queries)
    c = corpus(cfg)
    df = doc_frequency(cfg, c.term_off, c.terms) if cfg.sel_range else None
    return c, queries(cfg, df)
