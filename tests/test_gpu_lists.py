"""GPU parity of term-list storage (list_terms): predicate masks built from
per-document term lists through per-batch bitmaps of the batch's own terms
must be bit-exact against the oracle, for vocabularies far beyond what
per-term bitmaps can hold, through loads, updates, sparse routing and the
pre-selection path."""
from types import SimpleNamespace

import numpy as np
import pytest

import datagen
from helpers import check_query, gpu_index, masks_as_bytes, oracle_for

pytestmark = pytest.mark.gpu


def _big_vocab_corpus(n=30_011, d=64, vocab=400_000, seed=11):
    """Zipf(1.1) terms over a 400,000-id vocabulary (the bitmaps would take
    50 KB per document), 4-40 terms per document with repeats."""
    rng = np.random.default_rng(seed)
    emb = rng.standard_normal((n, d)).astype(np.float32)
    emb /= np.linalg.norm(emb, axis=1, keepdims=True)
    p = 1.0 / np.arange(1, vocab + 1) ** 1.1
    cdf = np.cumsum(p / p.sum())
    lens = rng.integers(4, 41, size=n)
    terms = np.searchsorted(cdf, rng.random(int(lens.sum())), side="right").astype(np.uint32)
    terms = np.minimum(terms, vocab - 1)
    off = np.zeros(n + 1, np.uint64)
    np.cumsum(lens, out=off[1:])
    ids = ((np.arange(n, dtype=np.uint64) * 2654435761) % 4294967291).astype(np.uint32)
    return SimpleNamespace(n=n, emb=emb, ids=ids, term_off=off, terms=terms,
                           cfg=SimpleNamespace(dim=d, vocab=vocab))


def _queries(c, n_q, seed=12):
    rng = np.random.default_rng(seed)
    emb = rng.standard_normal((n_q, c.cfg.dim)).astype(np.float32)
    emb /= np.linalg.norm(emb, axis=1, keepdims=True)
    head = np.arange(200)                              # frequent terms
    tail = rng.integers(200, c.cfg.vocab, size=4000)  # rare and absent ones
    cnfs = []
    for q in range(n_q):
        n_cl = int(rng.integers(0, 4))
        cnf = []
        for _ in range(n_cl):
            pool = head if rng.random() < 0.6 else tail
            cnf.append(sorted(int(t) for t in rng.choice(pool, size=int(rng.integers(1, 5)))))
        cnfs.append(cnf)
    return datagen.from_cnf_lists(emb, cnfs, [10] * n_q)


@pytest.fixture(scope="module")
def big():
    c = _big_vocab_corpus()
    return c, _queries(c, 70), oracle_for(c)


def test_masks_bit_exact_and_results(big):
    c, qb, o = big
    ix = gpu_index(c, k_max=10, list_terms=40, max_batch=128)
    n_words = (c.n + 63) // 64
    got = ix.debug_masks(qb)
    for q in range(qb.n):
        want = o.match_bitmap(qb.cnf(q))
        assert np.array_equal(masks_as_bytes(got[q], c.n), want), q
    res = ix.search(qb.emb, qb, 10)
    for q in range(qb.n):
        check_query(o, qb, q, res, 10)
    ix.close()


def test_same_results_as_bitmaps_on_a_small_vocabulary():
    c, qb = datagen.workload("tiny")
    a = gpu_index(c, k_max=10)
    b = gpu_index(c, k_max=10, list_terms=int(np.diff(c.term_off.astype(np.int64)).max()))
    ra, rb = a.search(qb.emb, qb, 10), b.search(qb.emb, qb, 10)
    assert np.array_equal(ra.ids, rb.ids) and np.array_equal(ra.scores, rb.scores)
    assert np.array_equal(ra.n_match, rb.n_match)
    a.close()
    b.close()


def test_updates_sparse_routing_and_preselect(big):
    from paper_2402_13435_amd.binding import FR_STRAT_NO_REFRESH, FR_STRAT_SPARSE
    from oracle.signcode import SignCodes
    c, qb, o0 = big
    o = oracle_for(c)
    ix = gpu_index(c, k_max=10, list_terms=40, capacity=c.n + 2000, quant_bits=128,
                   quant_factor=20, max_batch=128)
    p = datagen.sign_projection(c.cfg.dim, 128, seed=13)
    ix.set_quantizer(p.bin_off, p.bin_dim, p.bin_sign)
    rng = np.random.default_rng(14)
    extra = _big_vocab_corpus(n=1500, seed=15)
    live = list(int(x) for x in c.ids)
    for step in range(3):
        dels = np.array(sorted(rng.choice(live, size=500, replace=False)), np.uint32)
        live = [x for x in live if x not in set(dels.tolist())]
        sl = slice(500 * step, 500 * (step + 1))
        ins_ids = (np.arange(500, dtype=np.uint32) + 4_000_000_000 - 1000 * step)
        off = extra.term_off[sl.start:sl.stop + 1] - extra.term_off[sl.start]
        terms = extra.terms[int(extra.term_off[sl.start]):int(extra.term_off[sl.stop])]
        ix.update_docs(dels, ins_ids, extra.emb[sl], off, terms)
        o.update(dels, ins_ids, extra.emb[sl], off, terms)
        live += [int(x) for x in ins_ids]
    res = ix.search(qb.emb, qb, 10)
    for q in range(qb.n):
        check_query(o, qb, q, res, 10)
    ix.set_strategy(FR_STRAT_NO_REFRESH | FR_STRAT_SPARSE(7), pinned=True)
    r2 = ix.search(qb.emb, qb, 10)
    assert ix.stats().n_sparse > 0
    for q in range(qb.n):
        check_query(o, qb, q, r2, 10)
    sc = SignCodes(o, p.bin_off, p.bin_dim, p.bin_sign)
    r3 = ix.search(qb.emb, qb, 10, preselect=True)
    from oracle import check_result, tolerance
    for q in range(qb.n):
        a = sc.search_one(qb.emb[q], qb.cnf(q), 10, 200)
        surv = set(int(o.ids[r]) for r in sc.survivors(qb.emb[q], qb.cnf(q), 200))
        check_result(r3.ids[q], r3.scores[q], int(r3.count[q]), int(r3.n_match[q]),
                     a.ids, a.scores, a.n_match, 10,
                     lambda ids, q=q: o.score_ids(qb.emb[q], ids), lambda i: i in surv,
                     tolerance(o.dim))
    ix.close()


def test_limits():
    from paper_2402_13435_amd import FrError
    from paper_2402_13435_amd.binding import FR_EINVAL
    c = _big_vocab_corpus(n=3000)
    # a document with more terms than list_terms
    from paper_2402_13435_amd import Index
    ix = Index(c.n, c.cfg.dim, c.cfg.vocab, 10, list_terms=8, batch_terms=16)
    with pytest.raises(FrError) as e:
        ix.load_corpus(c.emb, c.ids, c.term_off, c.terms)
    assert e.value.status == FR_EINVAL
    ix.close()
    ix = gpu_index(c, k_max=10, list_terms=40, batch_terms=16)
    qb = datagen.from_cnf_lists(c.emb[:2], [[list(range(10))], [list(range(10, 20))]], [5, 5])
    with pytest.raises(FrError) as e:                   # 20 distinct terms > 16
        ix.search(qb.emb, qb, 5)
    assert e.value.status == FR_EINVAL
    ok = ix.search(qb.emb[:1], qb.subset([0]), 5)       # 10 terms: fine
    o = oracle_for(c)
    check_query(o, qb.subset([0]), 0, ok, 5)
    ix.close()
