"""Continuous batching: results of requests served in mixed, overlapping
batches equal the same requests searched alone."""
import threading
import time
from types import SimpleNamespace

import numpy as np
import pytest

import datagen
from helpers import gpu_index, oracle_for, check_query

pytestmark = pytest.mark.gpu


def test_alone_equals_in_the_mix():
    from paper_2402_13435_amd.serve import Server, latency_summary
    cfg = datagen.scaled(datagen.CONFIGS["fp32"], 50_000, 96)
    c = datagen.corpus(cfg)
    qb = datagen.queries(cfg, datagen.doc_frequency(cfg, c.term_off, c.terms))
    ix = gpu_index(c, k_max=100, max_batch=32, n_workspaces=3)
    rng = np.random.default_rng(5)
    ks = rng.choice([10, 100], size=qb.n)
    alone = []
    for q in range(qb.n):
        one = qb.subset([q])
        r = ix.search(one.emb, one, int(ks[q]))
        alone.append((r.ids[0, :r.count[0]].copy(), r.scores[0, :r.count[0]].copy(),
                      int(r.n_match[0])))
    srv = Server(ix, slots=3, max_batch=32)
    futs = []

    def client():
        for q in range(qb.n):
            futs.append((q, srv.submit(qb.emb[q], qb.cnf(q), int(ks[q]))))
            time.sleep(float(rng.exponential(2e-4)))

    t = threading.Thread(target=client)
    t.start()
    t.join()
    replies = []
    for q, f in futs:
        rep = f.result(timeout=60)
        replies.append(rep)
        ids, sc, nm = alone[q]
        assert np.array_equal(rep.ids, ids), q
        assert np.array_equal(rep.scores, sc), q
        assert rep.n_match == nm
    srv.close()
    assert max(srv.batches) > 1, srv.batches          # requests were batched together
    s = latency_summary(replies)
    assert s["n"] == qb.n and s["p99_ms"] >= s["p50_ms"] > 0


def test_updates_between_batches_are_visible():
    from paper_2402_13435_amd.serve import Server
    cfg = datagen.scaled(datagen.CONFIGS["tiny"], 4000, 16)
    c = datagen.corpus(cfg)
    qb = datagen.queries(cfg)
    o = oracle_for(c)
    ix = gpu_index(c, k_max=10, capacity=5000, max_batch=16, n_workspaces=2)
    srv = Server(ix, slots=2, max_batch=16)
    log = datagen.update_log(cfg, c.ids, 2, 400)
    for u in log:
        srv.update(u.del_ids, u.ins_ids, u.ins_emb, u.ins_term_off, u.ins_terms)
        o.update(u.del_ids, u.ins_ids, u.ins_emb, u.ins_term_off, u.ins_terms)
        futs = [srv.submit(qb.emb[q], qb.cnf(q), 10) for q in range(qb.n)]
        reps = [f.result(timeout=60) for f in futs]
        # the served rows, padded like a search result, through the checker
        ids = np.full((qb.n, 10), 0xFFFFFFFF, np.uint32)
        sc = np.full((qb.n, 10), -np.inf, np.float32)
        for q, rep in enumerate(reps):
            ids[q, :len(rep.ids)] = rep.ids
            sc[q, :len(rep.ids)] = rep.scores
        res = SimpleNamespace(ids=ids, scores=sc,
                              count=np.array([len(r.ids) for r in reps], np.uint32),
                              n_match=np.array([r.n_match for r in reps], np.uint64))
        for q in range(qb.n):
            check_query(o, qb, q, res, 10)
    srv.close()
