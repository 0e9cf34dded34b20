"""GPU parity of sparse routing (FR_STRAT_SPARSE): queries with few matches
skip the scan, their matching rows are listed from the masks and scored one
by one; results must equal the plain definition (the oracle) exactly as the
scan's do, whatever the level, dtype or batch composition."""
import numpy as np
import pytest

import datagen
from oracle import recall_at_k, tolerance
from helpers import check_query, gpu_index, oracle_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mid():
    # the fp32 recipe (selectivity 0.1%-50%) at a ragged 100,003 documents
    cfg = datagen.scaled(datagen.CONFIGS["fp32"], 100_003, 256)
    c = datagen.corpus(cfg)
    qb = datagen.queries(cfg, datagen.doc_frequency(cfg, c.term_off, c.terms))
    return c, qb, oracle_for(c)


def _strat(level):
    from paper_2402_13435_amd.binding import FR_STRAT_NO_REFRESH, FR_STRAT_SPARSE
    return FR_STRAT_NO_REFRESH | FR_STRAT_SPARSE(level)


@pytest.mark.parametrize("level", [3, 5, 7])
def test_f32_routing_matches_oracle(mid, level):
    c, qb, o = mid
    ix = gpu_index(c, k_max=100, max_batch=256)
    ix.set_strategy(_strat(level), pinned=True)
    res = ix.search(qb.emb, qb, 100)
    st = ix.stats()
    limit = c.n * 2.0 ** (level - 11)
    routed = int(np.sum(res.n_match.astype(np.float64) <= limit))
    assert st.n_sparse == routed and routed > 0
    for q in range(qb.n):
        check_query(o, qb, q, res, 100)
    # the routed queries' rows in a batch of their own (the scan gets none)
    few = [q for q in range(qb.n) if res.n_match[q] <= limit][:40]
    sub = qb.subset(few)
    r2 = ix.search(sub.emb, sub, 100)
    assert ix.stats().n_sparse == len(few)
    for i, q in enumerate(few):
        assert np.array_equal(r2.ids[i], res.ids[q]) and np.array_equal(r2.scores[i], res.scores[q])
    ix.close()


def test_routing_keeps_the_scan_results_of_the_other_queries(mid):
    c, qb, o = mid
    ix = gpu_index(c, k_max=100, max_batch=256)
    ix.set_strategy(_strat(0), pinned=True)
    plain = ix.search(qb.emb, qb, 100)
    ix.set_strategy(_strat(5), pinned=True)
    routed = ix.search(qb.emb, qb, 100)
    lim = c.n * 2.0 ** (5 - 11)
    for q in range(qb.n):
        assert routed.n_match[q] == plain.n_match[q] and routed.count[q] == plain.count[q]
        if plain.n_match[q] > lim:    # still scanned: the same MFMA arithmetic
            assert np.array_equal(routed.ids[q], plain.ids[q])
            assert np.array_equal(routed.scores[q], plain.scores[q])
        else:                          # FP32 row by row: same ids up to near-ties
            tol = tolerance(c.cfg.dim)
            n = int(plain.count[q])
            assert np.abs(routed.scores[q, :n] - plain.scores[q, :n]).max(initial=0) <= 2 * tol
    ix.close()


@pytest.mark.parametrize("dt", ["bf16", "fp8"])
def test_reduced_precision_routes_only_within_r(mid, dt):
    c, qb, o = mid
    k, r = 100, 1024
    ix = gpu_index(c, k_max=k, dtype=dt, rescore_r=r, max_batch=256)
    ix.set_strategy(_strat(7), pinned=True)
    res = ix.search(qb.emb, qb, k)
    st = ix.stats()
    limit = min(c.n * 2.0 ** (7 - 11), r)
    assert st.n_sparse == int(np.sum(res.n_match.astype(np.float64) <= limit))
    got, want = [], []
    tol = tolerance(c.cfg.dim)
    for q in range(qb.n):
        a = o.search_one(qb.emb[q], qb.cnf(q), k)
        cnt = int(res.count[q])
        assert cnt == a.count and res.n_match[q] == a.n_match
        if res.n_match[q] <= limit:
            check_query(o, qb, q, res, k)          # all matches scored in FP32: exact
        elif cnt:
            s = res.scores[q, :cnt].astype(np.float64)
            assert np.abs(s - o.score_ids(qb.emb[q], res.ids[q, :cnt])).max() <= tol
        got.append(res.ids[q, :cnt].tolist())
        want.append(a.ids.tolist())
    rec, _ = recall_at_k(got, want)
    assert rec >= 0.99, rec
    ix.close()


def test_all_queries_routed_and_graph_replay(mid):
    torch = pytest.importorskip("torch")
    from paper_2402_13435_amd import SearchResult
    c, qb, o = mid
    ix = gpu_index(c, k_max=50, max_batch=256, n_workspaces=2)
    ix.set_strategy(_strat(7), pinned=True)
    sel = [q for q in range(qb.n)][:64]
    sub = qb.subset(sel)
    # every query of a selective batch routed: the scan's list is empty
    lim = c.n * 2.0 ** (7 - 11)
    few = [q for q in range(qb.n) if o.match_rows(qb.cnf(q)).size <= lim][:33]
    fb = qb.subset(few)
    res = ix.search(fb.emb, fb, 50)
    assert ix.stats().n_sparse == len(few)
    for i in range(fb.n):
        check_query(o, fb, i, res, 50)
    # captured and replayed, with eager searches in between
    d = torch.device("cuda")
    q = torch.from_numpy(sub.emb).to(d)
    out = SearchResult(torch.empty((sub.n, 50), dtype=torch.int32, device=d),
                       torch.empty((sub.n, 50), dtype=torch.float32, device=d),
                       torch.empty(sub.n, dtype=torch.int32, device=d),
                       torch.empty(sub.n, dtype=torch.int64, device=d))
    s = torch.cuda.Stream()
    eager = ix.search(sub.emb, sub, 50)
    for _ in range(3):
        ix.search(q, sub, 50, out=out, stream=s, graph=True)
        s.synchronize()
        assert np.array_equal(out.ids.cpu().numpy().view(np.uint32), eager.ids)
        assert np.array_equal(out.scores.cpu().numpy(), eager.scores)
        ix.search(fb.emb, fb, 50)
    ix.close()


def test_autotuner_may_choose_routing(mid, tmp_path):
    c, qb, o = mid
    ix = gpu_index(c, k_max=100, max_batch=256)
    qbl, nw, g, strat = ix.autotune(qb.emb, qb, 100)
    res = ix.search(qb.emb, qb, 100)
    for q in range(0, qb.n, 4):
        check_query(o, qb, q, res, 100)
    path = str(tmp_path / "t.jsonl")
    ix.tuning_save(path)
    ix2 = gpu_index(c, k_max=100, max_batch=256)
    assert ix2.tuning_load(path) == 1
    assert ix2.tuning_choice(qb.n, np.full(qb.n, 100, np.uint32))[3] == strat
    ix.close()
    ix2.close()
