"""GPU parity of the scan's less common paths, through the C ABI, against
the FP64 oracle:

* work items: several per workgroup, switching query tiles (batches larger
  than one query tile, one group per item);
* 8-wavefront tilings with query-block sharing (batches of 1 .. 300);
* mixed per-query K up to 1000 (FP32 checker; BF16 with a per-query
  rescoring depth), the autotuned tiling and the captured graph;
* the exact selection's radix-select fallback (more than 8192 candidates at
  or above the final threshold, from a block of tied scores);
* thresholds over negative scores (the histogram spans [-|q| max|x|, +...]);
* a speculative starting threshold that proves too high (second pass from
  the safe one);
* the failure marker of a query that cannot be answered, on synchronous,
  device-pointer and asynchronous searches.
"""
from types import SimpleNamespace

import numpy as np
import pytest

import datagen
from oracle import recall_at_k, tolerance
from helpers import check_query, gpu_index, oracle_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    # the fp32 recipe at 300,001 documents (293 predicate groups, the last
    # partial) and 512 queries
    cfg = datagen.scaled(datagen.CONFIGS["fp32"], 300_001, 512)
    c = datagen.corpus(cfg)
    qb = datagen.queries(cfg, datagen.doc_frequency(cfg, c.term_off, c.terms))
    return c, qb, oracle_for(c)


def test_many_items_per_workgroup_and_query_tile_switch(big):
    """Tiling (1, 4, 1): 128 queries per tile -> 4 query tiles x 293 one-group
    items = 1172 items over the persistent workgroups (about 4.6 each), so
    workgroups take several items and switch query tiles between them."""
    c, qb, o = big
    ix = gpu_index(c, k_max=100, max_batch=512)
    ix.set_tiling(1, 4, 1)
    res = ix.search(qb.emb, qb, 100)
    print(f"[paths] (1,4,1): {ix.stats().n_passes} pass(es)", flush=True)
    for q in range(qb.n):
        check_query(o, qb, q, res, 100)
    # other tilings (query tiles of 256 and 128 queries, several groups per
    # item, the default) give the same rows bit for bit
    for til in ((1, 8, 1), (2, 4, 3), (1, 8, 4), (0, 0, 0)):
        ix.set_tiling(*til)
        t = ix.search(qb.emb, qb, 100)
        assert np.array_equal(t.ids, res.ids), til
        assert np.array_equal(t.scores, res.scores), til
        assert np.array_equal(t.n_match, res.n_match), til
    ix.close()


def test_eight_wave_query_block_sharing(big):
    """With 8 compute wavefronts a batch of 1, 32 or 64 queries fills 1 or 2
    of the 8 query blocks, which the idle wavefronts share (tile stride 8 or
    4); 300 queries leave the second query tile partial.  Every sub-batch's
    rows equal the full batch's."""
    c, qb, o = big
    ix = gpu_index(c, k_max=100, max_batch=512)
    ix.set_tiling(1, 8, 4)
    full = ix.search(qb.emb, qb, 100)
    for q in range(0, qb.n, 37):
        check_query(o, qb, q, full, 100)
    for n, g in ((1, 4), (32, 4), (64, 1), (300, 4), (300, 1)):
        idx = list(range(7, 7 + n))
        sub = qb.subset(idx)
        ix.set_tiling(1, 8, g)
        r = ix.search(sub.emb, sub, 100)
        assert np.array_equal(r.ids, full.ids[idx]), (n, g)
        assert np.array_equal(r.scores, full.scores[idx]), (n, g)
        assert np.array_equal(r.n_match, full.n_match[idx]), (n, g)
    ix.close()


@pytest.fixture(scope="module")
def mixed():
    # the batching recipe (V=16384, selectivity 1e-5..0.5, K in {10,100,1000})
    # at 200,000 documents and 192 queries
    cfg = datagen.scaled(datagen.CONFIGS["batching"], 200_000, 192)
    c = datagen.corpus(cfg)
    qb = datagen.queries(cfg, datagen.doc_frequency(cfg, c.term_off, c.terms))
    assert set(np.unique(qb.k).tolist()) == {10, 100, 1000}
    return c, qb, oracle_for(c)


def test_mixed_k_f32_autotuned(mixed, tmp_path):
    """Every search strategy without sparse routing, and the autotuned
    configuration when it does not route, give the default configuration's
    rows bit for bit (with routing, the routed queries' scores come from
    another FP32 summation order: checked against the oracle instead); the
    tuning table saved by one index is loaded by another and used by its
    searches."""
    from paper_2402_13435_amd.binding import FR_STRAT_NO_REFRESH, FR_STRAT_NO_SPECULATION
    c, qb, o = mixed
    ix = gpu_index(c, k_max=1000, max_batch=256)
    default = ix.search(qb.emb, qb, qb.k)
    for q in range(qb.n):
        check_query(o, qb, q, default, int(qb.k[q]))

    def same(r):
        return (np.array_equal(r.ids, default.ids) and np.array_equal(r.scores, default.scores)
                and np.array_equal(r.count, default.count)
                and np.array_equal(r.n_match, default.n_match))
    for strat in (FR_STRAT_NO_SPECULATION, FR_STRAT_NO_REFRESH,
                  FR_STRAT_NO_SPECULATION | FR_STRAT_NO_REFRESH):
        ix.set_strategy(strat, pinned=True)
        assert same(ix.search(qb.emb, qb, qb.k)), strat
    ix.set_strategy(0, pinned=False)
    til = ix.autotune(qb.emb, qb, qb.k)
    print(f"[paths] autotuned (query_blocks, waves, groups, strategy) {til}", flush=True)
    routes = (til[3] & 0xF0) != 0

    def same_or_exact(r):
        if not routes:
            return same(r)
        assert np.array_equal(r.count, default.count) and np.array_equal(r.n_match, default.n_match)
        for q in range(qb.n):
            check_query(o, qb, q, r, int(qb.k[q]))
        return True
    assert same_or_exact(ix.search(qb.emb, qb, qb.k))
    path = str(tmp_path / "tuning.jsonl")
    ix.tuning_save(path)
    ix.close()
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and '"strategy": %d' % til[3] in lines[0]
    ix2 = gpu_index(c, k_max=1000, max_batch=256)
    assert ix2.tuning_load(path) == 1
    assert same_or_exact(ix2.search(qb.emb, qb, qb.k))
    ix2.close()


def test_mixed_k_bf16_rescore_min_graph(mixed):
    """BF16 first pass with R_q = min(4096, max(1024, 4 K_q)) rescored in
    FP32; the autotuned tiling; eager and graph replays agree bit for bit."""
    torch = pytest.importorskip("torch")
    c, qb, o = mixed
    tol = tolerance(c.cfg.dim)
    ix = gpu_index(c, k_max=1000, dtype="bf16", rescore_r=4096, rescore_min=1024,
                   max_batch=256, n_workspaces=2)
    ix.autotune(qb.emb, qb, qb.k)
    res = ix.search(qb.emb, qb, qb.k)
    got, want = [], []
    for q in range(qb.n):
        k = int(qb.k[q])
        a = o.search_one(qb.emb[q], qb.cnf(q), k)
        cnt = int(res.count[q])
        assert cnt == a.count and int(res.n_match[q]) == a.n_match, q
        ids = res.ids[q, :cnt]
        if cnt:
            s = res.scores[q, :cnt].astype(np.float64)
            assert np.abs(s - o.score_ids(qb.emb[q], ids)).max() <= tol, q
            assert np.all(np.diff(s) <= 0)
        got.append(ids.tolist())
        want.append(a.ids.tolist())
    rec, _ = recall_at_k(got, want)
    assert rec >= 0.99, rec
    # the captured graph, replayed, gives the eager rows
    dev = torch.device("cuda:0")
    qd = torch.from_numpy(qb.emb).to(dev)
    s = torch.cuda.Stream()
    for _ in range(3):
        g = ix.search(qd, qb, qb.k, stream=s, graph=True)
        s.synchronize()
        assert len(g.failed()) == 0
        assert np.array_equal(g.ids.cpu().numpy().view(np.uint32), res.ids)
        assert np.array_equal(g.scores.cpu().numpy(), res.scores)
        e = ix.search(qb.emb, qb, qb.k)
        assert np.array_equal(e.ids, res.ids)
    ix.close()


def _tied_corpus(d=64, n_tied=20_000, n_high=3_000, n_rest=17_000, seed=3):
    """Documents scoring exactly 1.0 against e_0 (n_tied copies of e_0),
    some scoring in (0.6, 0.9) and the rest below 0.5; one term each."""
    rng = np.random.default_rng(seed)
    n = n_tied + n_high + n_rest
    emb = np.zeros((n, d), np.float32)
    emb[:n_tied, 0] = 1.0
    x = rng.standard_normal((n_high + n_rest, d))
    x[:, 0] = 0.0
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    h = np.concatenate([rng.uniform(0.6, 0.9, n_high), rng.uniform(-0.5, 0.5, n_rest)])
    x = x * np.sqrt(1.0 - h ** 2)[:, None]
    x[:, 0] = h
    emb[n_tied:] = x.astype(np.float32)
    perm = rng.permutation(n)
    emb = emb[perm]
    ids = (rng.permutation(4 * n)[:n] + 1).astype(np.uint32)
    cfg = datagen.scaled(datagen.CONFIGS["tiny"], n, 2)
    return SimpleNamespace(emb=emb, ids=ids, term_off=np.arange(n + 1, dtype=np.int64),
                           terms=np.zeros(n, np.uint32), n=n, cfg=cfg)


def test_select_radix_fallback_on_ties():
    """20,000 documents tie at score 1.0: with K = 4096 every one of them is
    at or above the final threshold, more than the 8192 the selection sorts
    in LDS, so it takes the radix-select path; the answer is the 4096
    smallest ids among the ties.  A second query (-e_0, no clause) ranks
    the same corpus the other way round in the same batch."""
    c = _tied_corpus()
    o = oracle_for(c)
    ix = gpu_index(c, k_max=4096)
    q = np.zeros((2, c.cfg.dim), np.float32)
    q[0, 0] = 1.0
    q[1, 0] = -1.0
    batch = datagen.from_cnf_lists(q, [[[0]], []], [4096, 4096])
    res = ix.search(q, batch, 4096)
    st = ix.stats()
    print(f"[paths] ties: {st.candidates} candidates, {st.n_passes} pass(es)", flush=True)
    tied = np.sort(c.ids[c.emb[:, 0] == 1.0])
    assert np.array_equal(res.ids[0], tied[:4096])
    assert np.all(res.scores[0] == 1.0)
    for i in range(2):
        check_query(o, batch, i, res, 4096)
    ix.close()


def test_negative_scores_raise_the_threshold():
    """Every match of the query scores below zero, the matches sit outside
    the starting threshold's sample (groups 33-40 of a 40-group corpus), and
    they outnumber the candidate buffer: the threshold must still rise from
    the histogram, so the search answers exactly instead of failing."""
    rng = np.random.default_rng(11)
    d, n_groups = 64, 40
    n = n_groups * 1024
    x = rng.standard_normal((n, d))
    x[:, 0] = 0.0
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    s = rng.uniform(-0.99, -0.4, n)
    x = x * np.sqrt(1.0 - s ** 2)[:, None]
    x[:, 0] = s
    emb = x.astype(np.float32)
    lists = [[0, 1] if i >= 33 * 1024 and i % 2 == 0 else [0] for i in range(n)]
    off = np.cumsum([0] + [len(t) for t in lists]).astype(np.int64)
    terms = np.concatenate([np.asarray(t, np.uint32) for t in lists])
    cfg = datagen.scaled(datagen.CONFIGS["tiny"], n, 2)
    c = SimpleNamespace(emb=emb, ids=np.arange(n, dtype=np.uint32) * 7 + 3, term_off=off,
                        terms=terms, n=n, cfg=cfg)
    o = oracle_for(c)
    ix = gpu_index(c, k_max=16, cand_cap=1024)
    q = np.zeros((2, d), np.float32)
    q[:, 0] = 1.0
    batch = datagen.from_cnf_lists(q, [[[1]], [[1], [0]]], [16, 16])
    res = ix.search(q, batch, 16)
    assert int(res.n_match[0]) == int(np.sum([1 in t for t in lists]))
    for i in range(2):
        check_query(o, batch, i, res, 16)
        assert np.all(res.scores[i, :16] < 0)
    ix.close()


def _front_loaded_corpus(n_groups=320, d=64, seed=13):
    """Scores against e_0: spread over 0.5..0.99 in the first 64 groups (the
    starting-threshold sample of every dtype), over -0.3..0.3 elsewhere.
    Terms: every document has term 0; one in three also has term 1."""
    rng = np.random.default_rng(seed)
    n = n_groups * 1024
    x = rng.standard_normal((n, d))
    x[:, 0] = 0.0
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    s = np.where(np.arange(n) < 64 * 1024, rng.uniform(0.5, 0.99, n), rng.uniform(-0.3, 0.3, n))
    x = x * np.sqrt(1.0 - s ** 2)[:, None]
    x[:, 0] = s
    lists = [[0, 1] if i % 3 == 0 else [0] for i in range(n)]
    off = np.cumsum([0] + [len(t) for t in lists]).astype(np.int64)
    terms = np.concatenate([np.asarray(t, np.uint32) for t in lists])
    cfg = datagen.scaled(datagen.CONFIGS["tiny"], n, 4)
    return SimpleNamespace(emb=x.astype(np.float32), ids=(np.arange(n, dtype=np.uint32) * 5 + 2),
                           term_off=off, terms=terms, n=n, cfg=cfg)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_speculative_start_falls_back_to_the_safe_one(dtype):
    """The starting threshold is first the sample's r-th best score for an r
    well below K' (the sample holds a tenth to a fifth of the matches).  Here
    every top-K' document lies in the sample, so that start is above the
    K'-th best: the first pass collects fewer than K' candidates, and the
    query is scanned again from the safe start (the sample's K'-th best).
    The query ranking the other way (-e_0) and a K=0 query in the same batch
    need no second pass; all of them match the oracle."""
    c = _front_loaded_corpus()
    o = oracle_for(c)
    kw = dict(rescore_r=400) if dtype == "bf16" else {}
    ix = gpu_index(c, k_max=100, dtype=dtype, **kw)
    q = np.zeros((4, c.cfg.dim), np.float32)
    q[0, 0] = q[2, 0] = q[3, 0] = 1.0
    q[1, 0] = -1.0
    batch = datagen.from_cnf_lists(q, [[], [], [[1]], []], [100, 100, 100, 0])
    res = ix.search(q, batch, batch.k)
    st = ix.stats()
    print(f"[paths] speculative fallback ({dtype}): {st.n_passes} passes, "
          f"{st.candidates} candidates", flush=True)
    assert st.n_passes == 2
    if dtype == "f32":
        for i in range(4):
            check_query(o, batch, i, res, int(batch.k[i]))
    else:
        # with q = +-e_0 a document's BF16 first-pass score is exactly
        # bf16(x_0), so the oracle's emulation of the pipeline (top 400 by
        # (approximate desc, id asc), FP32 rescoring, top 100) gives the ids
        tol = tolerance(c.cfg.dim)
        for i in range(4):
            k = int(batch.k[i])
            a = o.search_rescored_one(q[i], batch.cnf(i), k, 400, "bf16")
            cnt = int(res.count[i])
            assert cnt == a.count and int(res.n_match[i]) == a.n_match, i
            assert np.array_equal(res.ids[i, :cnt], a.ids), i
            assert np.all(np.abs(res.scores[i, :cnt] - a.scores) <= tol), i
    ix.close()


def _all_tied_index(torch_dev=False):
    from paper_2402_13435_amd import Index
    rng = np.random.default_rng(2)
    row = rng.standard_normal((1, 64)).astype(np.float32)
    emb = np.repeat(row, 200, axis=0)
    ix = Index(1000, 64, 4, 16, cand_cap=64)
    ix.load_corpus(emb, np.arange(200, dtype=np.uint32), np.arange(201), np.zeros(200, np.uint32))
    return ix, row


def test_failure_marker_on_device_and_async_searches():
    """200 identical rows tie above any threshold and do not fit a 64-entry
    candidate buffer: the query is marked failed (count 0xFFFFFFFF).  A
    synchronous search with device tensors raises like the host one; an
    asynchronous one returns, and the marker is in its counts."""
    torch = pytest.importorskip("torch")
    from paper_2402_13435_amd import FrError
    from paper_2402_13435_amd.binding import FR_EUNSUPPORTED
    ix, row = _all_tied_index()
    batch = datagen.from_cnf_lists(row, [[]], [16])
    with pytest.raises(FrError) as e:
        ix.search(row, batch, 16)
    assert e.value.status == FR_EUNSUPPORTED
    qd = torch.from_numpy(row).cuda()
    with pytest.raises(FrError) as e:
        ix.search(qd, batch, 16)
    assert e.value.status == FR_EUNSUPPORTED
    s = torch.cuda.Stream()
    out = ix.search(qd, batch, 16, stream=s)
    s.synchronize()
    assert out.failed().tolist() == [0]
    with pytest.raises(FrError):
        out.raise_if_failed()
    assert int(out.n_match.cpu()[0]) == 200
    # a query that can be answered on the same index is unaffected
    ok = ix.search(row, datagen.from_cnf_lists(row, [[[3]]], [16]), 16)
    assert ok.count[0] == 0
    ix.close()


def test_server_rejects_bad_requests_and_reports_failed_queries():
    from paper_2402_13435_amd import FrError
    from paper_2402_13435_amd.serve import Server
    ix, row = _all_tied_index()
    srv = Server(ix, max_inflight=1, max_batch=4096)          # clamped to the index's max_batch
    assert srv.max_batch == ix.max_batch
    with pytest.raises(ValueError):
        srv.submit(row[0], [], 17)                       # K > k_max
    with pytest.raises(ValueError):
        srv.submit(row[0], [[4]], 10)                    # term outside the vocabulary
    with pytest.raises(ValueError):
        srv.submit(row[0, :10], [], 10)                  # wrong dimension
    bad = srv.submit(row[0], [], 16)                     # cannot be answered
    with pytest.raises(FrError):
        bad.result(timeout=60)
    good = srv.submit(row[0], [[3]], 16)                 # the server keeps serving
    rep = good.result(timeout=60)
    assert rep.n_match == 0 and len(rep.ids) == 0
    srv.close()
    ix.close()
