"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Masks and ids are compared bit-exactly where the result is unique; scores
within tol_d = 2 gamma_d (the FP32 dot-product bound for unit vectors); the
top-K set exactly except for near-ties inside that tolerance (the checker's
rule).
"""
import numpy as np
import pytest

import datagen
from oracle import quant, recall_at_k, tolerance
from helpers import check_query, gpu_index, masks_as_bytes, oracle_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    c, qb = datagen.workload("tiny")
    return c, qb, oracle_for(c)


@pytest.fixture(scope="module")
def mid():
    # the fp32 recipe (d=128, V=4096, 16-48 terms, sel 0.1%-50%) at a ragged
    # 100,003 documents: 98 predicate groups, the last one partial
    cfg = datagen.scaled(datagen.CONFIGS["fp32"], 100_003, 256)
    c = datagen.corpus(cfg)
    qb = datagen.queries(cfg, datagen.doc_frequency(cfg, c.term_off, c.terms))
    return c, qb, oracle_for(c)


def test_tiny_f32_all_queries(tiny):
    c, qb, o = tiny
    ix = gpu_index(c, k_max=64)
    for k in (10, 1, 64):
        res = ix.search(qb.emb, qb, k)
        for q in range(qb.n):
            check_query(o, qb, q, res, k)


def test_tiny_masks_bit_exact(tiny):
    c, qb, o = tiny
    ix = gpu_index(c, k_max=10)
    words = ix.debug_masks(qb)
    for q in range(qb.n):
        want = o.match_bitmap(qb.cnf(q))
        assert np.array_equal(masks_as_bytes(words[q], c.n), want), q


def test_mid_f32_all_queries(mid):
    c, qb, o = mid
    ix = gpu_index(c, k_max=100, max_batch=256)
    res = ix.search(qb.emb, qb, 100)
    words = ix.debug_masks(qb)
    for q in range(qb.n):
        check_query(o, qb, q, res, 100)
    for q in range(0, qb.n, 16):
        assert np.array_equal(masks_as_bytes(words[q], c.n), o.match_bitmap(qb.cnf(q))), q


def test_unit_queries_give_exact_scores(tiny):
    c, qb, o = tiny
    ix = gpu_index(c, k_max=50)
    dims = [0, 5, 31, 32, 63]
    e = np.zeros((len(dims), c.cfg.dim), np.float32)
    for i, d in enumerate(dims):
        e[i, d] = 1.0
    cnf = datagen.from_cnf_lists(e, [[]] * len(dims), [50] * len(dims))
    res = ix.search(e, cnf, 50)
    for i, d in enumerate(dims):
        col = c.emb[:, d]
        order = np.lexsort((c.ids, -col.astype(np.float64)))[:50]
        assert np.array_equal(res.ids[i, :50], c.ids[order])
        assert np.array_equal(res.scores[i, :50], col[order])       # bit-exact


def test_edge_cases():
    from paper_2402_13435_amd import Index
    rng = np.random.default_rng(7)
    d, v = 64, 40
    # empty corpus
    ix = Index(5000, d, v, 8)
    q = rng.standard_normal((3, d)).astype(np.float32)
    res = ix.search(q, datagen.from_cnf_lists(q, [[], [[1]], [[]]], [8] * 3), 8)
    assert res.count.tolist() == [0, 0, 0] and res.n_match.tolist() == [0, 0, 0]
    assert np.all(res.ids == 0xFFFFFFFF) and np.all(np.isneginf(res.scores))
    # ragged 1,037 docs, every doc holds term 0; odd ones term 1
    n = 1037
    emb = rng.standard_normal((n, d)).astype(np.float32)
    ids = rng.permutation(10 ** 6)[:n].astype(np.uint32)
    lists = [[0, 1] if i % 2 else [0] for i in range(n)]
    off = np.cumsum([0] + [len(x) for x in lists]).astype(np.uint64)
    terms = np.concatenate([np.asarray(x, np.uint32) for x in lists])
    ix.load_corpus(emb, ids, off, terms)
    cnfs = [[], [[]], [[0]], [[1]], [[1], [0]], [[2]], [[1, 2], [0, 39]]]
    qs = rng.standard_normal((len(cnfs), d)).astype(np.float32)
    for k in (0, 1, 8):
        res = ix.search(qs, datagen.from_cnf_lists(qs, cnfs, [k] * len(cnfs)), k)
        want_nm = [n, 0, n, n // 2, n // 2, 0, n // 2]
        assert res.n_match.tolist() == want_nm
        assert res.count.tolist() == [min(k, x) for x in want_nm]
        for qi in range(len(cnfs)):
            cnt = int(res.count[qi])
            got = res.ids[qi, :cnt]
            if cnfs[qi] in ([[1]], [[1], [0]], [[1, 2], [0, 39]]):
                pos = np.searchsorted(np.sort(ids), got)
                assert all((np.flatnonzero(ids == g)[0] % 2) == 1 for g in got)
            assert np.all(res.ids[qi, cnt:] == 0xFFFFFFFF)
    # K larger than the matches: all of them, in order
    res = ix.search(qs[:1], datagen.from_cnf_lists(qs[:1], [[[5]]], [8]), 8)
    assert res.count[0] == 0
    with pytest.raises(Exception):
        ix.search(qs[:1], datagen.from_cnf_lists(qs[:1], [[[40]]], [8]), 8)   # term >= vocab
    with pytest.raises(Exception):
        ix.search(qs[:1], datagen.from_cnf_lists(qs[:1], [[[0]]], [9]), 9)    # K > k_max
    ix.close()


def test_long_predicates_take_the_general_mask_path(tiny):
    """Queries with more literals than the scan's literal table holds (12)
    are evaluated from the CSR arrays; both paths must agree with the
    oracle bit for bit."""
    c, qb, o = tiny
    ix = gpu_index(c, k_max=10)
    rng = np.random.default_rng(11)
    cnfs = []
    for n_lit in (11, 12, 13, 16, 24):
        terms = rng.choice(c.cfg.vocab, size=n_lit, replace=False).tolist()
        # three clauses: one big OR and two narrower ones
        cut = [n_lit // 3, 2 * n_lit // 3]
        cnfs.append([terms[:cut[0]] + [0, 1, 2], terms[cut[0]:cut[1]] + [3, 4],
                     terms[cut[1]:] + [5]])
    q = qb.emb[:len(cnfs)]
    batch = datagen.from_cnf_lists(q, cnfs, [10] * len(cnfs))
    words = ix.debug_masks(batch)
    res = ix.search(q, batch, 10)
    for i, cnf in enumerate(cnfs):
        assert np.array_equal(masks_as_bytes(words[i], c.n), o.match_bitmap(cnf)), i
        check_query(o, batch, i, res, 10)


def test_duplicate_rows_break_ties_by_id():
    from paper_2402_13435_amd import Index
    rng = np.random.default_rng(3)
    base = rng.standard_normal((40, 64)).astype(np.float32)
    emb = np.concatenate([base] * 5)
    ids = rng.permutation(10 ** 5)[:200].astype(np.uint32)
    off = np.arange(201, dtype=np.uint64)
    ix = Index(1000, 64, 4, 50)
    ix.load_corpus(emb, ids, off, np.zeros(200, np.uint32))
    res = ix.search(base[:4], datagen.from_cnf_lists(base[:4], [[[0]]] * 4, [50] * 4), 50)
    for q in range(4):
        s, i = res.scores[q], res.ids[q]
        for r in range(1, 50):
            assert s[r] < s[r - 1] or (s[r] == s[r - 1] and i[r] > i[r - 1])
        assert s[0] == s[4] and i[0] < i[1] < i[2] < i[3] < i[4]


def test_determinism_and_batch_invariance(mid):
    c, qb, o = mid
    ix = gpu_index(c, k_max=100, max_batch=256)
    a = ix.search(qb.emb, qb, 100)
    b = ix.search(qb.emb, qb, 100)
    assert np.array_equal(a.ids, b.ids) and np.array_equal(a.scores, b.scores)
    for q in (0, 17, 255):
        one = qb.subset([q])
        r = ix.search(one.emb, one, 100)
        assert np.array_equal(r.ids[0], a.ids[q]) and np.array_equal(r.scores[0], a.scores[q])
        assert r.n_match[0] == a.n_match[q]
    # batches that fill 2 and 3 of the 4 compute wavefronts' query blocks
    # (the first shares blocks between wavefronts, the second does not)
    for n in (40, 70):
        idx = list(range(100, 100 + n))
        sub = qb.subset(idx)
        ix.set_tiling(1, 4, 0)
        r = ix.search(sub.emb, sub, 100)
        ix.set_tiling(0, 0, 0)
        assert np.array_equal(r.ids, a.ids[idx]) and np.array_equal(r.scores, a.scores[idx])
        assert np.array_equal(r.n_match, a.n_match[idx])
    for qbk, nw, g in ((1, 4, 1), (2, 4, 2), (1, 4, 7), (1, 8, 3)):
        ix.set_tiling(qbk, nw, g)
        t = ix.search(qb.emb, qb, 100)
        assert np.array_equal(t.ids, a.ids) and np.array_equal(t.scores, a.scores)
        assert np.array_equal(t.n_match, a.n_match)


def test_quantizers_bit_exact(tiny):
    c, qb, o = tiny
    n = c.n
    for dt in ("bf16", "fp8"):
        ix = gpu_index(c, k_max=10, dtype=dt, rescore_r=64)
        codes, scales = ix.debug_rows(0, n)
        if dt == "bf16":
            want = quant.bf16_round(c.emb).view(np.uint32) >> 16
            assert np.array_equal(codes[:, :c.cfg.dim].astype(np.uint32), want)
        else:
            want, ws = quant.fp8_codes(c.emb)
            assert np.array_equal(codes[:, :c.cfg.dim], want)
            assert np.array_equal(scales.view(np.uint32), ws.view(np.uint32))
        assert np.all(codes[:, c.cfg.dim:] == 0)
        ix.close()


@pytest.mark.parametrize("dt", ["bf16", "fp8"])
def test_precision_forms(mid, dt):
    c, qb, o = mid
    k, r = 100, 1024
    ix = gpu_index(c, k_max=k, dtype=dt, rescore_r=r, max_batch=256)
    res = ix.search(qb.emb, qb, k)
    tol = tolerance(c.cfg.dim)
    got, want = [], []
    for q in range(qb.n):
        a = o.search_one(qb.emb[q], qb.cnf(q), k)
        cnt = int(res.count[q])
        assert cnt == a.count and res.n_match[q] == a.n_match
        ids = res.ids[q, :cnt]
        s = res.scores[q, :cnt].astype(np.float64)
        if cnt:
            assert np.abs(s - o.score_ids(qb.emb[q], ids)).max() <= tol       # FP32 rescore
            assert np.all(np.diff(s) <= 0)
        got.append(ids.tolist())
        want.append(a.ids.tolist())
    rec, _ = recall_at_k(got, want)
    assert rec >= 0.99, rec
    if dt == "fp8":
        # another query-block tiling and chunk size give the same answer
        ix.set_tiling(2, 4, 3)
        t = ix.search(qb.emb, qb, k)
        assert np.array_equal(t.ids, res.ids) and np.array_equal(t.scores, res.scores)
        ix.set_tiling(0, 0, 0)
    # first pass: approximate scores against the oracle's emulation
    cid, csc, ccnt = ix.debug_candidates(qb.n)
    for q in range(0, qb.n, 8):
        n = int(ccnt[q])
        assert n == min(r, int(res.n_match[q]))
        if not n:
            continue
        rows = np.array([o.row_of[int(i)] for i in cid[q, :n]])
        approx = o.approx_scores(qb.emb[q], rows, dt)
        assert np.abs(csc[q, :n] - approx).max() <= 2 * tol + 1e-6
        assert np.all(np.diff(csc[q, :n].astype(np.float64)) <= 0)


def test_rescore_covering_all_matches_equals_f32(tiny):
    c, qb, o = tiny
    f = gpu_index(c, k_max=10)
    a = f.search(qb.emb, qb, 10)
    for dt in ("bf16", "fp8"):
        ix = gpu_index(c, k_max=10, dtype=dt, rescore_r=4096)
        b = ix.search(qb.emb, qb, 10)
        for q in range(qb.n):
            if b.n_match[q] <= 4096:
                check_query(o, qb, q, b, 10)
                assert b.count[q] == a.count[q]
        ix.close()


def test_updates_match_rebuilt_oracle():
    cfg = datagen.scaled(datagen.CONFIGS["tiny"], 3000, 16)
    c = datagen.corpus(cfg)
    qb = datagen.queries(cfg)
    o = oracle_for(c)
    ix = gpu_index(c, k_max=20, capacity=3300)
    log = datagen.update_log(cfg, c.ids, 4, 300)
    epoch0 = ix.info()[1]
    for j, u in enumerate(log):
        ep = ix.update_docs(u.del_ids, u.ins_ids, u.ins_emb, u.ins_term_off, u.ins_terms)
        o.update(u.del_ids, u.ins_ids, u.ins_emb, u.ins_term_off, u.ins_terms)
        assert ep == epoch0 + j + 1
        res = ix.search(qb.emb, qb, 20)
        for q in range(qb.n):
            check_query(o, qb, q, res, 20)
        dead = set(int(x) for x in u.del_ids)
        assert not dead & set(res.ids[:, :].ravel().tolist())
    n_live, _, n_slots = ix.info()
    assert n_live == o.n_live and n_slots <= 3300
    # slot table agrees with the oracle's live ids
    slots = ix.debug_slots()
    assert set(int(x) for x in slots if x != 0xFFFFFFFF) == set(int(x) for x in o.ids[o.live])


def test_updates_are_ordered_with_asynchronous_searches():
    """Searches and updates issued with no host synchronisation between them
    (searches asynchronous on two streams, one through the scratch-array
    entry point): each search sees exactly the corpus of its place in the
    call sequence.  Every update deletes each query's current best match, so
    a search on the wrong side of an update returns a wrong row."""
    import copy
    from types import SimpleNamespace
    torch = pytest.importorskip("torch")
    from paper_2402_13435_amd.binding import SearchResult
    cfg = datagen.scaled(datagen.CONFIGS["tiny"], 3000, 16)
    c = datagen.corpus(cfg)
    qb = datagen.queries(cfg)
    o = oracle_for(c)
    ix = gpu_index(c, k_max=20, capacity=3600, n_workspaces=3)
    q = torch.from_numpy(qb.emb).cuda()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    log = datagen.update_log(cfg, c.ids, 4, 200)
    issued = []
    for j in range(5):
        s = streams[j % 2]
        if j == 2:
            out = SearchResult(torch.empty((qb.n, 20), dtype=torch.int32, device="cuda"),
                               torch.empty((qb.n, 20), dtype=torch.float32, device="cuda"),
                               torch.empty(qb.n, dtype=torch.int32, device="cuda"),
                               torch.empty(qb.n, dtype=torch.int64, device="cuda"))
            ix.search_noalloc(q, qb, 20, out, stream=s)
        else:
            out = ix.search(q, qb, 20, stream=s)
        issued.append((out, copy.deepcopy(o)))
        if j == 4:
            break
        best = set()
        for qi in range(qb.n):
            a = o.search_one(qb.emb[qi], qb.cnf(qi), 1)
            best.update(int(x) for x in a.ids[:a.count])
        dels = np.array(sorted(best), np.uint32)
        u = log[j]
        ix.update_docs(dels, u.ins_ids, u.ins_emb, u.ins_term_off, u.ins_terms)
        o.update(dels, u.ins_ids, u.ins_emb, u.ins_term_off, u.ins_terms)
    torch.cuda.synchronize()
    for out, snap in issued:
        res = SimpleNamespace(ids=out.ids.cpu().numpy().view(np.uint32),
                              scores=out.scores.cpu().numpy(),
                              count=out.count.cpu().numpy().view(np.uint32),
                              n_match=out.n_match.cpu().numpy().astype(np.uint64))
        for qi in range(qb.n):
            check_query(snap, qb, qi, res, 20)
    # the host term store cleared exactly the deleted documents' bits
    full = ix.search(qb.emb, qb, 20)
    for qi in range(qb.n):
        check_query(o, qb, qi, full, 20)
    ix.close()


def test_update_errors_leave_index_unchanged(tiny):
    from paper_2402_13435_amd import FrError
    from paper_2402_13435_amd.binding import FR_ECAPACITY, FR_EDUPID, FR_ENOTFOUND
    c, qb, o = tiny
    ix = gpu_index(c, k_max=10, capacity=c.n + 5)
    before = ix.search(qb.emb, qb, 10)
    info = ix.info()
    d = c.cfg.dim
    one = np.zeros((1, d), np.float32)
    bad = [
        (dict(del_ids=[123456789], ins_ids=[], ins_emb=np.zeros((0, d)), ins_term_off=[0],
              ins_terms=[]), FR_ENOTFOUND),
        (dict(del_ids=[c.ids[0], c.ids[0]], ins_ids=[], ins_emb=np.zeros((0, d)),
              ins_term_off=[0], ins_terms=[]), FR_ENOTFOUND),
        (dict(del_ids=[], ins_ids=[c.ids[1]], ins_emb=one, ins_term_off=[0, 1],
              ins_terms=[3]), FR_EDUPID),
        (dict(del_ids=[], ins_ids=np.arange(6) + 4000000000, ins_emb=np.zeros((6, d)),
              ins_term_off=np.zeros(7), ins_terms=[]), FR_ECAPACITY),
    ]
    for kw, status in bad:
        with pytest.raises(FrError) as e:
            ix.update_docs(**kw)
        assert e.value.status == status
    assert ix.info() == info
    after = ix.search(qb.emb, qb, 10)
    assert np.array_equal(before.ids, after.ids)
    # delete then re-insert the same id in one call is allowed
    ix.update_docs([c.ids[2]], [c.ids[2]], c.emb[2:3], [0, 2], [1, 2])


def test_candidate_overflow_second_pass_and_tie_limit():
    from paper_2402_13435_amd import FrError, Index
    from paper_2402_13435_amd.binding import FR_EUNSUPPORTED
    # 34 predicate groups, every document matches; the query is e_0 and a
    # document's score is its first coordinate: ~0 in the first 32 groups
    # (the sample the starting threshold comes from), spread over 0.5..0.99
    # in the last two.  The starting threshold is therefore low, the last
    # groups append far more than the 64-entry buffer holds, and the second
    # pass (from the first pass's histogram) fits.
    n_sample = 32 * 1024
    cfg = datagen.scaled(datagen.CONFIGS["tiny"], n_sample + 2048, 4)
    rng = np.random.default_rng(7)
    n, d = n_sample + 2048, cfg.dim
    emb = rng.standard_normal((n, d)).astype(np.float32)
    emb[:, 0] = 0.0
    emb /= np.linalg.norm(emb, axis=1, keepdims=True)
    hi = np.linspace(0.5, 0.99, 2048, dtype=np.float64)
    rng.shuffle(hi)
    emb[n_sample:] *= np.sqrt(1.0 - hi ** 2)[:, None].astype(np.float32)
    emb[n_sample:, 0] = hi.astype(np.float32)
    ids = np.arange(n, dtype=np.uint32) * 3 + 1
    term_off = np.arange(n + 1, dtype=np.int64)
    terms = np.zeros(n, np.uint32)
    from types import SimpleNamespace
    c = SimpleNamespace(emb=emb, ids=ids, term_off=term_off, terms=terms, n=n, cfg=cfg)
    o = oracle_for(c)
    ix = gpu_index(c, k_max=16, cand_cap=64)
    qe = np.zeros((4, d), np.float32)
    qe[:, 0] = 1.0
    empty = datagen.from_cnf_lists(qe, [[]] * 4, [16] * 4)
    res = ix.search(qe, empty, 16)
    assert ix.stats().n_passes == 2
    for q in range(4):
        check_query(o, empty, q, res, 16)
    # 200 identical rows tie above any threshold: more than the buffer holds
    emb = np.repeat(c.emb[:1], 200, axis=0)
    ix2 = Index(1000, cfg.dim, cfg.vocab, 16, cand_cap=64)
    ix2.load_corpus(emb, np.arange(200, dtype=np.uint32), np.arange(201), np.zeros(200, np.uint32))
    with pytest.raises(FrError) as e:
        ix2.search(c.emb[:1], datagen.from_cnf_lists(c.emb[:1], [[]], [16]), 16)
    assert e.value.status == FR_EUNSUPPORTED
    ok = ix2.search(c.emb[:1], datagen.from_cnf_lists(c.emb[:1], [[[5]]], [16]), 16)
    assert ok.count[0] == 0


def test_device_pointers_and_stream(tiny):
    torch = pytest.importorskip("torch")
    c, qb, o = tiny
    from paper_2402_13435_amd import Index
    ix = Index(c.n, c.cfg.dim, c.cfg.vocab, 10, n_workspaces=2)
    ix.load_corpus(torch.from_numpy(c.emb).cuda(), torch.from_numpy(c.ids.view(np.int32)).cuda(),
                   c.term_off, c.terms)
    q = torch.from_numpy(qb.emb).cuda()
    s = torch.cuda.Stream()
    out = ix.search(q, qb, 10, stream=s)
    s.synchronize()
    host = ix.search(qb.emb, qb, 10)
    assert np.array_equal(out.ids.cpu().numpy().view(np.uint32), host.ids)
    assert np.array_equal(out.scores.cpu().numpy(), host.scores)
    assert np.array_equal(out.n_match.cpu().numpy().astype(np.uint64), host.n_match)
    # the null (default) stream: enqueued asynchronously (FR_ASYNC), same result
    d = torch.cuda.current_stream()
    assert d.cuda_stream == 0
    out2 = ix.search(q, qb, 10, stream=d)
    torch.cuda.synchronize()
    assert np.array_equal(out2.ids.cpu().numpy().view(np.uint32), host.ids)
    assert np.array_equal(out2.scores.cpu().numpy(), host.scores)
    # a graph cannot be captured on the null stream
    from paper_2402_13435_amd import FrError
    from paper_2402_13435_amd.binding import FR_EINVAL
    with pytest.raises(FrError) as e:
        ix.search(q, qb, 10, stream=d, graph=True)
    assert e.value.status == FR_EINVAL
    ix.close()


def test_graph_replays_match_eager(mid):
    """The captured search graph replayed several times, with eager searches
    and different batch sizes in between, gives the eager result each time."""
    c, qb, o = mid
    ix = gpu_index(c, k_max=100, max_batch=256)
    eager = ix.search(qb.emb, qb, 100)
    sub = qb.subset(list(range(40)))
    for rep in range(4):
        g = ix.search(qb.emb, qb, 100, graph=True)
        assert np.array_equal(g.ids, eager.ids) and np.array_equal(g.scores, eager.scores)
        assert np.array_equal(g.n_match, eager.n_match) and np.array_equal(g.count, eager.count)
        small = ix.search(sub.emb, sub, 100, graph=True)
        assert np.array_equal(small.ids, eager.ids[:40])
        e2 = ix.search(sub.emb, sub, 100)
        assert np.array_equal(e2.ids, eager.ids[:40])
