"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against the paper's worked examples, a textbook
routine, brute force on tiny inputs, a closed form or an invariant, chosen so
that a plausible slip in the oracle (a dropped clause, OR/AND swapped, a
wrong sign in the sort key, a transposed operand) fails at least one.
"""
import json
import math
import os

import numpy as np
import pytest

import datagen
from oracle import OracleIndex, check_result, recall_at_k, tolerance
from oracle import brute, quant
from oracle.check import CheckError

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def tiny():
    c, qb = datagen.workload("tiny")
    ix = OracleIndex(c.cfg.dim, c.cfg.vocab)
    ix.load(c.emb, c.ids, c.term_off, c.terms)
    return c, qb, ix


def _term_sets(c):
    off = c.term_off.astype(np.int64)
    return [set(int(t) for t in c.terms[off[i]:off[i + 1]]) for i in range(c.n)]


# ----------------------------------------------------------------- F-TBR
def test_paper_tbr_example():
    g = json.load(open(os.path.join(GOLD, "paper_tbr_example.json")))
    base = g["field_base"]
    ids, term_off, terms = [], [0], []
    for d in g["docs"]:
        ids.append(d["id"])
        for f in ("geo", "skill"):
            terms.extend(base[f] + v for v in d[f])
        term_off.append(len(terms))
    # the stored matrix of the example holds the same attribute lists
    for row, d in zip(g["stored_matrix"]["attributes"], g["stored_matrix"]["offsets"]):
        assert d[0] == 0 and d[-1] <= g["stored_matrix"]["max_num_attr"]
    ix = OracleIndex(4, g["vocab"])
    ix.load(np.eye(2, 4, dtype=np.float32), ids, term_off, terms)
    for q in g["queries"]:
        cnf = [[base[f] + v for v in vals] for f, vals in q["cnf"].items()]
        got = sorted(int(ix.ids[r]) for r in ix.match_rows(cnf))
        assert got == q["match"], (q, got)


def test_paper_messenger_example():
    g = json.load(open(os.path.join(GOLD, "paper_messenger_example.json")))
    n = g["n_docs"]
    # term 0 on the single-query rows, terms 1 and 2 on the two batched queries
    lists = [[] for _ in range(n)]
    for r in g["single"]["rows"]:
        lists[r].append(0)
    for t, rows in enumerate(g["batch"]["rows"]):
        for r in rows:
            lists[r].append(1 + t)
    off = np.cumsum([0] + [len(x) for x in lists])
    ix = OracleIndex(2, 3)
    ix.load(np.ones((n, 2), dtype=np.float32), np.arange(n), off,
            np.concatenate([np.asarray(x, dtype=np.uint32) for x in lists]))
    assert ix.match_rows([[0]]).tolist() == g["single"]["rows"]
    per_q = [ix.match_rows([[1 + t]]).tolist() for t in range(2)]
    assert per_q == g["batch"]["rows"]
    messenger = sorted((r, b) for b, rows in enumerate(per_q) for r in rows)
    assert [list(m) for m in messenger] == g["batch"]["messenger"]


def test_mask_matches_brute_force_on_tiny(tiny):
    c, qb, ix = tiny
    sets = _term_sets(c)
    for q in range(qb.n):
        cnf = qb.cnf(q)
        want = [r for r in range(c.n) if brute.matches(sets[r], cnf)]
        assert ix.match_rows(cnf).tolist() == want


def test_mask_closed_forms(tiny):
    c, qb, ix = tiny
    sets = _term_sets(c)
    df = np.zeros(c.cfg.vocab, dtype=np.int64)
    for s in sets:
        for t in s:
            df[t] += 1
    for t in (0, 1, 17, 500, 1023):
        rows = ix.match_rows([[t]])
        assert len(rows) == df[t]                               # posting list
        assert all(t in sets[r] for r in rows)
    assert ix.match_rows([]).tolist() == list(range(c.n))       # no clause: all
    assert len(ix.match_rows([[]])) == 0                        # empty clause: none
    assert len(ix.match_rows([[3], []])) == 0
    a = set(ix.match_rows([[5]]).tolist())
    assert a <= set(ix.match_rows([[5, 9]]).tolist())           # OR widens
    assert set(ix.match_rows([[5], [9, 11]]).tolist()) <= a     # AND narrows
    # duplicate literals change nothing
    assert ix.match_rows([[5, 5], [9, 9]]).tolist() == ix.match_rows([[5], [9]]).tolist()


# ----------------------------------------------------------------- F-EBR
def test_scores_against_fsum(tiny):
    c, qb, ix = tiny
    rows = np.arange(0, c.n, 37)
    for q in range(4):
        s = ix.scores(qb.emb[q], rows)
        for r, v in zip(rows[:60], s[:60]):
            exact = brute.exact_dot(qb.emb[q], c.emb[r])
            bound = math.fsum(abs(float(a) * float(b)) for a, b in zip(qb.emb[q], c.emb[r]))
            assert abs(v - exact) <= 4 * 2.0 ** -53 * 64 * bound


def test_unit_query_scores_are_exact(tiny):
    c, qb, ix = tiny
    rows = np.arange(c.n)
    for k in (0, 7, 63):
        e = np.zeros(c.cfg.dim, dtype=np.float32)
        e[k] = 1.0
        assert np.array_equal(ix.scores(e, rows), c.emb[:, k].astype(np.float64))
        e[k] = -2.0                                              # sign and scale
        assert np.array_equal(ix.scores(e, rows), -2.0 * c.emb[:, k].astype(np.float64))


def test_tolerance_values():
    assert abs(tolerance(128) - 1.5259e-5) < 1e-8
    assert tolerance(64) < tolerance(128) < tolerance(256)


# ---------------------------------------------------------------- select
def test_search_matches_brute_force(tiny):
    c, qb, ix = tiny
    sets = _term_sets(c)
    live = [True] * c.n
    for q in range(qb.n):
        for k in (0, 1, 10, 50):
            res = ix.search_one(qb.emb[q], qb.cnf(q), k)
            ids, scores, nm = brute.search(c.emb, c.ids, sets, live, qb.emb[q], qb.cnf(q), k)
            assert res.n_match == nm and res.count == len(ids) == min(k, nm)
            assert res.ids.tolist() == ids
            assert np.allclose(res.scores, scores, rtol=0, atol=1e-15)


def test_selection_invariants_and_large_k(tiny):
    c, qb, ix = tiny
    for q in range(qb.n):
        res = ix.search_one(qb.emb[q], qb.cnf(q), 10 ** 9)
        assert res.count == res.n_match                          # K >= n_match: all
        assert len(set(res.ids.tolist())) == res.count
        assert np.all(np.diff(res.scores) <= 0)
        ok = set(int(ix.ids[r]) for r in ix.match_rows(qb.cnf(q)))
        assert set(res.ids.tolist()) == ok


def test_ties_break_by_id():
    rng = np.random.default_rng(5)
    base = rng.standard_normal((6, 8)).astype(np.float32)
    emb = np.concatenate([base, base, base])                     # 3 copies of each row
    ids = rng.permutation(1000)[:18].astype(np.uint32)
    ix = OracleIndex(8, 4)
    ix.load(emb, ids, np.arange(19), np.zeros(18, dtype=np.uint32))
    res = ix.search_one(base[2], [[0]], 18)
    for r in range(1, 18):
        if res.scores[r] == res.scores[r - 1]:
            assert res.ids[r] > res.ids[r - 1]
    assert res.scores[0] == res.scores[1] == res.scores[2]


def test_negative_zero_ties():
    emb = np.array([[0.0, 1.0], [-0.0, 1.0], [0.0, -0.0]], dtype=np.float32)
    ix = OracleIndex(2, 1)
    ix.load(emb, [9, 3, 5], [0, 1, 2, 3], [0, 0, 0])
    res = ix.search_one(np.array([1.0, 0.0], dtype=np.float32), [[0]], 3)
    assert res.ids.tolist() == [3, 5, 9]                          # all score 0


# --------------------------------------------------------------- updates
def test_updates_equal_rebuild():
    cfg = datagen.scaled(datagen.CONFIGS["tiny"], 3000, 8)
    c = datagen.corpus(cfg)
    qb = datagen.queries(cfg)
    ix = OracleIndex(cfg.dim, cfg.vocab)
    ix.load(c.emb, c.ids, c.term_off, c.terms)
    log = datagen.update_log(cfg, c.ids, 3, 200)
    for u in log:
        ix.update(u.del_ids, u.ins_ids, u.ins_emb, u.ins_term_off, u.ins_terms)
    # rebuild from the surviving rows
    keep = np.flatnonzero(ix.live)
    lists = [ix.term_set(r) for r in keep]
    off = np.cumsum([0] + [len(x) for x in lists])
    fresh = OracleIndex(cfg.dim, cfg.vocab)
    fresh.load(ix.emb[keep], ix.ids[keep], off, np.concatenate(lists))
    dead = set(int(x) for u in log for x in u.del_ids) - set(int(x) for u in log for x in u.ins_ids)
    for q in range(qb.n):
        a = ix.search_one(qb.emb[q], qb.cnf(q), 50)
        b = fresh.search_one(qb.emb[q], qb.cnf(q), 50)
        assert a.ids.tolist() == b.ids.tolist() and a.n_match == b.n_match
        assert not dead & set(a.ids.tolist())


def test_delete_top1_promotes_top2(tiny):
    c, qb, _ = tiny
    ix = OracleIndex(c.cfg.dim, c.cfg.vocab)
    ix.load(c.emb, c.ids, c.term_off, c.terms)
    before = ix.search_one(qb.emb[0], qb.cnf(0), 5)
    ix.update([before.ids[0]], [], np.zeros((0, c.cfg.dim), np.float32), [0], [])
    after = ix.search_one(qb.emb[0], qb.cnf(0), 4)
    assert after.ids.tolist() == before.ids[1:5].tolist()
    with pytest.raises(KeyError):
        ix.update([before.ids[0]], [], np.zeros((0, c.cfg.dim), np.float32), [0], [])


# --------------------------------------------------------------- checker
def test_checker_accepts_in_tolerance_swaps_rejects_others(tiny):
    c, qb, ix = tiny
    tol = tolerance(c.cfg.dim)
    q = int(np.argmax([len(ix.match_rows(qb.cnf(i))) for i in range(qb.n)]))
    res = ix.search_one(qb.emb[q], qb.cnf(q), 10)
    match = set(int(ix.ids[r]) for r in ix.match_rows(qb.cnf(q)))
    exact = lambda ids: ix.score_ids(qb.emb[q], ids)

    def run(ids, scores, count=None, nm=None):
        check_result(ids, scores, res.count if count is None else count,
                     res.n_match if nm is None else nm, res.ids, res.scores,
                     res.n_match, 10, exact, lambda i: i in match, tol)

    run(res.ids, res.scores.astype(np.float32))                 # itself
    s = res.scores.copy()
    s[3] += 0.5 * tol
    run(res.ids, s)                                              # small score error
    with pytest.raises(CheckError):
        s = res.scores.copy()
        s[3] += 3 * tol                                          # large score error
        run(res.ids, s)
    with pytest.raises(CheckError):                              # wrong order
        run(res.ids[::-1], res.scores[::-1])
    with pytest.raises(CheckError):                              # count
        run(res.ids, res.scores, count=9)
    with pytest.raises(CheckError):                              # n_match
        run(res.ids, res.scores, nm=res.n_match + 1)
    # a far-away replacement of the last id must fail
    full = ix.search_one(qb.emb[q], qb.cnf(q), 10 ** 6)
    far = full.ids[-1]
    ids = res.ids.copy()
    ids[-1] = far
    sc = res.scores.copy()
    sc[-1] = float(exact(np.array([far]))[0])
    with pytest.raises(CheckError):
        run(ids, sc)
    # a near-tie swap at the boundary (built by moving one score by < tol) passes
    ids = res.ids.copy()
    ids[-1] = full.ids[10]
    gap = full.scores[9] - full.scores[10]
    if gap < tol:
        sc = res.scores.copy()
        sc[-1] = full.scores[10]
        run(ids, sc)


def test_recall_definition():
    r, skipped = recall_at_k([[1, 2, 3], [4], [7]], [[1, 2, 9, 10], [4], []])
    assert skipped == 1 and abs(r - (0.5 + 1.0) / 2) < 1e-15


# ------------------------------------------------------------ quantizers
def test_bf16_matches_torch_cast():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(200000).astype(np.float32) * 0.1,
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3e-39], np.float32)])
    # exact halfway cases between BF16 neighbours
    hw = (rng.integers(0, 2 ** 15, 1000).astype(np.uint32) << 16) | 0x8000
    x = np.concatenate([x, hw.view(np.float32)[np.isfinite(hw.view(np.float32))]])
    want = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    got = quant.bf16_round(x)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_e4m3_matches_torch_cast():
    torch = pytest.importorskip("torch")
    if not hasattr(torch, "float8_e4m3fn"):
        pytest.skip("torch without float8_e4m3fn")
    rng = np.random.default_rng(2)
    y = np.concatenate([rng.uniform(-448, 448, 200000), rng.uniform(-1, 1, 20000),
                        rng.uniform(-0.02, 0.02, 20000)]).astype(np.float32)
    grid = quant.E4M3_GRID
    mids = ((grid[1:] + grid[:-1]) / 2).astype(np.float32)       # exact ties
    y = np.concatenate([y, mids, -mids, grid.astype(np.float32)])
    want = torch.from_numpy(y).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = quant.e4m3_encode(y)
    nz = ~((want & 0x7F) == 0)                                    # torch keeps -0
    assert np.array_equal(got[nz], want[nz])
    assert np.all((got[~nz] & 0x7F) == 0)
    assert quant.E4M3_MAX == 448.0 and len(grid) == 127


def test_fp8_row_scale_and_saturation():
    x = np.array([[0.5, -0.25, 0.0, 1e-4], [0, 0, 0, 0], [3.0, 1.0, -3.0, 0.1]], np.float32)
    v, s = quant.fp8_rows(x)
    assert s[1] == 1.0 and np.all(v[1] == 0)
    assert np.abs(v).max() <= 448.0
    assert v[0, 0] == 448.0 and v[2, 0] == 448.0 and v[2, 2] == -448.0
    assert np.allclose(v * s[:, None], x, rtol=2 ** -3, atol=s[:, None] * 2 ** -9)


def test_rescored_pipeline_reduces_to_exact_when_r_covers_matches(tiny):
    c, qb, ix = tiny
    for q in range(qb.n):
        nm = len(ix.match_rows(qb.cnf(q)))
        for storage in ("bf16", "fp8"):
            a = ix.search_rescored_one(qb.emb[q], qb.cnf(q), 10, max(nm, 1), storage)
            b = ix.search_one(qb.emb[q], qb.cnf(q), 10)
            assert a.ids.tolist() == b.ids.tolist()


def test_recall_non_decreasing_in_r(tiny):
    c, qb, ix = tiny
    exact = [ix.search_one(qb.emb[q], qb.cnf(q), 10).ids for q in range(qb.n)]
    last = -1.0
    for r in (10, 12, 20, 40, 200):
        got = [ix.search_rescored_one(qb.emb[q], qb.cnf(q), 10, r, "fp8").ids
               for q in range(qb.n)]
        rec, _ = recall_at_k(got, exact)
        assert rec >= last - 1e-12
        last = rec
    assert last == 1.0


def test_approx_scores_unit_query_bf16(tiny):
    c, qb, ix = tiny
    rows = np.arange(c.n)
    e = np.zeros(c.cfg.dim, dtype=np.float32)
    e[5] = 1.0
    got = ix.approx_scores(e, rows, "bf16")
    assert np.array_equal(got, quant.bf16_round(c.emb[:, 5]).astype(np.float64))


def _torch_e4m3(v: np.ndarray) -> np.ndarray:
    """Decoded E4M3FN values of FP32 inputs, by PyTorch's own cast (independent
    of ``oracle.quant``, which emulates the format by nearest grid point)."""
    torch = pytest.importorskip("torch")
    if not hasattr(torch, "float8_e4m3fn"):
        pytest.skip("torch without float8_e4m3fn")
    t = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32))
    return t.to(torch.float8_e4m3fn).float().numpy().astype(np.float64)


def _fp8_expected(x: np.ndarray):
    """(decoded codes, FP32 scale) per row: scale = fl32(amax / 448), codes
    from fl32(x * fl32(448 / amax)) through PyTorch's E4M3FN cast."""
    x = np.asarray(x, dtype=np.float32)
    amax = np.abs(x).max(axis=1).astype(np.float32)
    nz = amax > 0
    inv = np.where(nz, np.float32(448.0) / np.where(nz, amax, np.float32(1)),
                   np.float32(1)).astype(np.float32)
    scale = np.where(nz, amax / np.float32(448.0), np.float32(1)).astype(np.float32)
    return _torch_e4m3((x * inv[:, None]).astype(np.float32)), scale


def test_approx_scores_unit_query_fp8(tiny):
    """q = e_k quantises to 448 at k (scale fl32(1/448)), so the first-pass
    score of row i is decode(code_ik) * s_i * 448 * fl32(1/448): a dropped or
    swapped scale, or a wrong column, fails this."""
    c, qb, ix = tiny
    rows = np.arange(0, c.n, 7)
    dec, xs = _fp8_expected(c.emb[rows])
    qscale = float(np.float32(1.0) / np.float32(448.0))
    for k in (0, 5, 63):
        e = np.zeros(c.cfg.dim, dtype=np.float32)
        e[k] = 1.0
        got = ix.approx_scores(e, rows, "fp8")
        want = dec[:, k] * 448.0 * qscale * xs.astype(np.float64)
        assert np.allclose(got, want, rtol=4 * 2.0 ** -53, atol=0), k
        # a negative, scaled unit query: the same codes, sign flipped
        e[k] = -3.0
        got = ix.approx_scores(e, rows, "fp8")
        want = -dec[:, k] * 448.0 * float(np.float32(3.0) / np.float32(448.0)) * xs
        assert np.allclose(got, want, rtol=4 * 2.0 ** -53, atol=0), k


def test_approx_scores_fp8_brute_force(tiny):
    """Random queries and rows: math.fsum of the products of the decoded
    codes (PyTorch's cast), times both FP32 scales."""
    c, qb, ix = tiny
    rows = np.arange(3, c.n, 997)
    dec, xs = _fp8_expected(c.emb[rows])
    for q in range(4):
        qd, qs = _fp8_expected(qb.emb[q][None, :])
        got = ix.approx_scores(qb.emb[q], rows, "fp8")
        for i, r in enumerate(rows):
            dot = math.fsum(float(a) * float(b) for a, b in zip(dec[i], qd[0]))
            want = dot * float(qs[0]) * float(xs[i])
            bound = math.fsum(abs(float(a) * float(b)) for a, b in zip(dec[i], qd[0]))
            err = 64 * 2.0 ** -53 * bound * float(qs[0]) * float(xs[i]) + 4 * 2.0 ** -53 * abs(want)
            assert abs(got[i] - want) <= err, (q, r)


def test_approx_scores_bf16_brute_force(tiny):
    """BF16 first pass: fsum of the products of PyTorch-rounded operands."""
    torch = pytest.importorskip("torch")
    c, qb, ix = tiny
    rows = np.arange(11, c.n, 1013)
    xb = torch.from_numpy(c.emb[rows]).to(torch.bfloat16).double().numpy()
    for q in range(4):
        qbf = torch.from_numpy(qb.emb[q]).to(torch.bfloat16).double().numpy()
        got = ix.approx_scores(qb.emb[q], rows, "bf16")
        for i in range(len(rows)):
            want = math.fsum(float(a) * float(b) for a, b in zip(xb[i], qbf))
            bound = math.fsum(abs(float(a) * float(b)) for a, b in zip(xb[i], qbf))
            assert abs(got[i] - want) <= 64 * 2.0 ** -53 * bound, (q, i)


def test_update_inserts_against_set_brute_force():
    """Replay the update log on a pure-Python state (id -> (row, term set))
    built from the initial corpus and the log alone, never from the oracle's
    arrays, and compare every query's brute-force result (sets + fsum) with
    the oracle's.  An inserted row attached to the wrong id, or a term list
    shifted between documents, changes some result."""
    cfg = datagen.scaled(datagen.CONFIGS["tiny"], 2000, 8)
    c = datagen.corpus(cfg)
    qb = datagen.queries(cfg)
    ix = OracleIndex(cfg.dim, cfg.vocab)
    ix.load(c.emb, c.ids, c.term_off, c.terms)
    state = {}
    off = c.term_off.astype(np.int64)
    for i in range(c.n):
        state[int(c.ids[i])] = (c.emb[i], set(int(t) for t in c.terms[off[i]:off[i + 1]]))
    log = datagen.update_log(cfg, c.ids, 3, 240)
    for u in log:
        ix.update(u.del_ids, u.ins_ids, u.ins_emb, u.ins_term_off, u.ins_terms)
        for x in u.del_ids:
            del state[int(x)]
        uo = u.ins_term_off.astype(np.int64)
        for j, x in enumerate(u.ins_ids):
            state[int(x)] = (u.ins_emb[j], set(int(t) for t in u.ins_terms[uo[j]:uo[j + 1]]))
        ids = list(state)
        emb = [state[x][0] for x in ids]
        sets = [state[x][1] for x in ids]
        live = [True] * len(ids)
        # a query that favours the newest rows: their mean direction
        newest = np.asarray(u.ins_emb, dtype=np.float64).mean(axis=0)
        extra = (newest / np.linalg.norm(newest)).astype(np.float32)
        for q in range(qb.n + 1):
            qe = qb.emb[q] if q < qb.n else extra
            cnf = qb.cnf(q) if q < qb.n else []
            want_ids, want_s, nm = brute.search(emb, ids, sets, live, qe, cnf, 25)
            got = ix.search_one(qe, cnf, 25)
            assert got.n_match == nm and got.ids.tolist() == want_ids, q
            assert np.allclose(got.scores, want_s, rtol=0, atol=1e-15)
        assert ix.n_live == len(state)
