"""Pins of the sign-code pre-selection oracle (oracle.signcode).

Checked against closed forms (an identity table gives the coordinates' own
signs; two codes agree on numBits bits with themselves and on none with
their negation), the textbook collision probability of random sign
projections (agreement 1 - theta/pi for vectors at angle theta), an algebraic
identity of the popcount score, pure-Python brute force on tiny inputs, the
reduction to the plain exact search when quantK covers every match, and the
structure of the random tables.  A slip such as counting differing instead
of equal bits, setting the bit on a negative sum, or keeping the worst
instead of the best survivors fails at least one of them.
"""
import math

import numpy as np
import pytest

import datagen
from oracle import OracleIndex
from oracle.signcode import SignCodes, brute_search, pack_words, quant_score, sign_bits


def _identity_table(d, sign=1.0):
    return (np.arange(d + 1, dtype=np.uint32), np.arange(d, dtype=np.uint32),
            np.full(d, sign, np.float32))


def test_identity_table_codes_are_coordinate_signs():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((50, 64)).astype(np.float32)
    x[0, :5] = 0.0
    off, dim, sg = _identity_table(64)
    assert np.array_equal(sign_bits(x, off, dim, sg), x > 0)
    off, dim, sg = _identity_table(64, -1.0)
    assert np.array_equal(sign_bits(x, off, dim, sg), x < 0)


def test_popcount_score_counts_equal_bits():
    rng = np.random.default_rng(1)
    a = rng.random((20, 128)) < 0.5
    b = rng.random(128) < 0.5
    got = quant_score(pack_words(a), pack_words(b[None, :])[0])
    for i in range(20):
        assert got[i] == sum(1 for u, v in zip(a[i], b) if u == v)
    # the same count from the +-1 inner product: (numBits + <a', b'>) / 2
    pa, pb = np.where(a, 1, -1), np.where(b, 1, -1)
    assert np.array_equal(got, (128 + pa @ pb) // 2)


def test_self_and_negation_scores():
    p = datagen.sign_projection(128, 512, seed=3)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((10, 128)).astype(np.float32)
    cx = pack_words(sign_bits(x, p.bin_off, p.bin_dim, p.bin_sign))
    cn = pack_words(sign_bits(-x, p.bin_off, p.bin_dim, p.bin_sign))
    for i in range(10):
        assert quant_score(cx[i:i + 1], cx[i])[0] == 512
        # no bin sum of Gaussian data is exactly zero: -x flips every bit
        assert quant_score(cx[i:i + 1], cn[i])[0] == 0


@pytest.mark.parametrize("theta", [math.pi / 3, math.pi / 2, 2 * math.pi / 3])
def test_agreement_matches_angle(theta):
    # bins spanning all coordinates: each bit is the sign of a random +-1
    # projection, so two vectors at angle theta agree on a bit with
    # probability close to 1 - theta / pi
    d = 256
    p = datagen.sign_projection(d, 512, seed=4, bin_size=d)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((200, d))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    z = rng.standard_normal((200, d))
    z -= (z * x).sum(1, keepdims=True) * x
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    y = math.cos(theta) * x + math.sin(theta) * z
    cx = pack_words(sign_bits(x.astype(np.float32), p.bin_off, p.bin_dim, p.bin_sign))
    cy = pack_words(sign_bits(y.astype(np.float32), p.bin_off, p.bin_dim, p.bin_sign))
    frac = np.mean([quant_score(cx[i:i + 1], cy[i])[0] / 512 for i in range(200)])
    assert abs(frac - (1 - theta / math.pi)) < 0.012, frac


def test_bin_sums_are_fp32_in_table_order():
    # exact sum 1e-8 > 0, but in FP32 1 + 1e-8 rounds to 1 and the bin sums to 0
    x = np.array([[1.0, 1e-8, -1.0]], np.float32)
    off = np.array([0, 3], np.uint32)
    dim = np.array([0, 1, 2], np.uint32)
    sg = np.ones(3, np.float32)
    assert not sign_bits(x, off, dim, sg)[0, 0]
    # the other order: 1 - 1 = 0, then + 1e-8 > 0
    assert sign_bits(x, off, np.array([0, 2, 1], np.uint32), sg)[0, 0]


def test_sign_projection_structure():
    for d, bits, s in [(128, 512, 2), (256, 512, 2), (64, 512, 2), (256, 64, 4), (128, 64, 2)]:
        p = datagen.sign_projection(d, bits, seed=7)
        assert p.n_bits == bits
        assert np.array_equal(np.diff(p.bin_off.astype(np.int64)), np.full(bits, s))
        assert set(np.unique(p.bin_sign).tolist()) <= {-1.0, 1.0}
        pos = p.bin_dim.astype(np.int64)
        for a in range(0, len(pos) - d + 1, d):      # each whole permutation
            assert sorted(pos[a:a + d].tolist()) == list(range(d))
        assert pos.max() < d


def _tiny_corpus(n=60, d=16, vocab=6, seed=8):
    rng = np.random.default_rng(seed)
    emb = rng.standard_normal((n, d)).astype(np.float32)
    ids = (np.arange(n) * 7 + 3).astype(np.uint32)
    sets = [set(int(t) for t in rng.choice(vocab, size=rng.integers(1, 4), replace=False))
            for _ in range(n)]
    off = np.zeros(n + 1, np.uint64)
    off[1:] = np.cumsum([len(s) for s in sets])
    terms = np.array([t for s in sets for t in sorted(s)], np.uint32)
    o = OracleIndex(d, vocab)
    o.load(emb, ids, off, terms)
    return o, emb, ids, sets


def test_preselect_matches_brute_force():
    o, emb, ids, sets = _tiny_corpus()
    p = datagen.sign_projection(16, 64, seed=9)
    sc = SignCodes(o, p.bin_off, p.bin_dim, p.bin_sign)
    rng = np.random.default_rng(10)
    for t in range(12):
        q = rng.standard_normal(16).astype(np.float32)
        cnf = [] if t % 3 == 0 else [[int(rng.integers(6)), int(rng.integers(6))]]
        for quant_k, k in [(5, 3), (12, 4), (1, 1), (100, 5)]:
            a = sc.search_one(q, cnf, k, quant_k)
            b_ids, b_sc, b_n = brute_search(emb, ids, sets, [True] * len(ids), q, cnf, k,
                                            quant_k, p.bin_off, p.bin_dim, p.bin_sign)
            assert a.n_match == b_n
            assert a.ids.tolist() == b_ids, (t, quant_k, k)
            assert np.allclose(a.scores, b_sc, rtol=0, atol=1e-12)


def test_preselect_reduces_to_exact_when_quant_k_covers_matches():
    c, qb = datagen.workload("tiny")
    o = OracleIndex(c.cfg.dim, c.cfg.vocab)
    o.load(c.emb, c.ids, c.term_off, c.terms)
    p = datagen.sign_projection(c.cfg.dim, 128, seed=11)
    sc = SignCodes(o, p.bin_off, p.bin_dim, p.bin_sign)
    for q in range(qb.n):
        a = sc.search_one(qb.emb[q], qb.cnf(q), 10, o.n_rows)
        b = o.search_one(qb.emb[q], qb.cnf(q), 10)
        assert np.array_equal(a.ids, b.ids) and np.array_equal(a.scores, b.scores)
        assert a.n_match == b.n_match


def test_survivors_are_nested_and_best_first():
    c, qb = datagen.workload("tiny")
    o = OracleIndex(c.cfg.dim, c.cfg.vocab)
    o.load(c.emb, c.ids, c.term_off, c.terms)
    p = datagen.sign_projection(c.cfg.dim, 256, seed=12)
    sc = SignCodes(o, p.bin_off, p.bin_dim, p.bin_sign)
    for q in range(min(qb.n, 8)):
        small = sc.survivors(qb.emb[q], qb.cnf(q), 20)
        big = sc.survivors(qb.emb[q], qb.cnf(q), 60)
        assert set(small.tolist()) <= set(big.tolist())
        qs = quant_score(sc.words[big], sc.query_words(qb.emb[q]))
        rest = np.setdiff1d(o.match_rows(qb.cnf(q)), big)
        if len(rest) and len(big):
            worst = quant_score(sc.words[rest], sc.query_words(qb.emb[q])).max()
            assert worst <= qs.min()            # no dropped match beats a survivor
