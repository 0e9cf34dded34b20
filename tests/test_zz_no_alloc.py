"""fr_search_noalloc (the search that allocates nothing: its per-search
device memory lives in the library's fixed scratch array) against fr_search
on the same inputs, through the C ABI: two calls in a row, the second with
fewer queries, on an FP32 and a BF16 index; an asynchronous call on a torch
stream; and the rejection of a request larger than the scratch."""
import numpy as np
import pytest

import datagen
from helpers import check_query, gpu_index, oracle_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def data():
    cfg = datagen.scaled(datagen.CONFIGS["fp32"], 300_001, 256)
    c = datagen.corpus(cfg)
    qb = datagen.queries(cfg, datagen.doc_frequency(cfg, c.term_off, c.terms))
    return c, qb


def _dev_out(torch, n_q, k_max):
    from paper_2402_13435_amd.binding import SearchResult
    d = torch.device("cuda", 0)
    out = SearchResult(torch.full((n_q, k_max), 7, dtype=torch.int32, device=d),
                       torch.full((n_q, k_max), 7.0, dtype=torch.float32, device=d),
                       torch.full((n_q,), 7, dtype=torch.int32, device=d),
                       torch.full((n_q,), 7, dtype=torch.int64, device=d))
    # the fills run on torch's stream, the search on another one
    torch.cuda.synchronize()
    return out


def _host(r):
    return (r.ids.cpu().numpy().view(np.uint32), r.scores.cpu().numpy(),
            r.count.cpu().numpy().view(np.uint32), r.n_match.cpu().numpy().view(np.uint64))


def _same(a, b, what):
    for x, y, name in zip(a, b, ("ids", "scores", "count", "n_match")):
        assert np.array_equal(x, y), (what, name)


def _both(torch, ix, qb, idx, k):
    """(fr_search rows, fr_search_noalloc rows) of the sub-batch idx."""
    sub = qb.subset(idx)
    q = torch.from_numpy(np.ascontiguousarray(sub.emb)).cuda()
    ref = ix.search(q, sub, k)
    torch.cuda.synchronize()
    got = ix.search_noalloc(q, sub, k, _dev_out(torch, sub.n, ix.k_max))
    return sub, _host(ref), _host(got)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_noalloc_equals_search_twice(data, dtype):
    torch = pytest.importorskip("torch")
    c, qb = data
    o = oracle_for(c)
    kw = dict(rescore_r=256) if dtype == "bf16" else {}
    ix = gpu_index(c, k_max=100, dtype=dtype, max_batch=256, **kw)
    first = list(range(qb.n)) if dtype == "f32" else list(range(0, 256, 2))
    second = list(range(5, 45)) if dtype == "f32" else list(range(3, 27))
    for idx in (first, second):
        sub, ref, got = _both(torch, ix, qb, idx, 100)
        print(f"[noalloc] {dtype}: {sub.n} queries", flush=True)
        _same(ref, got, (dtype, sub.n))
        assert not np.any(got[2] == 0xFFFFFFFF)
    # the second (smaller) call's rows against the oracle as well
    from types import SimpleNamespace
    res = SimpleNamespace(ids=got[0], scores=got[1], count=got[2], n_match=got[3])
    for q in range(0, sub.n, 3):
        if dtype == "f32":
            check_query(o, sub, q, res, 100)
        else:
            a = o.search_one(sub.emb[q], sub.cnf(q), 100)
            assert int(res.n_match[q]) == a.n_match
            assert int(res.count[q]) == min(100, a.n_match)
    ix.close()


def test_noalloc_async_on_a_stream(data):
    torch = pytest.importorskip("torch")
    c, qb = data
    ix = gpu_index(c, k_max=100, max_batch=256)
    idx = list(range(100, 164))
    sub = qb.subset(idx)
    q = torch.from_numpy(np.ascontiguousarray(sub.emb)).cuda()
    ref = _host(ix.search(q, sub, 100))
    s = torch.cuda.Stream()
    out = _dev_out(torch, sub.n, 100)
    with torch.cuda.stream(s):
        ix.search_noalloc(q, sub, 100, out, stream=s)
    s.synchronize()
    _same(ref, _host(out), "async")
    ix.close()


def test_noalloc_rejects_requests_beyond_the_scratch(data):
    torch = pytest.importorskip("torch")
    from paper_2402_13435_amd.binding import FR_EINVAL, FrError
    c, qb = data
    # BF16 with R=4096: 65,536 candidate slots per query, 512 KiB each, so
    # 256 queries need more than the 128 MiB scratch
    ix = gpu_index(c, k_max=100, dtype="bf16", rescore_r=4096, max_batch=256)
    q = torch.from_numpy(np.ascontiguousarray(qb.emb)).cuda()
    with pytest.raises(FrError) as e:
        ix.search_noalloc(q, qb, 100, _dev_out(torch, qb.n, 100))
    assert e.value.status == FR_EINVAL and "scratch" in e.value.message
    # a smaller request on the same index still runs and agrees with fr_search
    sub, ref, got = _both(torch, ix, qb, list(range(32)), 100)
    _same(ref, got, "after rejection")
    ix.close()
