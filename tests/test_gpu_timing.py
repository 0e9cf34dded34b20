"""The device timings a search records (fr_timings, fr_stats): every call in
the history has a first-scan time and a call time that covers it, for
asynchronous device-buffer searches, synchronous host-buffer searches and
graph replays; a call that fails before any device work leaves no entry."""
import numpy as np
import pytest

import datagen
from helpers import gpu_index

pytestmark = pytest.mark.gpu


def test_timings_cover_every_kind_of_call():
    import torch
    from paper_2402_13435_amd import SearchResult
    c, qb = datagen.workload("tiny")
    ix = gpu_index(c, k_max=10, n_workspaces=2)
    dev = torch.device("cuda:0")
    q = torch.from_numpy(qb.emb).to(dev)
    out = SearchResult(torch.empty((qb.n, 10), dtype=torch.int32, device=dev),
                       torch.empty((qb.n, 10), dtype=torch.float32, device=dev),
                       torch.empty(qb.n, dtype=torch.int32, device=dev),
                       torch.empty(qb.n, dtype=torch.int64, device=dev))
    s = torch.cuda.Stream()
    for _ in range(3):
        ix.search(q, qb, 10, out=out, stream=s)                  # asynchronous, device buffers
    for _ in range(2):
        ix.search(qb.emb, qb, 10)                               # synchronous, host buffers
    for _ in range(2):
        ix.search(q, qb, 10, out=out, stream=s, graph=True)      # captured graph
    torch.cuda.synchronize()
    scan, total = ix.timings(64)
    assert len(scan) == 7 and len(total) == 7
    assert np.all(scan > 0) and np.all(np.isfinite(total))
    assert np.all(total >= scan * 0.999)
    st = ix.stats()
    assert st.ms_scan > 0 and st.ms_total >= st.ms_scan * 0.999
    assert st.ms_call >= st.ms_total * 0.999
    ix.close()


def test_a_call_that_fails_before_the_device_leaves_no_timing():
    from paper_2402_13435_amd import FrError
    from test_gpu_lists import _big_vocab_corpus
    c = _big_vocab_corpus(n=3000)
    ix = gpu_index(c, k_max=10, list_terms=40, batch_terms=16)
    ok = datagen.from_cnf_lists(c.emb[:1], [[list(range(10))]], [5])
    bad = datagen.from_cnf_lists(c.emb[:2], [[list(range(10))], [list(range(10, 20))]], [5, 5])
    ix.search(ok.emb, ok, 5)
    with pytest.raises(FrError):
        ix.search(bad.emb, bad, 5)                              # 20 distinct terms > 16
    ix.search(ok.emb, ok, 5)
    scan, total = ix.timings(64)
    assert len(scan) == 2 and np.all(scan > 0) and np.all(total >= scan * 0.999)
    ix.close()
