"""FP64 CPU oracle for exhaustive filtered top-K retrieval.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the GPU
library (no kernels, headers, helpers, tables or pre/post-processing); the
only thing both sides consume is the seeded input generator ``datagen``.

What it computes is the plain definition of the method of Sec. 5.3 (System
Implementation) and the appendix "Optimizing System on GPU":

* F-TBR: a document matches a query iff it satisfies every clause of the
  query's conjunctive normal form, a clause being satisfied iff the document
  holds at least one of its terms (appendix, "TBR").
* F-EBR: every matching document is scored by the inner product of its
  embedding with the query embedding (appendix, "EBR").
* top-K: the K best-scoring matches are returned (appendix, "Fast Top K
  Selection"; the bucket trick there is an exact speed-up of selection, so
  the oracle selects by a plain full sort).

Readings where the paper is silent (all listed in the design doc as well):
scores are raw dot products of the stored FP32 vectors evaluated in FP64;
ties are broken by external id ascending; -0.0 equals +0.0; a query with no
clause matches every live document and an empty clause matches nothing;
count = min(K, n_match).

Modules: ``core`` (the oracle), ``brute`` (pure-Python brute force used to
pin ``core``), ``quant`` (CPU emulation of the BF16 / FP8-E4M3 storage
formats used by the reduced-precision forms), ``check`` (the tolerance-aware
result checker and recall@k).
"""
from .core import OracleIndex, OracleResult, tolerance  # noqa: F401
from .check import check_result, recall_at_k  # noqa: F401
