"""Pure-Python brute force for tiny inputs, used only to pin ``oracle.core``.

TEST INFRASTRUCTURE ONLY.  Term sets are Python sets, a CNF is checked
clause by clause with set intersection, and each score is ``math.fsum`` of
the exact FP64 products, i.e. the correctly rounded value of the exact dot
product of the two FP32 vectors.  No NumPy reduction, bitmap or sort key is
shared with ``core``.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple


def matches(term_set: set, cnf: Sequence[Sequence[int]]) -> bool:
    for clause in cnf:
        if not term_set.intersection(clause):
            return False
    return True


def exact_dot(q: Sequence[float], x: Sequence[float]) -> float:
    return math.fsum(float(a) * float(b) for a, b in zip(q, x))


def search(emb, ids, term_sets: List[set], live: Sequence[bool], q, cnf, k: int
           ) -> Tuple[List[int], List[float], int]:
    """Returns (ids, scores, n_match) of the top-k by (score desc, id asc)."""
    cand = []
    for r in range(len(ids)):
        if live[r] and matches(term_sets[r], cnf):
            cand.append((-exact_dot(q, emb[r]), int(ids[r])))
    cand.sort()
    top = cand[:k]
    return [i for _s, i in top], [-s for s, _i in top], len(cand)
