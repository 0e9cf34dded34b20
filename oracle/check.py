"""Result checker ("exact except ties inside tolerance") and recall@k.

TEST INFRASTRUCTURE ONLY.

Several results are correct when scores tie within the arithmetic's
tolerance, so a GPU list G is accepted against the oracle list A (exact FP64
scores s, tolerance tol) when all of these hold:

1. |G| = |A| = min(K, n_match) and the GPU's n_match equals the oracle's;
2. every id of G is unique, live and matches the predicate;
3. G is ordered by (returned score desc, id asc);
4. every returned score is within tol of the exact score of its id;
5. with tau the oracle's last score, ids only in G have s >= tau - 2 tol and
   ids only in A have s <= tau + 2 tol;
6. rank by rank, |G score[r] - A score[r]| <= tol + score_tol (sorting
   perturbed values moves each rank by at most the perturbation).
"""
from __future__ import annotations

from typing import Callable, Iterable, List, Optional, Sequence

import numpy as np


class CheckError(AssertionError):
    pass


def check_result(g_ids: np.ndarray, g_scores: np.ndarray, g_count: int,
                 g_nmatch: int, a_ids: np.ndarray, a_scores: np.ndarray,
                 a_nmatch: int, k: int, exact: Callable[[np.ndarray], np.ndarray],
                 is_match: Callable[[int], bool], tol: float,
                 score_tol: Optional[float] = None) -> None:
    """Raise CheckError on the first violated rule.

    ``exact(ids)`` returns the oracle's FP64 score of each id; ``is_match``
    says whether a live id satisfies the query.  ``score_tol`` (default tol)
    bounds rule 4 separately, for forms whose returned scores are rescored.
    """
    score_tol = tol if score_tol is None else score_tol
    g_ids = np.asarray(g_ids[:g_count], dtype=np.uint32)
    g_scores = np.asarray(g_scores[:g_count], dtype=np.float64)
    want = min(int(k), int(a_nmatch))
    if int(g_nmatch) != int(a_nmatch):
        raise CheckError(f"n_match {g_nmatch} != {a_nmatch}")
    if int(g_count) != want or len(a_ids) != want:
        raise CheckError(f"count {g_count} != min(K, n_match) = {want}")
    if len(set(g_ids.tolist())) != len(g_ids):
        raise CheckError("duplicate ids")
    for i in g_ids.tolist():
        if not is_match(int(i)):
            raise CheckError(f"id {i} does not match / is not live")
    for r in range(1, len(g_ids)):
        if g_scores[r] > g_scores[r - 1] or (
                g_scores[r] == g_scores[r - 1] and g_ids[r] < g_ids[r - 1]):
            raise CheckError(f"order broken at rank {r}")
    if want == 0:
        return
    s = exact(g_ids)
    err = np.abs(g_scores - s)
    if err.max() > score_tol:
        r = int(err.argmax())
        raise CheckError(f"score error {err.max():.3g} > {score_tol:.3g} at rank {r}")
    tau = float(a_scores[-1])
    g_set, a_set = set(g_ids.tolist()), set(np.asarray(a_ids).tolist())
    only_g = np.array(sorted(g_set - a_set), dtype=np.uint32)
    if len(only_g):
        sg = exact(only_g)
        if sg.min() < tau - 2 * tol:
            raise CheckError(f"extra id with score {sg.min():.9g} < tau {tau:.9g}")
    only_a = np.array(sorted(a_set - g_set), dtype=np.uint32)
    if len(only_a):
        sa = exact(only_a)
        if sa.max() > tau + 2 * tol:
            raise CheckError(f"missing id with score {sa.max():.9g} > tau {tau:.9g}")
    rank_err = np.abs(g_scores - np.asarray(a_scores, dtype=np.float64))
    if rank_err.max() > tol + score_tol:
        raise CheckError(f"rank-wise score gap {rank_err.max():.3g}")


def recall_at_k(retrieved: Sequence[Iterable[int]], relevant: Sequence[Iterable[int]]):
    """recall@k = (1/N) sum_i |R_i & A_i| / |A_i| (Sec. 6.2, Offline Results).

    Queries whose relevant set is empty are excluded; returns (recall,
    n_excluded)."""
    tot, n, skipped = 0.0, 0, 0
    for r, a in zip(retrieved, relevant):
        a = set(int(x) for x in a)
        if not a:
            skipped += 1
            continue
        tot += len(a & set(int(x) for x in r)) / len(a)
        n += 1
    return (tot / n if n else 1.0), skipped
