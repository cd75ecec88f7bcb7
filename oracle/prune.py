"""Oracle of the pruning selection (TEST INFRASTRUCTURE ONLY, like the rest of
this package).

Speedy-Splat prunes a fixed fraction of the Gaussians ranked by its efficient
pruning score: Soft Pruning (Sec. 4.2.2) removes 80 % before each of the
opacity resets at iterations 6000, 9000 and 12000, Hard Pruning (Sec. 4.2.3)
removes 30 % every 3000 iterations from iteration 15000; the score is the
one of Sec. 4.2.1.  The plain definition of one prune: with n Gaussians and
ratio p, floor(p n) of them (the product in double precision) with the
lowest scores are removed.  Readings where the paper is silent: a score that
is NaN or not positive ranks as 0, and among equal scores the Gaussian with
the lower index is kept.  The kept indices are returned in ascending order.
"""
from __future__ import annotations

import math

import numpy as np


def n_keep(n: int, ratio: float) -> int:
    """Gaussians kept when pruning the fraction `ratio` of n."""
    assert 0.0 <= ratio <= 1.0
    return n - int(math.floor(float(ratio) * float(n)))


def score_rank_key(score) -> np.ndarray:
    """Ranking value of each score: the score itself, 0 for NaN or <= 0."""
    s = np.asarray(score, dtype=np.float32)
    return np.where(s > 0, s, np.float32(0)).astype(np.float32)


def prune_select(score, ratio: float) -> np.ndarray:
    """Kept indices (ascending): the n_keep highest scores, ties by lower index."""
    key = score_rank_key(score).astype(np.float64)
    n = len(key)
    k = n_keep(n, ratio)
    order = np.lexsort((np.arange(n), -key))      # score descending, then index
    return np.sort(order[:k]).astype(np.uint32)
