"""Pins of the pruning-selection oracle: a pure-Python loop over explicit
(score, index) comparisons on small inputs, the selection's invariants, and
the schedule arithmetic of Sec. 4.2.2 / 4.2.3."""
import math

import numpy as np
import pytest

from oracle import prune


def _brute(score, ratio):
    """Insertion of every Gaussian into a list kept ordered by 'beats': higher
    ranking score, or the same score and a lower index."""
    s = [float(x) if (x == x and x > 0) else 0.0 for x in np.asarray(score, np.float32)]
    ranked = []
    for i in range(len(s)):
        pos = 0
        while pos < len(ranked) and (s[ranked[pos]] > s[i] or
                                     (s[ranked[pos]] == s[i] and ranked[pos] < i)):
            pos += 1
        ranked.insert(pos, i)
    k = len(s) - int(math.floor(ratio * len(s)))
    return sorted(ranked[:k])


@pytest.mark.parametrize("seed", range(20))
def test_selection_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 60))
    # few distinct values so that ties at the threshold are common, plus
    # zeros, negatives and NaN
    score = rng.choice([0.0, 1.0, 2.5, 2.5000002, 7.0, -3.0, np.nan, 1e-30], size=n)
    score = score.astype(np.float32)
    for ratio in (0.0, 0.3, 0.5, 0.8, 1.0):
        got = prune.prune_select(score, ratio)
        assert got.tolist() == _brute(score, ratio), (seed, ratio)


def test_selection_invariants_at_scale():
    rng = np.random.default_rng(5)
    n = 200_003
    score = (rng.standard_normal(n) ** 2).astype(np.float32)
    score[rng.random(n) < 0.1] = 0.0
    score[::1000] = np.float32(0.75)                 # a block of exact ties
    for ratio in (0.3, 0.8):
        keep = prune.prune_select(score, ratio)
        assert len(keep) == n - math.floor(ratio * n)
        assert np.all(np.diff(keep.astype(np.int64)) > 0)
        kept = np.zeros(n, bool)
        kept[keep] = True
        ks, ds = score[kept], score[~kept]
        assert ks.min() >= ds.max()                  # every kept score beats every dropped one
        t = ks.min()
        if np.any(ds == t):                           # ties: kept indices precede dropped ones
            assert np.nonzero(kept & (score == t))[0].max() < np.nonzero(~kept & (score == t))[0].min()


def test_schedule_counts():
    """Sec. 4.2.2 and 4.2.3: three 80 % soft prunes and 30 % hard prunes on a
    fixed set: each prune keeps n - floor(p n)."""
    n = 1_000_000
    for p in (0.8, 0.8, 0.8):
        n = prune.n_keep(n, p)
    assert n == 8000
    for p in (0.3,) * 5:
        n = prune.n_keep(n, p)
    assert n == 1345
