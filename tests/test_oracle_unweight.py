"""Pins of the oracle's unweighting (hit-or-miss acceptance) against what the method fixes.

* Kept events follow the target density: weights w(x) = 3 x^2 on uniform x give kept
  x with distribution function x^3 (Kolmogorov-Smirnov), at the expected acceptance
  rate 1/3 (binomial error).
* Exact cases: non-positive and NaN weights are never kept; a weight at or above w_max
  is always kept with factor w / w_max; the comparison is strict (u w_max = w is not
  kept); kept events are listed in increasing order.
* The acceptance stream is uniform and is not the phase-space stream.
* Planted mistakes (each in a copy of the function) fail one of these.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import philox, unweight as uw


def _density_case(seed=3, n=200_000):
    x = philox.uniforms(seed, n, 1)[0]
    w = 3.0 * x * x
    u = uw.acceptance_uniforms(seed, n)
    return x, w, u


def test_kept_events_follow_the_weight_density():
    x, w, u = _density_case()
    kept, fac = uw.unweight(w, u, 3.0)
    n = x.shape[0]
    rate = kept.size / n
    assert abs(rate - 1 / 3) < 4 * np.sqrt((1 / 3) * (2 / 3) / n)
    assert stats.kstest(x[kept], lambda t: t ** 3).pvalue > 1e-3
    assert stats.kstest(x[kept], 'uniform').pvalue < 1e-6        # not the input distribution
    assert (fac == 1.0).all()
    assert (np.diff(kept) > 0).all()


def test_batch_max_reference():
    x, w, u = _density_case(seed=4, n=50_000)
    wm = uw.batch_max(w)
    assert wm == w.max()
    kept, _ = uw.unweight(w, u, wm)
    assert int(np.argmax(w)) in set(kept.tolist())               # the largest weight is always kept
    assert uw.batch_max(np.array([-1.0, np.nan, 0.0])) == 0.0


def test_exact_cases():
    w = np.array([0.0, -1.0, np.nan, 1.0, 2.0, 5.0, 1.0, 0.5])
    u = np.array([0.0, 0.0, 0.0, 0.5, 0.99, 0.99, 0.0, 0.25])
    kept, fac = uw.unweight(w, u, 2.0)
    # 0, -1, NaN never; 1.0 at u = 0.5: 0.5 * 2 = 1.0 is not < 1.0; 2.0 = w_max always;
    # 5.0 > w_max: factor 2.5; u = 0 keeps any positive weight; 0.25 * 2 = 0.5 is not < 0.5
    assert kept.tolist() == [4, 5, 6]
    assert fac.tolist() == [1.0, 2.5, 1.0]
    # nothing positive: nothing kept
    assert uw.unweight(np.zeros(4), np.zeros(4), 0.0)[0].size == 0


def test_acceptance_stream_is_uniform_and_separate():
    u = uw.acceptance_uniforms(9, 100_000)
    assert stats.kstest(u, 'uniform').pvalue > 1e-3
    x = philox.uniforms(9, 100_000, 2)
    assert not np.any(u == x[0]) and not np.any(u == x[1])
    # the stream continues across offsets
    assert np.array_equal(uw.acceptance_uniforms(9, 10, offset=5), u[5:15])


def _plant(fn):
    """Run the pins against a planted variant of unweight."""
    orig = uw.unweight
    uw.unweight = fn
    try:
        failed = False
        for t in (test_kept_events_follow_the_weight_density, test_exact_cases):
            try:
                t()
            except AssertionError:
                failed = True
        return failed
    finally:
        uw.unweight = orig


def test_planted_mistakes_are_caught():
    def non_strict(w, u, w_max):
        w = np.asarray(w, dtype=np.float64)
        kept = np.nonzero((w > 0) & (u * w_max <= w))[0]
        return kept, np.where(w[kept] > w_max, w[kept] / w_max, 1.0)

    def no_reference(w, u, w_max):
        w = np.asarray(w, dtype=np.float64)
        kept = np.nonzero((w > 0) & (u < w))[0]
        return kept, np.ones(kept.size)

    def unit_factors(w, u, w_max):
        w = np.asarray(w, dtype=np.float64)
        kept = np.nonzero((w > 0) & (u * w_max < w))[0]
        return kept, np.ones(kept.size)

    def keeps_nonpositive(w, u, w_max):
        w = np.asarray(w, dtype=np.float64)
        kept = np.nonzero(~(u * w_max >= w))[0]
        return kept, np.ones(kept.size)

    for f in (non_strict, no_reference, unit_factors, keeps_nonpositive):
        assert _plant(f), f.__name__
