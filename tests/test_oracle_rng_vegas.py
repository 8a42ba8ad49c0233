"""Pins for the oracle's Philox generator and Vegas algorithm (CPU only)."""
import math
import os

import numpy as np
import pytest

from oracle import philox, vegas

GOLDEN = os.path.join(os.path.dirname(__file__), 'golden')


def _kat_rows():
    rows = []
    for line in open(os.path.join(GOLDEN, 'philox4x32_10_kat.txt')):
        if line.startswith('#') or not line.strip():
            continue
        w = [int(t, 16) for t in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize('row', _kat_rows())
def test_philox_known_answers(row):
    ctr, key, want = row
    got = philox.philox4x32_10(np.array(ctr, dtype=np.uint32), np.array(key, dtype=np.uint32))
    assert [int(v) for v in got] == want


def test_uniforms_range_and_moments():
    x = philox.uniforms(12345, 200000, 3)
    assert x.min() >= 0.0 and x.max() < 1.0
    # mean and variance of U[0,1) within 6 sigma
    for k in range(3):
        assert abs(x[k].mean() - 0.5) < 6 * math.sqrt(1 / 12 / x.shape[1])
        assert abs(x[k].var() - 1 / 12) < 6 * math.sqrt(1 / 180 / x.shape[1])
    # dimensions are uncorrelated
    c = np.corrcoef(x)
    assert np.abs(c - np.eye(3)).max() < 6 / math.sqrt(x.shape[1])


def test_uniforms_offset_consistency():
    a = philox.uniforms(7, 1000, 5, offset=0)
    b = philox.uniforms(7, 400, 5, offset=600)
    assert np.array_equal(a[:, 600:], b)
    c = philox.uniforms(8, 1000, 5)
    assert not np.array_equal(a, c)


def test_uniforms_53_bit_grid():
    x = philox.uniforms(3, 1000, 2)
    assert np.all((x * 2.0 ** 53) == np.floor(x * 2.0 ** 53))


def test_vegas_identity_grid():
    x = philox.uniforms(1, 1000, 4)
    y, b, J = vegas.vegas_map(x, vegas.uniform_grid(4, 50))
    assert np.allclose(y, x, rtol=0, atol=1e-15)
    assert np.allclose(J, 1.0, rtol=1e-14)
    assert np.array_equal(b, np.floor(x * 50).astype(int))


def test_vegas_uniform_histogram_is_fixed_point():
    e = vegas.uniform_grid(3, 50)
    new = vegas.refine(e, np.ones((3, 50)))
    assert np.allclose(new, e, rtol=0, atol=1e-15)
    # also for a non-uniform grid: equal histogram keeps it
    rng = np.random.default_rng(0)
    w = rng.uniform(0.5, 1.5, 50)
    g = np.concatenate([[0.0], np.cumsum(w) / w.sum()])
    new = vegas.refine(g[None, :], np.ones((1, 50)))
    assert np.allclose(new, g[None, :], rtol=0, atol=1e-14)


def test_vegas_refine_alpha_zero_subdivides_support():
    # alpha = 0: every bin with non-zero smoothed weight gets r = 1, so the new
    # edges split the support into equal counts of old bins.  h = (1,1,0,0):
    # smoothed (1, 2/3, 1/3, 0) -> r = (1,1,1,0), sum 3, targets 0.75, 1.5, 2.25.
    e = vegas.uniform_grid(1, 4)
    new = vegas.refine(e, np.array([[1.0, 1.0, 0.0, 0.0]]), alpha=0.0)
    assert np.allclose(new[0], [0.0, 0.1875, 0.375, 0.5625, 1.0], rtol=0, atol=1e-15)


def test_vegas_refine_monotone_and_concentrates():
    rng = np.random.default_rng(1)
    h = rng.uniform(0, 1, (2, 50)) ** 4
    new = vegas.refine(vegas.uniform_grid(2, 50), h)
    assert np.all(np.diff(new, axis=1) > 0)
    # bins where h is largest get narrower than average
    k = np.argmax(h[0])
    assert new[0, k + 1] - new[0, k] < 1.0 / 50


def test_vegas_known_integrals_within_sigma():
    # prod_d (pi/2) sin(pi x_d) integrates to 1 in any d
    for d in (2, 5, 8):
        f = lambda y: np.prod(0.5 * math.pi * np.sin(math.pi * y), axis=0)
        I, sig, chi2, its, _ = vegas.integrate(f, d, 20000, 5, seed=10 + d)
        assert abs(I - 1.0) < 4 * sig, (d, I, sig)


def test_vegas_adapts_to_a_peak():
    # normalised narrow Gaussian product (value 1 up to erf tails)
    w = 0.05
    norm = math.sqrt(2 * math.pi) * w * math.erf(0.5 / (math.sqrt(2) * w))
    d = 3
    f = lambda y: np.prod(np.exp(-0.5 * ((y - 0.5) / w) ** 2) / norm, axis=0)
    I, sig, chi2, its, edges = vegas.integrate(f, d, 20000, 6, seed=4)
    assert abs(I - 1.0) < 4 * sig
    # the grid adapts: last iteration's variance far below the first one's
    assert its[-1][1] < 0.1 * its[0][1]


def test_vegas_combination():
    I, sig, chi2 = vegas.combine([1.0, 3.0], [1.0, 1.0])
    assert I == 2.0 and abs(sig - math.sqrt(0.5)) < 1e-15 and chi2 == 2.0
