"""Pins for the oracle's random-variate transforms: ranges, exact
representability, and distributional agreement with scipy."""
import numpy as np
from scipy import stats
from scipy.special import softmax

from oracle import rng


def test_uniform_range_and_float32_exact():
    w = np.array([0, 1, 511, 512, 2 ** 32 - 1, 2 ** 31], dtype=np.uint32)
    u = rng.uniform(w)
    assert u.min() == 2.0 ** -24 and u.max() == 1 - 2.0 ** -24
    assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_gumbel_and_logistic_bounds():
    w = np.array([0, 2 ** 32 - 1], dtype=np.uint32)
    g = rng.gumbel(w)
    assert np.isclose(g[0], rng.GUMBEL_MIN) and np.isclose(g[1], rng.GUMBEL_MAX)
    assert abs(rng.GUMBEL_MAX - 16.6355) < 1e-3 and abs(rng.GUMBEL_MIN + 2.8116) < 1e-3
    L = rng.logistic(w)
    assert np.isclose(L[1], rng.LOGISTIC_MAX) and np.isclose(L[0], -rng.LOGISTIC_MAX)


def test_gumbel_logistic_normal_distributions():
    w = rng.block(5, 3, np.arange(100_000, dtype=np.uint64), 0, 0)
    assert stats.kstest(rng.gumbel(w[0]), stats.gumbel_r.cdf).pvalue > 1e-3
    assert stats.kstest(rng.logistic(w[1]), stats.logistic.cdf).pvalue > 1e-3
    assert stats.kstest(rng.box_muller(w[2], w[3]), stats.norm.cdf).pvalue > 1e-3


def test_gumbel_max_frequencies_match_softmax():
    logits = np.array([0.3, -1.0, 2.0, 0.0, 1.2, -0.5])
    n = 200_000
    i = np.arange(n, dtype=np.uint64)
    g = np.stack([rng.gumbel(rng.block(11, 2, i, rng.TAG_GUMBEL, k // 4)[k % 4]) for k in range(6)], axis=1)
    z = np.argmax(logits + g, axis=1)
    counts = np.bincount(z, minlength=6)
    exp = softmax(logits) * n
    assert stats.chisquare(counts, exp).pvalue > 1e-3


def test_gamma_variates_match_scipy():
    for shape in (0.3, 1.0, 2.5, 50.0, 1e4):
        lg = rng.log_gamma_variates(9, 1, np.arange(20_000), rng.TAG_WEIGHTS, 0, shape)
        assert stats.kstest(np.exp(lg), stats.gamma(shape).cdf).pvalue > 1e-3, shape


def test_gamma_draws_are_per_element_independent_of_batch():
    shapes = np.array([0.5, 3.0, 700.0])
    full = rng.log_gamma_variates(4, 2, [10, 11, 12], 16, [0, 1, 2], shapes)
    for j in range(3):
        one = rng.log_gamma_variates(4, 2, 10 + j, 16, j, shapes[j])
        assert one[0] == full[j]


def test_chi2_variates():
    lc = rng.log_chi2_variates(3, 1, np.arange(20_000), rng.TAG_NIW, 5, 7.5)
    assert stats.kstest(np.exp(lc), stats.chi2(7.5).cdf).pvalue > 1e-3
