"""Pins for the Dirichlet-multinomial oracle against scipy and the Polya urn."""
import numpy as np
from scipy import stats
from scipy.special import gammaln

from oracle import dirmult


def test_log_marginal_matches_scipy_dirichlet_multinomial():
    beta = np.array([0.5, 1.0, 2.0, 0.1, 3.0])
    pr = dirmult.DirPrior(beta)
    c = np.array([3, 0, 7, 1, 2])
    T = c.sum()
    coef = gammaln(T + 1) - np.sum(gammaln(c + 1))
    ref = stats.dirichlet_multinomial(beta, T).logpmf(c)
    assert np.isclose(dirmult.log_marginal(pr, c) + coef, ref, rtol=1e-12)


def test_log_marginal_polya_urn_chain_rule():
    beta = np.array([0.7, 1.3, 0.2])
    pr = dirmult.DirPrior(beta)
    tokens = [0, 2, 2, 1, 0, 0, 2, 1]
    lp = 0.0
    counts = np.zeros(3)
    for v in tokens:
        lp += np.log((beta[v] + counts[v]) / (beta.sum() + counts.sum()))
        counts[v] += 1
    assert np.isclose(dirmult.log_marginal(pr, counts), lp, rtol=1e-12)


def test_dirichlet_draw_mean():
    pr = dirmult.DirPrior(np.ones(4))
    c = np.array([10, 0, 5, 30])
    th = np.exp(np.stack([dirmult.sample_log_theta(pr, c, 3, 1, e) for e in range(3000)]))
    assert np.allclose(th.sum(1), 1.0)
    assert np.allclose(th.mean(0), (1 + c) / (4 + c.sum()), atol=0.01)


def test_loglik_is_dot_product():
    x = np.array([[1, 2, 0], [0, 0, 5]])
    lt = np.log(np.array([0.2, 0.5, 0.3]))
    assert np.allclose(dirmult.loglik(x, lt), [np.log(0.2) + 2 * np.log(0.5), 5 * np.log(0.3)])
