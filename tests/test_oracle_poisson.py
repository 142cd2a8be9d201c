"""Pins of the oracle's Poisson family (Gamma prior): the marginal
likelihood against numerical quadrature and against the chain rule of
negative-binomial predictives, the posterior draws against the Gamma
posterior (moments and a KS test), the component log-likelihood against
scipy, and one sampler step."""
import numpy as np
import pytest
from scipy import integrate, stats
from scipy.special import gammaln

from oracle import poisson, sampler


def test_log_marginal_by_quadrature():
    prior = poisson.GammaPrior([2.5], [0.7])
    x = np.array([3, 0, 5, 2, 7])
    a, b = 2.5, 0.7

    def integrand(lam):
        # prod_i lam^x_i e^-lam (no 1/x!) times the Gamma(a, b) density
        return np.exp(np.sum(x) * np.log(lam) - x.size * lam + a * np.log(b) - gammaln(a) + (a - 1) * np.log(lam)
                      - b * lam)

    val, _ = integrate.quad(integrand, 0, np.inf, limit=200)
    assert np.isclose(poisson.log_marginal(prior, x.size, [x.sum()]), np.log(val), rtol=1e-9)


def test_log_marginal_chain_rule_negative_binomial():
    g = np.random.Generator(np.random.PCG64(3))
    d = 4
    prior = poisson.GammaPrior(g.uniform(0.5, 3.0, d), g.uniform(0.2, 2.0, d))
    X = g.poisson(3.0, size=(9, d))
    total = 0.0
    for i in range(X.shape[0]):
        n, s = i, X[:i].sum(0)
        r = prior.shape + s
        p = (prior.rate + n) / (prior.rate + n + 1)
        # predictive of point i given the first i: negative binomial per coordinate, times prod x! back
        total += np.sum(stats.nbinom.logpmf(X[i], r, p) + gammaln(X[i] + 1))
    assert np.isclose(poisson.log_marginal(prior, X.shape[0], X.sum(0)), total, rtol=1e-11)
    assert poisson.log_marginal(prior, 0, np.zeros(d)) == 0.0


def test_posterior_draws_are_gamma():
    prior = poisson.GammaPrior([1.5, 4.0], [0.5, 2.0])
    n, s = 12, np.array([30, 7])
    draws = np.array([np.exp(poisson.sample_log_lambda(prior, n, s, 9, t, 4)) for t in range(1, 4001)])
    shape = prior.shape + s
    rate = prior.rate + n
    assert np.allclose(draws.mean(0), shape / rate, rtol=0.02)
    assert np.allclose(draws.var(0), shape / rate ** 2, rtol=0.1)
    for j in range(2):
        assert stats.kstest(draws[:, j], stats.gamma(shape[j], scale=1 / rate[j]).cdf).pvalue > 1e-3


def test_loglik_against_scipy():
    g = np.random.Generator(np.random.PCG64(5))
    x = g.poisson(2.0, size=(50, 3))
    ll = np.log(np.array([0.7, 3.0, 12.0]))
    ref = stats.poisson.logpmf(x, np.exp(ll)).sum(1) + gammaln(x + 1).sum(1)
    assert np.allclose(poisson.loglik(x, ll), ref, rtol=1e-12)


def test_sampler_step_poisson():
    g = np.random.Generator(np.random.PCG64(8))
    rates = np.array([[1.0, 9.0, 0.5], [8.0, 1.0, 4.0]])
    lab = g.integers(0, 2, 400)
    x = g.poisson(rates[lab])
    model = sampler.Model("poisson", 2.0, poisson.GammaPrior(np.ones(3), np.ones(3)), seed=3, burn_out=0)
    st = sampler.initial_state(model, x.shape[0])
    for t in range(1, 31):
        st, info = sampler.step(model, x, st, t)
        sts = sampler.suffstats(model, x, st.z, st.zsub, st.K)
        assert sts.n.sum() == x.shape[0] and sts.s.sum() == x.sum()
    from oracle import nmi
    assert st.K >= 2 and nmi.nmi(lab, st.z) > 0.8
