"""Pins for the NIW oracle: multivariate-gamma and marginal-likelihood closed
forms against independent routes (scipy's multigammaln, the chain rule of
Student-t predictives, 1-D quadrature), posterior invariants and the
Monte-Carlo behaviour of the Bartlett draw."""
import numpy as np
import pytest
from scipy import integrate, stats
from scipy.special import multigammaln

from oracle import niw


def _prior(d, seed=0):
    g = np.random.Generator(np.random.PCG64(seed))
    a = g.standard_normal((d, d))
    return niw.NIWPrior(1.7, g.standard_normal(d), d + 2.5, a @ a.T + d * np.eye(d))


def _stats(x):
    return x.shape[0], x.sum(0), x.T @ x


def test_log_multigamma_matches_scipy():
    for d in (1, 2, 5, 32):
        for a in (d / 2 + 0.3, d / 2 + 7.25, 1000.5):
            assert np.isclose(niw.log_multigamma(a, d), multigammaln(a, d), rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("d", [1, 2, 4])
def test_log_marginal_equals_chain_of_t_predictives(d):
    # p(x_1..x_n) = prod_i p(x_i | x_<i); the NIW predictive is a multivariate t
    # with nu_n - d + 1 dof, location m_n, shape Psi_n (kappa_n + 1)/(kappa_n (nu_n - d + 1)).
    pr = _prior(d, d)
    g = np.random.Generator(np.random.PCG64(10 + d))
    x = g.standard_normal((7, d)) * 1.5 + 0.7
    total = 0.0
    for i in range(x.shape[0]):
        kn, mn, nun, psin = niw.posterior(pr, *_stats(x[:i])) if i else (pr.kappa, pr.m, pr.nu, pr.psi)
        dof = nun - d + 1
        shape = psin * (kn + 1) / (kn * dof)
        total += stats.multivariate_t(loc=mn, shape=shape, df=dof).logpdf(x[i])
    assert np.isclose(niw.log_marginal(pr, *_stats(x)), total, rtol=1e-11, atol=1e-9)


def test_log_marginal_1d_quadrature():
    # d = 1: integrate N(x | mu, s2) N(mu | m, s2/kappa) InvGamma(s2 | nu/2, psi/2) numerically.
    pr = niw.NIWPrior(0.8, [0.3], 3.0, [[2.0]])
    x = np.array([0.1, 1.4, -0.6])

    def integrand(mu, ls2):
        s2 = np.exp(ls2)
        lik = np.prod(stats.norm.pdf(x, mu, np.sqrt(s2)))
        return (lik * stats.norm.pdf(mu, pr.m[0], np.sqrt(s2 / pr.kappa))
                * stats.invgamma.pdf(s2, pr.nu / 2, scale=pr.psi[0, 0] / 2) * s2)

    val, _ = integrate.dblquad(integrand, -14.0, 14.0, -20.0, 20.0, epsabs=1e-14, epsrel=1e-10)
    assert np.isclose(niw.log_marginal(pr, *_stats(x[:, None])), np.log(val), rtol=1e-7)


def test_posterior_batch_equals_sequential_and_empty_is_prior():
    pr = _prior(3, 4)
    g = np.random.Generator(np.random.PCG64(3))
    x = g.standard_normal((20, 3))
    kn, mn, nun, psin = niw.posterior(pr, *_stats(x))
    pr2 = niw.NIWPrior(*niw.posterior(pr, *_stats(x[:8])))
    kn2, mn2, nun2, psin2 = niw.posterior(pr2, *_stats(x[8:]))
    assert np.isclose(kn, kn2) and np.isclose(nun, nun2)
    assert np.allclose(mn, mn2, rtol=1e-12) and np.allclose(psin, psin2, rtol=1e-11)
    k0, m0, n0, p0 = niw.posterior(pr, 0, np.zeros(3), np.zeros((3, 3)))
    assert k0 == pr.kappa and np.all(m0 == pr.m) and np.all(p0 == pr.psi)
    assert niw.log_marginal(pr, 0, np.zeros(3), np.zeros((3, 3))) == 0.0


def test_logpdf_matches_scipy():
    pr = _prior(5, 8)
    g = np.random.Generator(np.random.PCG64(1))
    x = g.standard_normal((30, 5))
    mu = g.standard_normal(5)
    ref = stats.multivariate_normal(mu, pr.psi).logpdf(x)
    assert np.allclose(niw.logpdf(x, mu, pr.psi), ref, rtol=1e-12, atol=1e-10)


def test_bartlett_draw_moments_and_distribution():
    d = 3
    pr = _prior(d, 2)
    kn, mn, nun, psin = 4.0, np.array([1.0, -2.0, 0.5]), 9.0, pr.psi
    n = 4000
    sig = np.empty((n, d, d))
    mus = np.empty((n, d))
    for e in range(n):
        mus[e], sig[e] = niw.sample(kn, mn, nun, psin, seed=77, t=3, entity=e)
    mean_sig = sig.mean(0)
    expect = psin / (nun - d - 1)
    assert np.allclose(mean_sig, expect, rtol=0.08, atol=0.05 * np.abs(expect).max())
    assert np.allclose(mus.mean(0), mn, atol=4 * np.sqrt(np.diag(expect) / kn / n).max() + 0.02)
    ref = stats.invwishart(df=nun, scale=psin).rvs(size=n, random_state=5)
    ld = np.linalg.slogdet(sig)[1]
    ldr = np.linalg.slogdet(ref)[1]
    assert stats.ks_2samp(ld, ldr).pvalue > 1e-3
    tr = np.trace(sig, axis1=1, axis2=2)
    assert stats.ks_2samp(tr, np.trace(ref, axis1=1, axis2=2)).pvalue > 1e-3
    # conditional mean law: (mu - m_n) scaled by Sigma^-1/2 sqrt(kappa_n) is standard normal
    zs = np.array([np.linalg.solve(np.linalg.cholesky(sig[e] / kn), mus[e] - mn) for e in range(n)])
    assert stats.kstest(zs.ravel(), stats.norm.cdf).pvalue > 1e-3


def test_bartlett_draw_index_layout():
    off, diag, eps = niw.bartlett_draw_index(4)
    used = sorted(list(off[off >= 0]) + list(diag) + list(eps))
    assert used == list(range(4 * 3 // 2 + 8))
