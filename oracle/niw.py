"""Gaussian components with a Normal-Inverse-Wishart prior (test-only, float64).

The component model of Sec. 2.1 (multivariate Gaussian pdf) with the NIW
prior of Sec. 2.2, NIW(mu, Sigma; kappa, m, nu, Psi) = N(mu; m, Sigma/kappa)
IW(Sigma; nu, Psi), kappa > 0, nu > d - 1.  The paper defers the posterior and
marginal-likelihood expressions to the cited theses/textbook (Sec. 2.3, the
split Hastings ratio); the standard conjugate results (Gelman et al., BDA3,
Sec. 3.6) are written out here.
"""
import numpy as np
from scipy.special import gammaln

from . import rng

LOG_PI = np.log(np.pi)
LOG_2PI = np.log(2.0 * np.pi)


class NIWPrior:
    def __init__(self, kappa, m, nu, psi):
        self.kappa = float(kappa)
        self.m = np.asarray(m, dtype=np.float64).copy()
        self.nu = float(nu)
        self.psi = np.asarray(psi, dtype=np.float64).copy()
        self.d = self.m.shape[0]
        if not (self.kappa > 0 and self.nu > self.d - 1):
            raise ValueError("NIW prior needs kappa > 0 and nu > d - 1")


def log_multigamma(a, d):
    """log Gamma_d(a) = d(d-1)/4 log(pi) + sum_{j=1..d} lgamma(a + (1-j)/2)."""
    j = np.arange(1, d + 1)
    return 0.25 * d * (d - 1) * LOG_PI + float(np.sum(gammaln(a + 0.5 * (1 - j))))


def logdet_spd(a):
    """log|A| of an SPD matrix through its Cholesky factor."""
    L = np.linalg.cholesky(a)
    return 2.0 * float(np.sum(np.log(np.diag(L))))


def posterior(prior, n, s, S):
    """NIW posterior hyper-parameters from statistics (n, s = sum x, S = sum x x^T).

    kappa_n = kappa + n, nu_n = nu + n, m_n = (kappa m + s) / kappa_n,
    Psi_n = Psi + C + (kappa n / kappa_n) (xbar - m)(xbar - m)^T with C the
    scatter about the sample mean xbar (BDA3 Sec. 3.6).  n = 0 returns the prior.
    """
    n = float(n)
    kn = prior.kappa + n
    nun = prior.nu + n
    if n == 0:
        return kn, prior.m.copy(), nun, prior.psi.copy()
    s = np.asarray(s, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    xbar = s / n
    C = S - n * np.outer(xbar, xbar)
    dm = xbar - prior.m
    mn = (prior.kappa * prior.m + s) / kn
    psin = prior.psi + C + (prior.kappa * n / kn) * np.outer(dm, dm)
    psin = 0.5 * (psin + psin.T)
    return kn, mn, nun, psin


def log_marginal(prior, n, s, S):
    """log p(x_1..x_n | prior) for n points with statistics (n, s, S).

    -(n d / 2) log pi + log Gamma_d(nu_n/2) - log Gamma_d(nu/2)
    + (nu/2) log|Psi| - (nu_n/2) log|Psi_n| + (d/2)(log kappa - log kappa_n).
    The empty set has marginal likelihood 1 (log 0.0).
    """
    d = prior.d
    if n == 0:
        return 0.0
    kn, mn, nun, psin = posterior(prior, n, s, S)
    return (-0.5 * n * d * LOG_PI
            + log_multigamma(0.5 * nun, d) - log_multigamma(0.5 * prior.nu, d)
            + 0.5 * prior.nu * logdet_spd(prior.psi) - 0.5 * nun * logdet_spd(psin)
            + 0.5 * d * (np.log(prior.kappa) - np.log(kn)))


def bartlett_draw_index(d):
    """Draw-number layout of one NIW draw of dimension d.

    Returns (offdiag, diag, eps): offdiag[i, j] (i > j) is the normal draw of
    the Bartlett factor entry A[i, j]; diag[i] the chi-square draw of A[i, i];
    eps[r] the normal draw of the mean's noise vector.
    """
    off = np.full((d, d), -1, dtype=np.int64)
    q = 0
    for i in range(d):
        for j in range(i):
            off[i, j] = q
            q += 1
    diag = np.arange(q, q + d, dtype=np.int64)
    eps = np.arange(q + d, q + 2 * d, dtype=np.int64)
    return off, diag, eps


def sample(kappa_n, m_n, nu_n, psi_n, seed, t, entity):
    """Draw (mu, Sigma) ~ NIW(kappa_n, m_n, nu_n, Psi_n) with Bartlett's method.

    Psi_n = L L^T (lower Cholesky).  A is lower triangular with
    A[i, i] = sqrt(chi2(nu_n - i)) (i = 0..d-1) and A[i, j] ~ N(0, 1) for i > j,
    so A A^T ~ Wishart(nu_n, I) (Bartlett 1933) and the precision
    Lambda = L^-T A A^T L^-1 ~ Wishart(nu_n, Psi_n^-1).  Hence
    Sigma = Lambda^-1 = F F^T with F = L A^-T, and mu = m_n + F eps / sqrt(kappa_n)
    is N(m_n, Sigma / kappa_n).  Draw numbers follow `bartlett_draw_index`
    under tag TAG_NIW.
    """
    d = len(m_n)
    off, diag, eps_q = bartlett_draw_index(d)
    A = np.zeros((d, d))
    if d > 1:
        ii, jj = np.nonzero(off >= 0)
        A[ii, jj] = rng.normals(seed, t, entity, rng.TAG_NIW, off[ii, jj])
    A[np.arange(d), np.arange(d)] = np.exp(0.5 * rng.log_chi2_variates(
        seed, t, entity, rng.TAG_NIW, diag, nu_n - np.arange(d)))
    eps = rng.normals(seed, t, entity, rng.TAG_NIW, eps_q)
    L = np.linalg.cholesky(psi_n)
    # F = L A^{-T}: solve F A^T = L, i.e. A F^T = L^T
    F = np.linalg.solve(A, L.T).T
    sigma = F @ F.T
    sigma = 0.5 * (sigma + sigma.T)
    mu = m_n + F @ eps / np.sqrt(kappa_n)
    return mu, sigma


def logpdf(x, mu, sigma):
    """log N(x; mu, Sigma) for the rows of x (Sec. 2.1, Gaussian pdf)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    d = x.shape[1]
    sign, logdet = np.linalg.slogdet(sigma)
    if sign <= 0:
        raise np.linalg.LinAlgError("covariance is not positive definite")
    diff = x - mu
    sol = np.linalg.solve(sigma, diff.T).T
    maha = np.einsum("ij,ij->i", diff, sol)
    return -0.5 * (d * LOG_2PI + logdet + maha)
