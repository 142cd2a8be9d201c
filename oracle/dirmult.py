"""Multinomial components with a Dirichlet prior (test-only, float64).

The pmf components of Sec. 2.1 (mixture of multinomials) with their
conjugate Dirichlet prior; the paper defers the marginal-likelihood
expression to Chang's thesis (Sec. 2.3), so the standard Dirichlet-
multinomial (Polya) form is written out.  Per-point multinomial
coefficients do not depend on the cluster and cancel in every ratio the
sampler forms; they are left out of the log-likelihoods below.
"""
import numpy as np
from scipy.special import gammaln, logsumexp

from . import rng


class DirPrior:
    def __init__(self, beta):
        self.beta = np.asarray(beta, dtype=np.float64).copy()
        self.d = self.beta.shape[0]
        if np.any(~(self.beta > 0)):
            raise ValueError("Dirichlet prior needs beta > 0")


def log_marginal(prior, counts):
    """log of the Dirichlet-multinomial probability of a token sequence.

    lgamma(B) - lgamma(B + T) + sum_v [lgamma(beta_v + c_v) - lgamma(beta_v)]
    with B = sum beta, c = summed counts of the set, T = sum c.
    """
    c = np.asarray(counts, dtype=np.float64)
    B = float(np.sum(prior.beta))
    T = float(np.sum(c))
    return float(gammaln(B) - gammaln(B + T) + np.sum(gammaln(prior.beta + c) - gammaln(prior.beta)))


def sample_log_theta(prior, counts, seed, t, entity):
    """log theta for theta ~ Dir(beta + c): normalised Gamma draws.

    Draw v of (entity, TAG_DIRTHETA) is Gamma(beta_v + c_v); log theta_v is
    its log minus the log-sum-exp over v.
    """
    a = prior.beta + np.asarray(counts, dtype=np.float64)
    lg = rng.log_gamma_variates(seed, t, entity, rng.TAG_DIRTHETA, np.arange(a.shape[0]), a)
    return lg - logsumexp(lg)


def loglik(x, log_theta):
    """sum_v x_v log theta_v for the rows of the count matrix x."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    return x @ np.asarray(log_theta, dtype=np.float64)
