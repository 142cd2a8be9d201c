"""Poisson components with a Gamma prior (test-only, float64).

The paper's software is said to adapt to any exponential-family component
(Sec. 3.4, with Poisson as its example; Sec. 6).  Here a component is a
product of independent Poisson counts, f(x | lambda) = prod_j
Poisson(x_j; lambda_j), with the conjugate prior lambda_j ~ Gamma(a_j, b_j)
(shape a, rate b).  The per-point factor prod_j 1 / x_j! is the same for
every component and cancels in every ratio the sampler forms (split, merge,
label draws, the log posterior up to a constant); it is left out below, as
the multinomial coefficient is for the multinomial family.
"""
import numpy as np
from scipy.special import gammaln

from . import rng


class GammaPrior:
    def __init__(self, shape, rate):
        self.shape = np.asarray(shape, dtype=np.float64).copy()
        self.rate = np.asarray(rate, dtype=np.float64).copy()
        self.d = self.shape.shape[0]
        if self.rate.shape != self.shape.shape or np.any(~(self.shape > 0)) or np.any(~(self.rate > 0)):
            raise ValueError("Gamma prior needs shape > 0 and rate > 0 of one length")


def log_marginal(prior, n, s):
    """log of int prod_i prod_j lambda_j^x_ij e^-lambda_j Gamma(lambda_j; a_j, b_j) d lambda
    for n points with count sums s (the 1 / x_ij! factors left out):

    sum_j [a_j log b_j - lgamma(a_j) + lgamma(a_j + s_j) - (a_j + s_j) log(b_j + n)].
    The empty set gives 0.
    """
    if n == 0:
        return 0.0
    a, b = prior.shape, prior.rate
    s = np.asarray(s, dtype=np.float64)
    return float(np.sum(a * np.log(b) - gammaln(a) + gammaln(a + s) - (a + s) * np.log(b + n)))


def sample_log_lambda(prior, n, s, seed, t, entity):
    """log lambda for lambda_j ~ Gamma(a_j + s_j, b_j + n) (shape, rate): draw
    j of (entity, TAG_DIRTHETA) is a Gamma(a_j + s_j, 1) variate, divided by
    the rate."""
    a = prior.shape + np.asarray(s, dtype=np.float64)
    lg = rng.log_gamma_variates(seed, t, entity, rng.TAG_DIRTHETA, np.arange(a.shape[0]), a)
    return lg - np.log(prior.rate + n)


def loglik(x, log_lambda):
    """sum_j x_j log lambda_j - lambda_j for the rows of the count matrix x."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    ll = np.asarray(log_lambda, dtype=np.float64)
    return x @ ll - np.sum(np.exp(ll))
