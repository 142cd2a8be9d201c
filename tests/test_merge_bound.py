"""The upper bound on a merge's log Hastings ratio that lets the device skip
the merged set's Cholesky factorisation (a pair whose bound lies below the
log of its uniform is rejected without it).  For clusters 1, 2 with scatters
C1, C2 (about their means), sizes n1, n2, means xbar1, xbar2, and the union U:

  Psi_n(U) = Psi + C1 + C2 + (n1 n2 / n) dx dx^T + (kappa n / kappa_n) (xbar - m)(xbar - m)^T
           >= X + Y + b b^T,   X = Psi/2 + C1,  Y = Psi/2 + C2,  b = sqrt(n1 n2 / n) dx,
  log|X + Y| >= d log(|X|^(1/d) + |Y|^(1/d))                   (Minkowski),
  b^T (X + Y)^-1 b >= |b|^2 / (lambda_max(Psi) + tr C1 + tr C2),

so log|Psi_n(U)| >= LB and the NIW marginal of U is at most its value at LB.
Checked here against the exact merge ratio of the oracle (both merge forms)
on separated, overlapping, nested and coincident clusters."""
import numpy as np
import pytest
from scipy.special import gammaln

from oracle import niw, sampler


def _bound(prior, alpha, stats, k1, k2, paper_form):
    d = prior.d
    n1, s1, S1 = stats.cluster(k1)
    n2, s2, S2 = stats.cluster(k2)
    n = n1 + n2
    x1, x2 = s1 / n1, s2 / n2
    C1 = S1 - n1 * np.outer(x1, x1)
    C2 = S2 - n2 * np.outer(x2, x2)
    lX = niw.logdet_spd(0.5 * prior.psi + C1)
    lY = niw.logdet_spd(0.5 * prior.psi + C2)
    a, c = lX / d, lY / d
    lam = np.max(np.sum(np.abs(prior.psi), axis=1))  # Gershgorin: >= lambda_max(Psi)
    b2 = n1 * n2 / n * np.sum((x1 - x2) ** 2)
    lb = d * (max(a, c) + np.log1p(np.exp(-abs(a - c)))) + np.log1p(b2 / (lam + np.trace(C1) + np.trace(C2)))
    nun, kn = prior.nu + n, prior.kappa + n
    ub_lu = (-0.5 * n * d * niw.LOG_PI + niw.log_multigamma(0.5 * nun, d) - niw.log_multigamma(0.5 * prior.nu, d)
             + 0.5 * prior.nu * niw.logdet_spd(prior.psi) - 0.5 * nun * lb + 0.5 * d * (np.log(prior.kappa) - np.log(kn)))
    l1 = niw.log_marginal(prior, n1, s1, S1)
    l2 = niw.log_marginal(prior, n2, s2, S2)
    g = gammaln(n) - np.log(alpha) - gammaln(n1) - gammaln(n2)
    if paper_form:
        g += gammaln(alpha) - gammaln(alpha + n) + gammaln(0.5 * alpha + n1) + gammaln(0.5 * alpha + n2) \
            - 2 * gammaln(0.5 * alpha)
    return g + ub_lu - l1 - l2


@pytest.mark.parametrize("d", [1, 2, 5, 16])
@pytest.mark.parametrize("form", ["paper", "inverse_split"])
def test_bound_is_above_the_exact_merge_ratio(d, form):
    g = np.random.Generator(np.random.PCG64(40 + d))
    A = g.standard_normal((d, d))
    psi = A @ A.T / d + 0.3 * np.eye(d)
    prior = niw.NIWPrior(0.7, g.standard_normal(d), d + 2.5, psi)
    model = sampler.Model("gaussian", 3.0, prior, seed=1, merge_form=form)
    worst = -np.inf
    for trial in range(60):
        sep = [0.0, 0.3, 1.0, 3.0, 10.0][trial % 5]
        n1, n2 = g.integers(1, 400, 2)
        scale2 = [1.0, 0.05, 20.0][trial % 3]  # nested shapes
        x1 = g.standard_normal((n1, d))
        x2 = g.standard_normal((n2, d)) * scale2 + sep * g.standard_normal(d)
        x = np.concatenate([x1, x2])
        z = np.concatenate([np.zeros(n1, int), np.ones(n2, int)])
        st = sampler.suffstats(model, x, z, g.integers(0, 2, n1 + n2), 2)
        exact = sampler.merge_log_h(model, st, 0, 1)
        ub = _bound(prior, model.alpha, st, 0, 1, form == "paper")
        assert ub >= exact - 1e-9 * (1 + abs(exact)), (trial, ub, exact)
        worst = max(worst, exact - ub)
    assert worst <= 0


def test_bound_prunes_separated_clusters():
    """Far apart, the bound alone rejects the merge (far below log 2^-24)."""
    d = 8
    prior = niw.NIWPrior(1.0, np.zeros(d), d + 3, np.eye(d))
    model = sampler.Model("gaussian", 10.0, prior, seed=1)
    g = np.random.Generator(np.random.PCG64(3))
    x = np.concatenate([g.standard_normal((500, d)), g.standard_normal((500, d)) + 6.0])
    z = np.repeat([0, 1], 500)
    st = sampler.suffstats(model, x, z, g.integers(0, 2, 1000), 2)
    assert _bound(prior, 10.0, st, 0, 1, True) < np.log(2.0 ** -24) - 100
