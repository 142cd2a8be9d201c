"""Exact DPMM partition posterior on tiny inputs (test-only, float64).

Under the model of Sec. 2.2 (pi ~ GEM(alpha), conjugate component prior),
integrating out pi and the component parameters gives the posterior over set
partitions rho of the points (Chinese-restaurant-process prior times the
marginal likelihoods):

    p(rho | x) proportional to alpha^|rho| prod_{B in rho} Gamma(|B|) f(x_B; lambda).

All partitions of N <= 8 points can be listed (Bell(8) = 4140), which turns a
sampler's long-run partition histogram into a checkable quantity.  Neal's
(2000) Algorithm 3 (collapsed Gibbs) is included as a sampler known to leave
this posterior invariant, to validate the comparison harness itself.
"""
import numpy as np
from scipy.special import gammaln, logsumexp


def set_partitions(n):
    """All partitions of range(n) as restricted-growth label tuples."""
    out = []

    def rec(prefix, m):
        if len(prefix) == n:
            out.append(tuple(prefix))
            return
        for b in range(m + 1):
            rec(prefix + [b], max(m, b + 1))

    if n == 0:
        return [()]
    rec([0], 1)
    return out


def canonical(labels):
    """Relabel a label vector in order of first appearance."""
    mapping = {}
    out = []
    for v in labels:
        v = int(v)
        if v not in mapping:
            mapping[v] = len(mapping)
        out.append(mapping[v])
    return tuple(out)


def exact_posterior(x, alpha, log_marginal_of_rows):
    """Dict partition -> posterior probability, by enumeration."""
    N = x.shape[0]
    parts = set_partitions(N)
    logp = np.empty(len(parts))
    cache = {}
    for j, p in enumerate(parts):
        p = np.asarray(p)
        K = p.max() + 1
        lp = K * np.log(alpha)
        for b in range(K):
            rows = tuple(np.nonzero(p == b)[0])
            if rows not in cache:
                cache[rows] = log_marginal_of_rows(list(rows))
            lp += gammaln(len(rows)) + cache[rows]
        logp[j] = lp
    prob = np.exp(logp - logsumexp(logp))
    return {parts[j]: prob[j] for j in range(len(parts))}


def neal_algorithm3(x, alpha, log_marginal_of_rows, iters, rng):
    """Collapsed Gibbs over labels (Neal 2000, Algorithm 3); yields partitions."""
    N = x.shape[0]
    z = np.zeros(N, dtype=np.int64)
    for _ in range(iters):
        for i in range(N):
            others = [j for j in range(N) if j != i]
            zo = z[others]
            labels = sorted(set(zo.tolist()))
            logp = []
            for c in labels:
                members = [others[j] for j in range(len(others)) if zo[j] == c]
                logp.append(np.log(len(members)) + log_marginal_of_rows(sorted(members + [i]))
                            - log_marginal_of_rows(members))
            logp.append(np.log(alpha) + log_marginal_of_rows([i]))
            logp = np.asarray(logp)
            pr = np.exp(logp - logsumexp(logp))
            c = rng.choice(len(pr), p=pr)
            z[i] = labels[c] if c < len(labels) else (max(labels) + 1 if labels else 0)
        yield canonical(z)


def total_variation(hist, exact):
    keys = set(hist) | set(exact)
    total = sum(hist.values())
    return 0.5 * sum(abs(hist.get(k, 0) / total - exact.get(k, 0.0)) for k in keys)
