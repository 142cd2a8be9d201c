"""Helpers of the GPU parity tests: seeded inputs and the comparison rules.

Comparison rules (given fixed parameters and the same (seed, t)):
  * log-likelihood: |l_gpu - l_oracle| <= 1e-5 * M with the scale
    M = |log w| + 1/2 |log|Sigma|| + d/2 log 2pi + 1/2 q (Gaussian; q the
    squared Mahalanobis distance) or |log w| + sum_v x_v |log theta_v|;
  * labels: a point may differ from the oracle only when the oracle's two
    best perturbed scores a, b are closer than
    1e-5 (M_a + M_b) + 4 * 2^-24 (|g_a| + |g_b| + 1);
  * sub-labels (compared where z agrees): only when |gap + L| is below
    1e-5 (M_l + M_r) + 4 * 2^-24 (|L| + 1);
  * statistics: counts bit-exact, moments within 1e-6 of the sum of the
    absolute per-point terms.
"""
import numpy as np

from oracle import niw, rng, sampler

LOG_2PI = np.log(2 * np.pi)


def random_gauss_params(K, d, seed, spread=4.0, cond=10.0):
    g = np.random.Generator(np.random.PCG64(seed))
    mu = g.normal(0, spread, size=(K, 3, d))
    mu[:, 1:] = mu[:, :1] + g.normal(0, 0.5, size=(K, 2, d))
    sigma = np.empty((K, 3, d, d))
    for k in range(K):
        for c in range(3):
            q, _ = np.linalg.qr(g.standard_normal((d, d)))
            ev = np.exp(g.uniform(0, np.log(cond), size=d)) * 0.3
            sigma[k, c] = (q * ev) @ q.T
            sigma[k, c] = 0.5 * (sigma[k, c] + sigma[k, c].T)
    log_pi = np.log(g.dirichlet(np.ones(K)))
    log_pisub = np.log(g.dirichlet(np.ones(2), size=K))
    return sampler.Params(log_pi, log_pisub, mu=mu, sigma=sigma)


def gauss_points(params, n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    K, _, d = params.mu.shape
    lab = g.integers(0, K, n)
    x = np.empty((n, d))
    for k in range(K):
        idx = np.nonzero(lab == k)[0]
        L = np.linalg.cholesky(params.sigma[k, 0])
        x[idx] = params.mu[k, 0] + g.standard_normal((idx.size, d)) @ L.T
    return x.astype(np.float32)


def comp_array(params):
    """Oracle Params -> the ABI's comp[K][3][d + d*d] (Gaussian) or [K][3][V]."""
    if params.mu is not None:
        K, _, d = params.mu.shape
        return np.concatenate([params.mu, params.sigma.reshape(K, 3, d * d)], axis=2)
    return params.log_theta


def gauss_scale(x, params):
    """M for clusters [N, K] and sub-clusters [N, K, 2]."""
    K, _, d = params.mu.shape
    x = np.asarray(x, dtype=np.float64)
    Mc = np.zeros((x.shape[0], K))
    Ms = np.zeros((x.shape[0], K, 2))
    for k in range(K):
        for c in range(3):
            ld = np.linalg.slogdet(params.sigma[k, c])[1]
            diff = x - params.mu[k, c]
            q = np.einsum("ij,ij->i", diff, np.linalg.solve(params.sigma[k, c], diff.T).T)
            lw = params.log_pi[k] if c == 0 else params.log_pisub[k, c - 1]
            M = abs(lw) + 0.5 * abs(ld) + 0.5 * d * LOG_2PI + 0.5 * q
            if c == 0:
                Mc[:, k] = M
            else:
                Ms[:, k, c - 1] = M
    return Mc, Ms


def mult_scale(x, params):
    K = params.log_theta.shape[0]
    x = np.asarray(x, dtype=np.float64)
    Mc = np.zeros((x.shape[0], K))
    Ms = np.zeros((x.shape[0], K, 2))
    for k in range(K):
        Mc[:, k] = abs(params.log_pi[k]) + x @ np.abs(params.log_theta[k, 0])
        for h in range(2):
            Ms[:, k, h] = abs(params.log_pisub[k, h]) + x @ np.abs(params.log_theta[k, 1 + h])
    return Mc, Ms


def check_loglik(ll_gpu, lc, ls, Mc, Ms):
    K = lc.shape[1]
    err_c = np.abs(ll_gpu[:, :K] - lc) / Mc
    err_s = np.abs(ll_gpu[:, K:].reshape(-1, K, 2) - ls) / Ms
    return max(err_c.max(), err_s.max())


def label_mismatches(seed, t, z_gpu, zs_gpu, lc, ls, Mc, Ms, points=None):
    """Return (bad_cluster, bad_sub, n_tie_cluster, n_tie_sub): points whose
    GPU label differs from the oracle although the oracle's margin exceeds the
    tolerance, and how many differences fell inside the tolerance."""
    N, K = lc.shape
    g = sampler.gumbels(seed, t, N, K, points=points)
    z_o, zs_o = sampler.draw_labels(seed, t, lc, ls, points=points)
    pert = lc + g
    idx = np.arange(N)
    order = np.argsort(-pert, axis=1)
    a = order[:, 0]
    b = order[:, 1] if K > 1 else order[:, 0]
    margin = pert[idx, a] - pert[idx, b]
    tol = 1e-5 * (Mc[idx, a] + Mc[idx, b]) + 4 * 2.0 ** -24 * (np.abs(g[idx, a]) + np.abs(g[idx, b]) + 1)
    diff_c = z_gpu != z_o
    bad_c = np.nonzero(diff_c & (margin > tol))[0]
    L = sampler.logistics(seed, t, N, K, points=points)
    same = ~diff_c
    gap = ls[idx, z_o, 0] - ls[idx, z_o, 1] + L
    tol_s = 1e-5 * (Ms[idx, z_o, 0] + Ms[idx, z_o, 1]) + 4 * 2.0 ** -24 * (np.abs(L) + 1)
    diff_s = same & (zs_gpu != zs_o)
    bad_s = np.nonzero(diff_s & (np.abs(gap) > tol_s))[0]
    return bad_c, bad_s, int(diff_c.sum()) - bad_c.size, int(diff_s.sum()) - bad_s.size


def stats_array(st, family):
    """Oracle Stats -> the ABI's stats layout."""
    K = st.n.shape[0]
    if family == "gaussian":
        d = st.s.shape[2]
        return np.concatenate([st.n[..., None].astype(np.float64), st.s, st.S.reshape(K, 2, d * d)], axis=2)
    return np.concatenate([st.n[..., None], st.s], axis=2).astype(np.int64)
