"""Learned split/merge proposal: set features and the exact MH move (test-only).

Not part of the paper (an added form).  A Metropolis-Hastings move in the
collapsed space of partitions (Hastings 1970; split/merge proposals as in
Jain & Neal 2004, which the paper cites for its split/merge framework):

  * move type: split if K = 1, else split or merge with probability 1/2 each
    (uniform word 0 of block (0, t, TAG_MOVE, 0)); target: cluster
    floor(u K) or the floor(u C(K,2))-th pair in lexicographic order (word 1);
    acceptance uniform: word 2;
  * split of cluster C: every point i of C goes to side A with probability
    b_i = clip(sigmoid(MLP(phi_C(x_i))), 1e-6, 1 - 1e-6), drawn as
    u_i < b_i with u_i from word 0 of block (i, t, TAG_BERN, 0); a proposal
    with an empty side is rejected.  The proposal probability of the unordered
    partition {A, B} is q(s) + q(not s);
  * merge of the pair (k1, k2): the exact reverse, with the partition
    probability evaluated on the merged set's features.
With the collapsed target p(partition) proportional to
alpha^K prod_B Gamma(|B|) f(x_B), the Hastings ratio of a split K -> K + 1 is

  alpha Gamma(N_A) f(A) Gamma(N_B) f(B) / (Gamma(N_C) f(C))
  * [P_merge(K+1) / C(K+1, 2)] / [P_split(K) / K * (q(s) + q(not s))]

and a merge uses the reciprocal with the roles of forward and reverse moves
exchanged, so the move leaves the partition posterior invariant whatever the
network's weights are.

Set features phi_C depend only on the statistics (n, sum x, sum x x^T) of
C: the sample mean mu and covariance Sigma (regularised by
1e-9 (1 + tr Sigma / d) I), its eigen-decomposition with eigenvalues in
decreasing order and each eigenvector's largest-magnitude entry made
positive; for the first m axes the coordinate v_j^T (x - mu) / sqrt(lambda_j)
and the eigenvalue share lambda_j / sum lambda.  F = 2m features.
"""
import numpy as np
from scipy.special import gammaln, logsumexp

from . import mlp, niw, rng, sampler

TAG_LEARNSUB = 4
CLIP = 1e-6


def set_frame(n, s, S, m):
    """(mu, P[m][d], ratios[m]) of a set with statistics (n, s, S); features
    of a point x are [P (x - mu), ratios]."""
    s = np.asarray(s, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    d = s.shape[0]
    mu = s / n
    cov = S / n - np.outer(mu, mu)
    cov = 0.5 * (cov + cov.T)
    cov = cov + 1e-9 * (1.0 + np.trace(cov) / d) * np.eye(d)
    lam, V = np.linalg.eigh(cov)
    order = np.argsort(-lam, kind="stable")
    lam = lam[order]
    V = V[:, order]
    for j in range(d):
        a = int(np.argmax(np.abs(V[:, j])))
        if V[a, j] < 0:
            V[:, j] = -V[:, j]
    lam = np.maximum(lam, 1e-300)
    P = (V[:, :m] / np.sqrt(lam[:m])).T
    ratios = lam[:m] / np.sum(lam)
    return mu, P, ratios


def features(x, n, s, S, m):
    mu, P, ratios = set_frame(n, s, S, m)
    X = np.asarray(x, dtype=np.float64)
    U = (X - mu) @ P.T
    return np.concatenate([U, np.broadcast_to(ratios, (X.shape[0], m))], axis=1)


def probs(theta, feats, F):
    o, _ = mlp.forward(theta, feats, F)
    return np.clip(1.0 / (1.0 + np.exp(-o)), CLIP, 1.0 - CLIP)


def log_q_partition(b, side_a):
    """log of q(s) + q(not s) for the unordered partition given by side_a."""
    la = np.log(b)
    lb = np.log1p(-b)
    q_s = np.sum(np.where(side_a, la, lb))
    q_n = np.sum(np.where(side_a, lb, la))
    return float(np.logaddexp(q_s, q_n))


def _stats_of(model, x, idx):
    xs = np.asarray(x, dtype=np.float64)[idx]
    return idx.size, xs.sum(0), xs.T @ xs


def _lml(model, n, s, S):
    return niw.log_marginal(model.prior, n, s, S) if n > 0 else 0.0


def pair_of(p, K):
    k1 = 0
    while p >= K - 1 - k1:
        p -= K - 1 - k1
        k1 += 1
    return k1, k1 + 1 + p


def split_log_h(model, x, z, K, k, theta, m, side):
    """log Hastings ratio of splitting cluster k (labels z, K clusters) into
    side A = points of k with side True and side B, under weights theta."""
    C = np.nonzero(z == k)[0]
    n, s, S = _stats_of(model, x, C)
    b = probs(theta, features(np.asarray(x)[C], n, s, S, m), 2 * m)
    A, B = C[side], C[~side]
    nA, sA, SA = _stats_of(model, x, A)
    nB, sB, SB = _stats_of(model, x, B)
    p_split = 1.0 if K == 1 else 0.5
    lq_fwd = np.log(p_split) - np.log(K) + log_q_partition(b, side)
    lq_rev = np.log(0.5) - np.log((K + 1) * K / 2.0)
    return float(np.log(model.alpha) + gammaln(nA) + _lml(model, nA, sA, SA) + gammaln(nB)
                 + _lml(model, nB, sB, SB) - gammaln(n) - _lml(model, n, s, S) + lq_rev - lq_fwd)


def merge_log_h(model, x, z, K, k1, k2, theta, m):
    """log Hastings ratio of merging clusters k1 < k2 (labels z, K clusters)."""
    C = np.nonzero((z == k1) | (z == k2))[0]
    n, s, S = _stats_of(model, x, C)
    b = probs(theta, features(np.asarray(x)[C], n, s, S, m), 2 * m)
    side = z[C] == k1
    A, B = C[side], C[~side]
    nA, sA, SA = _stats_of(model, x, A)
    nB, sB, SB = _stats_of(model, x, B)
    npairs = K * (K - 1) // 2
    lq_fwd = np.log(0.5) - np.log(npairs)
    p_split_rev = 1.0 if K - 1 == 1 else 0.5
    lq_rev = np.log(p_split_rev) - np.log(K - 1) + log_q_partition(b, side)
    return float(-(np.log(model.alpha) + gammaln(nA) + _lml(model, nA, sA, SA) + gammaln(nB)
                   + _lml(model, nB, sB, SB) - gammaln(n) - _lml(model, n, s, S)) + lq_rev - lq_fwd)


def move(model, x, state, theta, m, t):
    """One learned move on a Gaussian model; returns (new_state, info dict)."""
    K = state.K
    w = rng.block(model.seed, t, 0, rng.TAG_MOVE, 0)
    u_type, u_pick, u_acc = (float(rng.uniform(w[j])) for j in range(3))
    do_split = K == 1 or u_type < 0.5
    z = state.z
    info = {"kind": "split" if do_split else "merge", "accepted": False, "log_h": None, "empty": False}
    if do_split:
        k = min(int(u_pick * K), K - 1)
        C = np.nonzero(z == k)[0]
        n, s, S = _stats_of(model, x, C)
        b = probs(theta, features(np.asarray(x)[C], n, s, S, m), 2 * m)
        ub = rng.uniform(rng.block(model.seed, t, C.astype(np.uint64), rng.TAG_BERN, 0)[0])
        side = ub < b
        info.update(target=(k,), b=b, side=side)
        if side.all() or not side.any():
            info["empty"] = True
            return state, info
        lh = split_log_h(model, x, z, K, k, theta, m, side)
        info["log_h"] = lh
        if np.log(u_acc) < lh:
            info["accepted"] = True
            A = C[side]
            znew = z.copy()
            znew[A] = K
            fresh = (rng.block(model.seed, t, C.astype(np.uint64), TAG_LEARNSUB, 0)[0] & np.uint32(1)).astype(np.int64)
            zs = state.zsub.copy()
            zs[C] = fresh
            age = np.concatenate([state.age, [0]])
            age[k] = 0
            return sampler.State(K + 1, znew, zs, age), info
        return state, info
    npairs = K * (K - 1) // 2
    p = min(int(u_pick * npairs), npairs - 1)
    k1, k2 = pair_of(p, K)
    lh = merge_log_h(model, x, z, K, k1, k2, theta, m)
    info.update(target=(k1, k2), log_h=lh)
    if np.log(u_acc) < lh:
        info["accepted"] = True
        znew = z.copy()
        zs = state.zsub.copy()
        zs[z == k1] = 0
        zs[z == k2] = 1
        znew[z == k2] = k1
        age = state.age.copy()
        age[k1] = 0
        keep = np.ones(K, dtype=bool)
        keep[k2] = False
        return sampler.compact(sampler.State(K, znew, zs, age), keep), info
    return state, info


def training_set(model, x, state, m, with_rows=False):
    """Features and targets from the sampler's own sub-labels: points of every
    cluster with age >= burn_out and both sub-clusters non-empty; target 1 for
    sub-label l, flipped per cluster so that the l side has the larger mean
    first principal coordinate.  Rows come cluster by cluster (each in index
    order); with_rows also returns their point indices."""
    X, Y, R = [], [], []
    for k in range(state.K):
        if state.age[k] < model.burn_out:
            continue
        C = np.nonzero(state.z == k)[0]
        y = (state.zsub[C] == 0).astype(np.float64)
        if y.all() or not y.any():
            continue
        n, s, S = _stats_of(model, x, C)
        f = features(np.asarray(x)[C], n, s, S, m)
        if f[y == 1, 0].mean() < f[y == 0, 0].mean():
            y = 1.0 - y
        X.append(f)
        Y.append(y)
        R.append(C)
    if not X:
        out = (np.zeros((0, 2 * m)), np.zeros(0), np.zeros(0, dtype=np.int64))
    else:
        out = (np.concatenate(X), np.concatenate(Y), np.concatenate(R))
    return out if with_rows else out[:2]
