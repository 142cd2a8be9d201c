"""One iteration of the sub-cluster split/merge DPMM sampler (test-only, float64).

Follows Sec. 2.3 (augmented space, restricted Gibbs sampler, split/merge
framework, split Hastings ratio) and Sec. 4.1 (steps (a)-(f): cluster weights
eq. sample_weights, sub-cluster weights eq. sample_sub_weights, cluster and
sub-cluster parameters eqs. sample_params / sample_sub_params, labels eq.
sample_labels, sub-labels eq. sample_sub_labels; then split proposals eq.
sample_splits and merge proposals eq. sample_merges), with the parallel-merge
constraint of Sec. 4.3.

Readings taken where the paper is silent or garbled (each also listed in the
design notes of the repository):
  * sub-label weights are the sub-cluster weights pi-bar (the printed pi in
    eq. sample_sub_labels is read as pi-bar, defined by eq. sample_sub_weights);
  * the cluster-weight Dirichlet includes the alpha slot (eq. sample_weights);
  * the split ratio's second sub-cluster is the right one (C-bar_{k,r});
  * merge ratio: eq. sample_merges by default ("paper"); the Sec. 2.3 sentence
    H_merge = 1/H_split is available as merge_form="inverse_split";
  * empty clusters are deleted (stable compaction) after the statistics step;
    an empty sub-cluster has prior parameters and marginal likelihood 1, and a
    split with an empty side is rejected;
  * after an accepted split both new clusters get fresh random sub-labels; the
    left part keeps slot k and the right part is appended at slot
    K + (rank of k among this iteration's accepted splits);
  * after an accepted merge of k1 < k2 the merged cluster keeps slot k1, its
    old k1 points get sub-label l and its old k2 points sub-label r;
  * merges visit pairs in lexicographic order; a cluster that split or merged
    in this iteration is not eligible again; a cluster younger than burn_out
    iterations is not eligible to split or merge; new clusters have age 0 and
    every age grows by one at the end of an iteration;
  * initial state: one cluster, random sub-labels drawn at t = 0;
  * ties in the Gumbel-max go to the lowest cluster index.
Labels: z in 0..K-1, sub-label 0 = l, 1 = r.  Components of cluster k are
indexed c = 0 (cluster), 1 (sub l), 2 (sub r); their random-stream entity is
3k + c.
"""
from dataclasses import dataclass, field

import numpy as np
from scipy.special import gammaln, logsumexp

from . import dirmult, niw, poisson, rng


@dataclass
class Model:
    family: str            # "gaussian", "multinomial" or "poisson"
    alpha: float
    prior: object          # niw.NIWPrior or dirmult.DirPrior
    seed: int
    burn_out: int = 15
    merge_form: str = "paper"   # or "inverse_split"


@dataclass
class State:
    K: int
    z: np.ndarray          # int64[N]
    zsub: np.ndarray       # int64[N], 0 = l, 1 = r
    age: np.ndarray        # int64[K]


@dataclass
class Stats:
    """Per sub-cluster statistics; a cluster's statistics are the sum of its two.

    Gaussian: n[K,2], s[K,2,d] = sum x, S[K,2,d,d] = sum x x^T.
    Multinomial and Poisson: n[K,2] point counts, s[K,2,V] summed counts (S unused).
    """
    n: np.ndarray
    s: np.ndarray
    S: np.ndarray = None

    def cluster(self, k):
        S = None if self.S is None else self.S[k].sum(axis=0)
        return int(self.n[k].sum()), self.s[k].sum(axis=0), S

    def sub(self, k, h):
        S = None if self.S is None else self.S[k, h]
        return int(self.n[k, h]), self.s[k, h], S


@dataclass
class Params:
    """Sampled parameters of K clusters and their 2K sub-clusters.

    log_pi[K], log_pisub[K,2]; Gaussian: mu[K,3,d], sigma[K,3,d,d];
    multinomial: log_theta[K,3,V].  Index 0 of axis 1 is the cluster, 1 and 2
    its sub-clusters l and r.
    """
    log_pi: np.ndarray
    log_pisub: np.ndarray
    mu: np.ndarray = None
    sigma: np.ndarray = None
    log_theta: np.ndarray = None

    @property
    def K(self):
        return self.log_pi.shape[0]


@dataclass
class IterInfo:
    K: int = 0
    splits: int = 0
    merges: int = 0
    logpost: float = 0.0
    split_log_h: list = field(default_factory=list)
    merge_log_h: list = field(default_factory=list)


# ----------------------------------------------------------------------------
# initial state and statistics


def initial_state(model, n_points):
    """K = 1, every z = 0, sub-labels from TAG_SUBINIT at t = 0, age 0."""
    i = np.arange(n_points, dtype=np.uint64)
    w = rng.block(model.seed, 0, i, rng.TAG_SUBINIT, 0)[0]
    zsub = (w & np.uint32(1)).astype(np.int64)
    return State(K=1, z=np.zeros(n_points, dtype=np.int64), zsub=zsub,
                 age=np.zeros(1, dtype=np.int64))


def suffstats(model, x, z, zsub, K):
    """Sufficient statistics per sub-cluster (Sec. 4.4, statistics update)."""
    z = np.asarray(z); zsub = np.asarray(zsub)
    seg = 2 * z + zsub
    if model.family == "gaussian":
        x = np.asarray(x, dtype=np.float64)
        d = x.shape[1]
        n = np.bincount(seg, minlength=2 * K).astype(np.int64).reshape(K, 2)
        s = np.zeros((2 * K, d))
        S = np.zeros((2 * K, d, d))
        for g in range(2 * K):
            xs = x[seg == g]
            s[g] = xs.sum(axis=0)
            S[g] = xs.T @ xs
        return Stats(n=n, s=s.reshape(K, 2, d), S=S.reshape(K, 2, d, d))
    x = np.asarray(x, dtype=np.int64)
    V = x.shape[1]
    n = np.bincount(seg, minlength=2 * K).astype(np.int64).reshape(K, 2)
    s = np.zeros((2 * K, V), dtype=np.int64)
    for g in range(2 * K):
        s[g] = x[seg == g].sum(axis=0)
    return Stats(n=n, s=s.reshape(K, 2, V))


def log_marginal(model, n, s, S):
    if model.family == "gaussian":
        return niw.log_marginal(model.prior, n, s, S)
    if model.family == "poisson":
        return poisson.log_marginal(model.prior, n, s)
    return dirmult.log_marginal(model.prior, s) if n > 0 else 0.0


# ----------------------------------------------------------------------------
# steps (a)-(d): weights and parameters


def sample_weights(model, stats, t):
    """Steps (a) and (b): log pi ~ Dir(N_1..N_K, alpha) and log pi-bar_k."""
    K = stats.n.shape[0]
    Nk = stats.n.sum(axis=1).astype(np.float64)
    if np.any(Nk <= 0):
        raise ValueError("empty cluster reached the weight step")
    shapes = np.concatenate([Nk, [model.alpha]])
    lg = rng.log_gamma_variates(model.seed, t, np.arange(K + 1), rng.TAG_WEIGHTS, 0, shapes)
    log_pi = lg[:K] - logsumexp(lg)
    sub_shapes = stats.n.astype(np.float64) + 0.5 * model.alpha
    ent = np.repeat(np.arange(K), 2)
    q = np.tile(np.arange(2), K)
    lgs = rng.log_gamma_variates(model.seed, t, ent, rng.TAG_SUBWEIGHTS, q, sub_shapes.ravel()).reshape(K, 2)
    log_pisub = lgs - logsumexp(lgs, axis=1, keepdims=True)
    return log_pi, log_pisub


def sample_params(model, stats, t):
    """Steps (a)-(d): weights and the parameters of all 3K components."""
    log_pi, log_pisub = sample_weights(model, stats, t)
    K = stats.n.shape[0]
    if model.family == "gaussian":
        d = model.prior.d
        mu = np.zeros((K, 3, d))
        sigma = np.zeros((K, 3, d, d))
        for k in range(K):
            comps = [stats.cluster(k), stats.sub(k, 0), stats.sub(k, 1)]
            for c, (n, s, S) in enumerate(comps):
                kn, mn, nun, psin = niw.posterior(model.prior, n, s, S)
                mu[k, c], sigma[k, c] = niw.sample(kn, mn, nun, psin, model.seed, t, 3 * k + c)
        return Params(log_pi, log_pisub, mu=mu, sigma=sigma)
    V = model.prior.d
    lt = np.zeros((K, 3, V))
    for k in range(K):
        comps = [stats.cluster(k), stats.sub(k, 0), stats.sub(k, 1)]
        for c, (n, s, _) in enumerate(comps):
            if model.family == "poisson":  # log lambda (rates) in place of log theta
                lt[k, c] = poisson.sample_log_lambda(model.prior, n, s, model.seed, t, 3 * k + c)
            else:
                lt[k, c] = dirmult.sample_log_theta(model.prior, s, model.seed, t, 3 * k + c)
    return Params(log_pi, log_pisub, log_theta=lt)


# ----------------------------------------------------------------------------
# steps (e) and (f): labels and sub-labels


def component_loglik(model, x, params, k, c):
    if model.family == "gaussian":
        return niw.logpdf(x, params.mu[k, c], params.sigma[k, c])
    if model.family == "poisson":
        return poisson.loglik(x, params.log_theta[k, c])
    return dirmult.loglik(x, params.log_theta[k, c])


def loglik(model, x, params):
    """Weighted component log-likelihoods.

    lc[i, k]    = log pi_k + log f(x_i; theta_k)
    ls[i, k, h] = log pi-bar_kh + log f(x_i; theta-bar_kh)
    """
    K = params.K
    N = x.shape[0]
    lc = np.zeros((N, K))
    ls = np.zeros((N, K, 2))
    for k in range(K):
        lc[:, k] = params.log_pi[k] + component_loglik(model, x, params, k, 0)
        for h in range(2):
            ls[:, k, h] = params.log_pisub[k, h] + component_loglik(model, x, params, k, 1 + h)
    return lc, ls


def _points(N, point_offset, points):
    if points is not None:
        return np.asarray(points, dtype=np.uint64)
    return np.arange(N, dtype=np.uint64) + np.uint64(point_offset)


def gumbels(seed, t, N, K, point_offset=0, points=None):
    """g[i, k] for i < N, k < K: block k // 4, word k % 4 of (i, t, TAG_GUMBEL).
    `points` gives the point indices (entities) of the rows, if not 0..N-1."""
    i = _points(N, point_offset, points)
    g = np.zeros((N, K))
    for b in range((K + 3) // 4):
        w = rng.block(seed, t, i, rng.TAG_GUMBEL, b)
        for j in range(4):
            k = 4 * b + j
            if k < K:
                g[:, k] = rng.gumbel(w[j])
    return g


def logistics(seed, t, N, K, point_offset=0, points=None):
    """The sub-label logistics of the rows at step t with K clusters (the word
    of rng.sub_label_word)."""
    i = _points(N, point_offset, points)
    return rng.logistic(rng.sub_label_word(seed, t, i, K))


def draw_labels(seed, t, lc, ls, point_offset=0, points=None):
    """Gumbel-max draw of z (eq. sample_labels) and the logistic draw of the
    sub-label (eq. sample_sub_labels): z = argmax_k lc + g; sub-label l iff
    ls[z, l] - ls[z, r] + L > 0."""
    N, K = lc.shape
    g = gumbels(seed, t, N, K, point_offset, points)
    z = np.argmax(lc + g, axis=1)
    idx = np.arange(N)
    delta = ls[idx, z, 0] - ls[idx, z, 1]
    L = logistics(seed, t, N, K, point_offset, points)
    zsub = np.where(delta + L > 0, 0, 1)
    return z.astype(np.int64), zsub.astype(np.int64)


def sample_labels(model, x, params, t, point_offset=0, points=None):
    lc, ls = loglik(model, x, params)
    return draw_labels(model.seed, t, lc, ls, point_offset, points)


# ----------------------------------------------------------------------------
# compaction, splits and merges


def compact(state, keep):
    """Delete clusters with keep[k] False; survivors keep their order."""
    keep = np.asarray(keep, dtype=bool)
    new_index = np.cumsum(keep) - 1
    z = new_index[state.z]
    return State(K=int(keep.sum()), z=z.astype(np.int64), zsub=state.zsub.copy(),
                 age=state.age[keep].copy())


def drop_empty(model, x, state):
    stats = suffstats(model, x, state.z, state.zsub, state.K)
    keep = stats.n.sum(axis=1) > 0
    if keep.all():
        return state, stats
    state = compact(state, keep)
    return state, suffstats(model, x, state.z, state.zsub, state.K)


def split_log_h(model, stats, k):
    """log H_split (Sec. 2.3 eq. HastingsRatioSplit, Sec. 4.1 eq. sample_splits)."""
    nl, sl, Sl = stats.sub(k, 0)
    nr, sr, Sr = stats.sub(k, 1)
    n, s, S = stats.cluster(k)
    if nl == 0 or nr == 0:
        return -np.inf
    return (np.log(model.alpha) + gammaln(nl) + log_marginal(model, nl, sl, Sl)
            + gammaln(nr) + log_marginal(model, nr, sr, Sr)
            - gammaln(n) - log_marginal(model, n, s, S))


def merge_log_h(model, stats, k1, k2):
    """log H_merge of clusters k1, k2 (Sec. 4.1 eq. sample_merges by default)."""
    n1, s1, S1 = stats.cluster(k1)
    n2, s2, S2 = stats.cluster(k2)
    n = n1 + n2
    s = s1 + s2
    S = None if S1 is None else S1 + S2
    a = model.alpha
    base = (gammaln(n) - np.log(a) - gammaln(n1) - gammaln(n2)
            + log_marginal(model, n, s, S) - log_marginal(model, n1, s1, S1)
            - log_marginal(model, n2, s2, S2))
    if model.merge_form == "inverse_split":
        return base
    return (base + gammaln(a) - gammaln(a + n) + gammaln(0.5 * a + n1)
            + gammaln(0.5 * a + n2) - 2.0 * gammaln(0.5 * a))


def split_merge(model, state, stats, t):
    """Split proposals for every eligible cluster, then merge proposals for every
    eligible pair; returns the relabelled, compacted state and an IterInfo."""
    K = state.K
    info = IterInfo()
    z = state.z.copy()
    zsub = state.zsub.copy()
    age = list(state.age)
    touched = np.zeros(K, dtype=bool)
    # splits
    new_slot = K
    split_of = {}
    for k in range(K):
        if state.age[k] < model.burn_out:
            continue
        lh = split_log_h(model, stats, k)
        u = rng.uniform(rng.block(model.seed, t, k, rng.TAG_SPLIT, 0)[0])
        info.split_log_h.append((k, lh))
        if np.log(u) < lh:
            split_of[k] = new_slot
            touched[k] = True
            new_slot += 1
    if split_of:
        fresh = (rng.block(model.seed, t, np.arange(len(z), dtype=np.uint64),
                           rng.TAG_SUBINIT, 0)[0] & np.uint32(1)).astype(np.int64)
        for k, slot in split_of.items():
            mk = z == k
            right = mk & (zsub == 1)
            z[right] = slot
            zsub[mk] = fresh[mk]
            age[k] = 0
            age.append(0)
    info.splits = len(split_of)
    K_after_split = new_slot
    # merges among the clusters that existed before the splits
    keep = np.ones(K_after_split, dtype=bool)
    for k1 in range(K):
        for k2 in range(k1 + 1, K):
            if touched[k1] or touched[k2]:
                continue
            if state.age[k1] < model.burn_out or state.age[k2] < model.burn_out:
                continue
            lh = merge_log_h(model, stats, k1, k2)
            u = rng.uniform(rng.block(model.seed, t, (k1 << 16) | k2, rng.TAG_MERGE, 0)[0])
            info.merge_log_h.append((k1, k2, lh))
            if np.log(u) < lh:
                touched[k1] = touched[k2] = True
                m1 = z == k1
                m2 = z == k2
                zsub[m1] = 0
                zsub[m2] = 1
                z[m2] = k1
                keep[k2] = False
                age[k1] = 0
                info.merges += 1
    new_state = State(K=K_after_split, z=z, zsub=zsub, age=np.asarray(age, dtype=np.int64))
    if not keep.all():
        new_state = compact(new_state, keep)
    return new_state, info


def log_posterior(model, stats):
    """log p(z | x) up to a constant: K log alpha + lgamma(alpha) - lgamma(alpha + N)
    + sum_k [lgamma(N_k) + log f(C_k; lambda)] (DP partition prior times the
    marginal likelihoods)."""
    K = stats.n.shape[0]
    Nk = stats.n.sum(axis=1)
    N = int(Nk.sum())
    a = model.alpha
    lp = K * np.log(a) + gammaln(a) - gammaln(a + N)
    for k in range(K):
        n, s, S = stats.cluster(k)
        lp += gammaln(n) + log_marginal(model, n, s, S)
    return float(lp)


def step(model, x, state, t):
    """One full iteration t >= 1 (Sec. 4.1 order: (a)-(f), splits, merges)."""
    stats = suffstats(model, x, state.z, state.zsub, state.K)
    params = sample_params(model, stats, t)
    z, zsub = sample_labels(model, x, params, t)
    state = State(K=state.K, z=z, zsub=zsub, age=state.age.copy())
    state, stats = drop_empty(model, x, state)
    state, info = split_merge(model, state, stats, t)
    state.age = state.age + 1
    stats = suffstats(model, x, state.z, state.zsub, state.K)
    info.K = state.K
    info.logpost = log_posterior(model, stats)
    return state, info
