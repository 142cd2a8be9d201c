"""Seeded synthetic workloads (no sampler arithmetic lives here).

Shapes and distributions follow the synthetic experiments of Sec. 5 (Gaussian
mixtures with random means and Wishart covariances; multinomial mixtures with
Dirichlet topics) at the sizes of the five standard workloads below.  Data
are drawn with numpy's PCG64 from the given seed, so the oracle and the GPU
path can be fed identical inputs.

Workloads
---------
gauss_d2      N=1e4, d=2, 6 Gaussians, means U[-10,10]^2, covariances
              Wishart(4, I), equal weights.
gauss_d32     N=1e6, d=32, 20 Gaussians, means N(0, 25 I), covariances
              Wishart(d+2, I/d), weights Dirichlet(1).
mult_v100     N=1e6 count vectors, V=100, 50 topics Dirichlet(0.1), row
              totals uniform in [50, 200], equal weights.
gauss_d128    N=1e7, d=128, 100 Gaussians, means N(0, 9 I), covariances
              Wishart(d+2, I/d), weights Dirichlet(1).
gauss_d64     N=2e6, d=64, 200 overlapping Gaussians, means N(0, 4 I),
              covariances Wishart(d+2, I/d), weights Dirichlet(1).
news_v20k     N=11314 documents over V=20000 words, 20 topics: the shape
              of the 20newsgroups run of Sec. 5 (a synthetic stand-in; the
              corpus is not used).  Word frequencies of the corpus are
              Zipf(1.07) over a random word order; topic k mixes them 50/50
              with its own Dirichlet(0.02) word distribution; document
              lengths are lognormal (median 150 tokens, sigma 0.9, clipped to
              [10, 4000]); topics uniform.  Rows are compressed sparse rows
              (sorted words, int32 counts): about 160 distinct words a row.
pois_d20      N=1e6 count vectors, d=20 independent Poisson counts, 20
              clusters with rates Gamma(1, scale 10) per cluster and
              coordinate, equal weights (the Poisson family, an exponential
              family of the kind Sec. 3.4 names).
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class GaussianSpec:
    n: int
    d: int
    k: int
    mean_kind: str      # "uniform" (half-width mean_scale) or "normal" (std mean_scale)
    mean_scale: float
    wishart_dof: float  # covariance ~ Wishart(dof, wishart_scale * I)
    wishart_scale: float
    weights: str        # "equal" or "dirichlet1"


@dataclass
class MultinomialSpec:
    n: int
    v: int
    k: int
    topic_conc: float
    total_lo: int
    total_hi: int


@dataclass
class SparseTopicSpec:
    n: int
    v: int
    k: int
    zipf: float         # background word frequencies ~ rank^-zipf
    topic_conc: float   # topic-specific part ~ Dirichlet(topic_conc)
    mix: float          # weight of the background in every topic
    len_median: float   # document length (tokens) ~ lognormal(log median, len_sigma)
    len_sigma: float
    len_lo: int
    len_hi: int


@dataclass
class CSRCounts:
    """Count rows in compressed sparse rows (host arrays)."""
    indptr: np.ndarray   # int64 [n + 1]
    indices: np.ndarray  # int32 [nnz], sorted within a row
    data: np.ndarray     # int32 [nnz]
    shape: tuple

    def rows(self, idx):
        """Dense int32 rows idx (for checks on a few rows)."""
        idx = np.asarray(idx)
        out = np.zeros((idx.size, self.shape[1]), dtype=np.int32)
        for r, i in enumerate(idx):
            a, b = self.indptr[i], self.indptr[i + 1]
            np.add.at(out[r], self.indices[a:b], self.data[a:b])
        return out

    def toarray(self):
        return self.rows(np.arange(self.shape[0]))


@dataclass
class PoissonSpec:
    n: int
    d: int
    k: int
    rate_shape: float   # rates ~ Gamma(rate_shape, scale rate_scale)
    rate_scale: float


WORKLOADS = {
    "gauss_d2": GaussianSpec(10_000, 2, 6, "uniform", 10.0, 4.0, 1.0, "equal"),
    "gauss_d32": GaussianSpec(1_000_000, 32, 20, "normal", 5.0, 34.0, 1.0 / 32, "dirichlet1"),
    "mult_v100": MultinomialSpec(1_000_000, 100, 50, 0.1, 50, 200),
    "gauss_d128": GaussianSpec(10_000_000, 128, 100, "normal", 3.0, 130.0, 1.0 / 128, "dirichlet1"),
    "gauss_d64": GaussianSpec(2_000_000, 64, 200, "normal", 2.0, 66.0, 1.0 / 64, "dirichlet1"),
    "pois_d20": PoissonSpec(1_000_000, 20, 20, 1.0, 10.0),
    "news_v20k": SparseTopicSpec(11_314, 20_000, 20, 1.07, 0.02, 0.5, 150.0, 0.9, 10, 4000),
}


def _wishart(rng, dof, scale, d):
    """Wishart(dof, scale * I) as a sum of outer products (integer dof) or
    via Bartlett's factor (any dof > d - 1)."""
    A = np.zeros((d, d))
    for i in range(d):
        A[i, i] = np.sqrt(rng.chisquare(dof - i))
        A[i, :i] = rng.standard_normal(i)
    return scale * (A @ A.T)


def gaussian_params(spec, seed):
    """True mixture: weights[k], means[k, d], covariances[k, d, d]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d, k = spec.d, spec.k
    if spec.mean_kind == "uniform":
        means = rng.uniform(-spec.mean_scale, spec.mean_scale, size=(k, d))
    else:
        means = rng.normal(0.0, spec.mean_scale, size=(k, d))
    covs = np.stack([_wishart(rng, spec.wishart_dof, spec.wishart_scale, d) for _ in range(k)])
    if spec.weights == "equal":
        w = np.full(k, 1.0 / k)
    else:
        w = rng.dirichlet(np.ones(k))
    return w, means, covs


def gaussian_data(spec, seed, n=None, dtype=np.float32):
    """x[n, d] (row-major, point-major) and the true labels."""
    n = spec.n if n is None else int(n)
    w, means, covs = gaussian_params(spec, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    labels = rng.choice(spec.k, size=n, p=w)
    x = np.empty((n, spec.d), dtype=np.float64)
    for c in range(spec.k):
        idx = np.nonzero(labels == c)[0]
        L = np.linalg.cholesky(covs[c])
        x[idx] = means[c] + rng.standard_normal((idx.size, spec.d)) @ L.T
    return x.astype(dtype), labels.astype(np.int32)


def multinomial_data(spec, seed, n=None):
    """Counts x[n, V] (int32, row totals in [lo, hi]) and the true labels."""
    n = spec.n if n is None else int(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    topics = rng.dirichlet(np.full(spec.v, spec.topic_conc), size=spec.k)
    rng2 = np.random.Generator(np.random.PCG64(seed + 1))
    labels = rng2.integers(0, spec.k, size=n)
    totals = rng2.integers(spec.total_lo, spec.total_hi + 1, size=n)
    x = np.empty((n, spec.v), dtype=np.int32)
    for c in range(spec.k):
        idx = np.nonzero(labels == c)[0]
        x[idx] = rng2.multinomial(totals[idx], topics[c])
    return x, labels.astype(np.int32)


def poisson_data(spec, seed, n=None):
    """Counts x[n, d] (int32, independent Poisson per coordinate) and the true labels."""
    n = spec.n if n is None else int(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    rates = rng.gamma(spec.rate_shape, spec.rate_scale, size=(spec.k, spec.d))
    rng2 = np.random.Generator(np.random.PCG64(seed + 1))
    labels = rng2.integers(0, spec.k, size=n)
    x = rng2.poisson(rates[labels]).astype(np.int32)
    return x, labels.astype(np.int32)


def sparse_topic_data(spec, seed, n=None):
    """CSRCounts of n documents and their topics.  Tokens are drawn by
    inverting each topic's word CDF at uniform variates; repeated words of a
    document are summed."""
    n = spec.n if n is None else int(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    bg = np.arange(1, spec.v + 1, dtype=np.float64) ** -spec.zipf
    bg = bg[rng.permutation(spec.v)]
    bg /= bg.sum()
    topics = spec.mix * bg + (1 - spec.mix) * rng.dirichlet(np.full(spec.v, spec.topic_conc), size=spec.k)
    rng2 = np.random.Generator(np.random.PCG64(seed + 1))
    labels = rng2.integers(0, spec.k, size=n)
    lens = np.clip(np.rint(np.exp(rng2.normal(np.log(spec.len_median), spec.len_sigma, size=n))),
                   spec.len_lo, spec.len_hi).astype(np.int64)
    doc = np.repeat(np.arange(n, dtype=np.int64), lens)
    word = np.empty(doc.size, dtype=np.int64)
    tok_topic = labels[doc]
    for c in range(spec.k):
        sel = np.nonzero(tok_topic == c)[0]
        cdf = np.cumsum(topics[c])
        cdf /= cdf[-1]
        word[sel] = np.minimum(np.searchsorted(cdf, rng2.random(sel.size), side="right"), spec.v - 1)
    key, cnt = np.unique(doc * spec.v + word, return_counts=True)
    rows = key // spec.v
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=indptr[1:])
    return CSRCounts(indptr, (key % spec.v).astype(np.int32), cnt.astype(np.int32), (n, spec.v)), \
        labels.astype(np.int32)


def workload(name, seed, n=None):
    spec = WORKLOADS[name]
    if isinstance(spec, SparseTopicSpec):
        return sparse_topic_data(spec, seed, n)
    if isinstance(spec, GaussianSpec):
        return gaussian_data(spec, seed, n)
    if isinstance(spec, PoissonSpec):
        return poisson_data(spec, seed, n)
    return multinomial_data(spec, seed, n)
