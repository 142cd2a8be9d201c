"""Pins of the oracle's log posterior, its compaction and the learned
proposal's training set, each against a quantity computed another way.

* log_posterior(z) = K log alpha + lgamma(alpha) - lgamma(alpha + N)
  + sum_k [lgamma(N_k) + log f(C_k)] is checked against the Chinese-restaurant
  seating product (points arrive one at a time: an occupied table c with
  probability n_c / (alpha + i), a new one with alpha / (alpha + i)) times the
  marginal likelihoods, for every partition of N = 5 points, NIW,
  Dirichlet-multinomial and Gamma-Poisson; and its differences between partitions against the
  log-ratios of the enumerated exact posterior (Sec. 2.2 model, pi and the
  component parameters integrated out).
* compact() on a deletion in the middle of the cluster range: the surviving
  clusters shift down by the number of deleted clusters below them.
* training_set() on a hand-built state whose eligible cluster, row order and
  principal-axis targets are known without the oracle.
"""
import numpy as np
import pytest

from oracle import dirmult, learned, niw, partitions, poisson, sampler


def _crp_log_prior(z, alpha):
    """log p(z) under the Chinese restaurant process, seat by seat."""
    counts = {}
    lp = 0.0
    for i, c in enumerate(z):
        c = int(c)
        if c in counts:
            lp += np.log(counts[c]) - np.log(alpha + i)
            counts[c] += 1
        else:
            lp += np.log(alpha) - np.log(alpha + i)
            counts[c] = 1
    return lp


GX = np.array([[-1.2, 0.4], [-0.9, 0.1], [0.1, -0.3], [1.5, 0.9], [1.8, 1.1]])
GPRIOR = niw.NIWPrior(0.7, [0.1, -0.2], 4.0, [[0.8, 0.1], [0.1, 0.5]])
MX = np.array([[3, 0, 1], [2, 1, 0], [0, 4, 1], [0, 3, 2], [1, 1, 5]])
MPRIOR = dirmult.DirPrior([0.5, 1.0, 2.0])


PPRIOR = poisson.GammaPrior([1.5, 0.5, 2.0], [1.0, 0.3, 2.0])


def _family(name):
    if name == "poisson":
        model = sampler.Model("poisson", 1.7, PPRIOR, seed=1, burn_out=0)

        def lm(rows):
            return poisson.log_marginal(PPRIOR, len(rows), MX[rows].sum(0))
        return model, MX, lm
    if name == "gaussian":
        model = sampler.Model("gaussian", 1.7, GPRIOR, seed=1, burn_out=0)

        def lm(rows):
            xs = GX[rows]
            return niw.log_marginal(GPRIOR, len(rows), xs.sum(0), xs.T @ xs)
        return model, GX, lm
    model = sampler.Model("multinomial", 1.7, MPRIOR, seed=1, burn_out=0)

    def lm(rows):
        return dirmult.log_marginal(MPRIOR, MX[rows].sum(0))
    return model, MX, lm


@pytest.mark.parametrize("family", ["gaussian", "multinomial", "poisson"])
def test_log_posterior_is_crp_seating_times_marginals(family):
    model, x, lm = _family(family)
    zsub = np.array([0, 1, 0, 1, 1])
    for part in partitions.set_partitions(5):
        z = np.asarray(part)
        K = int(z.max()) + 1
        lp = sampler.log_posterior(model, sampler.suffstats(model, x, z, zsub, K))
        ref = _crp_log_prior(z, model.alpha) + sum(lm(list(np.nonzero(z == k)[0])) for k in range(K))
        assert abs(lp - ref) <= 1e-11 * (1 + abs(ref)), part


@pytest.mark.parametrize("family", ["gaussian", "multinomial", "poisson"])
def test_log_posterior_differences_match_enumerated_posterior(family):
    model, x, lm = _family(family)
    ex = partitions.exact_posterior(x, model.alpha, lm)
    parts = list(ex)
    zsub = np.zeros(5, dtype=np.int64)
    lp = {}
    for p in parts:
        z = np.asarray(p)
        lp[p] = sampler.log_posterior(model, sampler.suffstats(model, x, z, zsub, int(z.max()) + 1))
    ref = parts[0]
    for p in parts[1:]:
        assert np.isclose(lp[p] - lp[ref], np.log(ex[p]) - np.log(ex[ref]), rtol=1e-10, atol=1e-10), p


def test_log_posterior_invariant_under_cluster_order_and_sublabels():
    model, x, _ = _family("gaussian")
    z = np.array([0, 0, 1, 2, 2])
    a = sampler.log_posterior(model, sampler.suffstats(model, x, z, np.array([0, 1, 0, 0, 1]), 3))
    perm = np.array([2, 0, 1])  # rename clusters 0 -> 2, 1 -> 0, 2 -> 1
    b = sampler.log_posterior(model, sampler.suffstats(model, x, perm[z], np.array([1, 1, 1, 0, 0]), 3))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_compact_shifts_clusters_above_a_deleted_one():
    z = np.array([0, 2, 3, 2, 0, 3, 3])
    zsub = np.array([1, 0, 1, 1, 0, 0, 1])
    st = sampler.State(4, z, zsub, np.array([7, 8, 9, 10]))
    out = sampler.compact(st, [True, False, True, True])
    assert out.K == 3
    assert np.array_equal(out.z, [0, 1, 2, 1, 0, 2, 2])
    assert np.array_equal(out.zsub, zsub)
    assert np.array_equal(out.age, [7, 9, 10])
    out2 = sampler.compact(st, [False, False, True, True])
    assert np.array_equal(out2.z[z >= 2], [0, 1, 0, 1, 1])


def test_drop_empty_deletes_a_middle_cluster():
    model, x, _ = _family("gaussian")
    z = np.array([0, 0, 3, 3, 2])  # cluster 1 is empty
    st = sampler.State(4, z, np.array([0, 1, 0, 1, 0]), np.array([5, 6, 7, 8]))
    out, stats = sampler.drop_empty(model, x, st)
    assert out.K == 3
    assert np.array_equal(out.z, [0, 0, 2, 2, 1])
    assert np.array_equal(out.age, [5, 7, 8])
    assert np.array_equal(stats.n, [[1, 1], [1, 0], [1, 1]])


def _training_case(l_on_positive):
    """Cluster 0: six points on the line x2 = 0 (first principal axis e1, whose
    sign convention makes +e1 positive); cluster 1 is too young; cluster 2 has
    only left sub-labels; cluster 3 is eligible but one point only on each
    side is missing (it has a single sub-cluster).  The points of cluster 0
    are interleaved with the others so that the row order is tested."""
    x = np.array([[-3.0, 0.0], [5.0, 5.0], [2.0, 0.0], [9.0, 1.0], [-1.0, 0.0],
                  [3.0, 0.0], [9.5, 1.0], [5.5, 5.0], [-2.0, 0.0], [1.0, 0.0], [4.0, 4.0]])
    z = np.array([0, 1, 0, 2, 0, 0, 2, 1, 0, 0, 3])
    pos = x[:, 0] > 0
    zsub = np.where(pos, 0 if l_on_positive else 1, 1 if l_on_positive else 0)
    zsub[[3, 6]] = 0
    age = np.array([4, 1, 4, 4])
    return x, sampler.State(4, z, zsub, age)


@pytest.mark.parametrize("l_on_positive", [True, False])
def test_training_set_rows_and_canonical_targets(l_on_positive):
    x, st = _training_case(l_on_positive)
    prior = niw.NIWPrior(1.0, np.zeros(2), 5.0, np.eye(2))
    model = sampler.Model("gaussian", 1.0, prior, seed=0, burn_out=3)
    X, Y = learned.training_set(model, x, st, 1)
    rows = np.array([0, 2, 4, 5, 8, 9])  # cluster 0's points in index order
    assert X.shape == (rows.size, 2) and Y.shape == (rows.size,)
    # the first feature is the coordinate on the principal axis +e1, centred on
    # the set mean (0) and scaled by the root of the largest eigenvalue
    xs = x[rows, 0]
    lam = np.mean(xs ** 2) - np.mean(xs) ** 2
    lam += 1e-9 * (1 + lam / 2)
    assert np.allclose(X[:, 0], (xs - xs.mean()) / np.sqrt(lam), rtol=1e-9)
    # the second is the eigenvalue share: the other axis has (regularised) zero variance
    assert np.allclose(X[:, 1], lam / (lam + 1e-9 * (1 + lam / 2)), rtol=1e-9)
    # target 1 on the side with the larger mean principal coordinate, whichever
    # sub-label it carried
    assert np.array_equal(Y, (xs > 0).astype(np.float64))


def test_training_set_empty_when_nothing_qualifies():
    x, st = _training_case(True)
    prior = niw.NIWPrior(1.0, np.zeros(2), 5.0, np.eye(2))
    model = sampler.Model("gaussian", 1.0, prior, seed=0, burn_out=5)
    X, Y = learned.training_set(model, x, st, 1)
    assert X.shape == (0, 2) and Y.shape == (0,)
