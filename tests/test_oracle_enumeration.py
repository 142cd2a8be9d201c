"""Whole-chain checks on N = 5 points against the exact partition posterior.

Neal's Algorithm 3 is provably invariant for this posterior, so its histogram
pins the enumeration harness (exact posterior, canonical labels, total
variation).  The sub-cluster sampler with the printed split/merge ratios is run
through the same harness; its distance to the exact posterior is a reported
property of the printed algorithm (long runs: TV about 0.31 with the merge
ratio of eq. sample_merges and 0.44 with H_merge = 1/H_split, against 0.017
for Neal's sampler at the same length), not a tolerance the oracle is tuned to.
"""
from collections import Counter

import numpy as np
import pytest

from oracle import niw, partitions, sampler

X = np.array([[-1.2], [-0.9], [0.1], [1.5], [1.8]])
PRIOR = niw.NIWPrior(0.5, [0.0], 2.0, [[0.5]])
ALPHA = 1.0


def _lm(rows):
    xs = X[rows]
    return niw.log_marginal(PRIOR, len(rows), xs.sum(0), xs.T @ xs)


def test_partition_count_and_exact_posterior_normalised():
    assert len(partitions.set_partitions(5)) == 52
    assert len(partitions.set_partitions(8)) == 4140
    ex = partitions.exact_posterior(X, ALPHA, _lm)
    assert np.isclose(sum(ex.values()), 1.0)


def test_neal_algorithm3_matches_exact_posterior():
    ex = partitions.exact_posterior(X, ALPHA, _lm)
    h = Counter(partitions.neal_algorithm3(X, ALPHA, _lm, 4000, np.random.default_rng(0)))
    assert partitions.total_variation(h, ex) < 0.05


@pytest.mark.slow
@pytest.mark.parametrize("form", ["paper", "inverse_split"])
def test_subcluster_sampler_partition_histogram(form):
    ex = partitions.exact_posterior(X, ALPHA, _lm)
    model = sampler.Model("gaussian", ALPHA, PRIOR, seed=3, burn_out=0, merge_form=form)
    st = sampler.initial_state(model, 5)
    h = Counter()
    for t in range(1, 2501):
        st, info = sampler.step(model, X, st, t)
        h[partitions.canonical(st.z)] += 1
    tv = partitions.total_variation(h, ex)
    print(f"merge_form={form}: TV to exact posterior = {tv:.3f}")
    # the chain moves across the whole space: every partition holding more
    # than 3% of the exact mass is visited
    assert all(h[p] > 0 for p, pr in ex.items() if pr > 0.03)
    assert tv < 0.7
