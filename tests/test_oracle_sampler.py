"""Pins for the oracle sampler's steps: label and sub-label draws against
scipy log-densities and softmax/sigmoid frequencies, statistics invariants,
the worked N = 2 split/merge ratios, merge-then-split restoring statistics,
weights moments and NMI against scikit-learn."""
import numpy as np
import pytest
from scipy import stats
from scipy.special import expit, gammaln, softmax

from oracle import dirmult, niw, nmi, rng, sampler


def _gauss_model(d=2, seed=5, burn_out=0, alpha=3.0):
    return sampler.Model("gaussian", alpha, niw.NIWPrior(1.0, np.zeros(d), d + 3, np.eye(d)),
                         seed=seed, burn_out=burn_out)


def _random_params(K, d, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    mu = g.normal(0, 3, size=(K, 3, d))
    a = g.standard_normal((K, 3, d, d))
    sigma = a @ np.swapaxes(a, -1, -2) + 0.5 * np.eye(d)
    lp = np.log(g.dirichlet(np.ones(K)))
    lps = np.log(g.dirichlet(np.ones(2), size=K))
    return sampler.Params(lp, lps, mu=mu, sigma=sigma)


def test_loglik_against_scipy_and_label_argmax():
    model = _gauss_model(d=3)
    K, N = 5, 64
    p = _random_params(K, 3, 1)
    g = np.random.Generator(np.random.PCG64(2))
    x = g.normal(0, 4, size=(N, 3))
    lc, ls = sampler.loglik(model, x, p)
    for k in range(K):
        ref = p.log_pi[k] + stats.multivariate_normal(p.mu[k, 0], p.sigma[k, 0]).logpdf(x)
        assert np.allclose(lc[:, k], ref, rtol=1e-12, atol=1e-9)
        for h in range(2):
            ref = p.log_pisub[k, h] + stats.multivariate_normal(p.mu[k, 1 + h], p.sigma[k, 1 + h]).logpdf(x)
            assert np.allclose(ls[:, k, h], ref, rtol=1e-12, atol=1e-9)
    z, zs = sampler.sample_labels(model, x, p, t=4)
    for i in range(N):
        w = [rng.block(model.seed, 4, i, rng.TAG_GUMBEL, k // 4)[k % 4] for k in range(K)]
        pert = [lc[i, k] + float(rng.gumbel(np.uint32(w[k]))) for k in range(K)]
        assert z[i] == int(np.argmax(pert))
        # the logistic's word: the last Gumbel block's unused word when K % 4 != 0
        wl = rng.block(model.seed, 4, i, rng.TAG_GUMBEL, K // 4)[K % 4] if K % 4 else \
            rng.block(model.seed, 4, i, rng.TAG_LOGISTIC, 0)[0]
        L = float(rng.logistic(np.uint32(wl)))
        assert zs[i] == (0 if ls[i, z[i], 0] - ls[i, z[i], 1] + L > 0 else 1)


@pytest.mark.parametrize("K", [4, 5, 6, 7, 8])
def test_sub_label_independent_of_cluster_draw(K):
    """The sub-label's logistic shares the last Gumbel block when K % 4 != 0:
    the joint frequencies of (z, sub-label) must still be the product of the
    softmax and the sigmoid.  A logistic word that coincided with a cluster's
    Gumbel word (an index off by one) would tie the two draws together."""
    N = 150_000
    logits = np.linspace(0.8, -0.6, K)
    lc = np.tile(logits, (N, 1))
    ls = np.zeros((N, K, 2))
    ls[:, :, 0] = 0.4
    z, zs = sampler.draw_labels(23, 5, lc, ls)
    table = np.zeros((K, 2))
    np.add.at(table, (z, zs), 1)
    expect = np.outer(softmax(logits), [expit(0.4), 1.0 - expit(0.4)]) * N
    assert stats.chisquare(table.ravel(), expect.ravel()).pvalue > 1e-3


def test_label_frequencies_follow_softmax_and_sigmoid():
    N, K = 120_000, 5
    logits = np.array([0.5, -0.3, 1.7, 0.0, -2.0])
    lc = np.tile(logits, (N, 1))
    ls = np.zeros((N, K, 2))
    ls[:, :, 0] = 0.8
    z, zs = sampler.draw_labels(17, 9, lc, ls)
    counts = np.bincount(z, minlength=K)
    assert stats.chisquare(counts, softmax(logits) * N).pvalue > 1e-3
    p_l = expit(0.8)
    n_l = int(np.sum(zs == 0))
    assert abs(n_l - p_l * N) < 5 * np.sqrt(N * p_l * (1 - p_l))


def test_suffstats_invariants():
    model = _gauss_model(d=3)
    g = np.random.Generator(np.random.PCG64(3))
    x = g.standard_normal((500, 3))
    z = g.integers(0, 4, 500)
    zs = g.integers(0, 2, 500)
    st = sampler.suffstats(model, x, z, zs, 4)
    assert st.n.sum() == 500
    for k in range(4):
        n, s, S = st.cluster(k)
        m = z == k
        assert n == m.sum()
        assert np.allclose(s, x[m].sum(0)) and np.allclose(S, x[m].T @ x[m])
        assert st.n[k, 0] == np.sum(m & (zs == 0))


def test_split_merge_ratios_worked_case_two_points():
    model = _gauss_model(d=2, alpha=2.5)
    x = np.array([[0.3, -1.0], [2.0, 0.4]])
    st = sampler.suffstats(model, x, np.array([0, 0]), np.array([0, 1]), 1)
    f1 = niw.log_marginal(model.prior, 1, x[0], np.outer(x[0], x[0]))
    f2 = niw.log_marginal(model.prior, 1, x[1], np.outer(x[1], x[1]))
    f12 = niw.log_marginal(model.prior, 2, x.sum(0), x.T @ x)
    a = model.alpha
    # Gamma(1) = Gamma(2) = 1: H_split = alpha f1 f2 / f12
    assert np.isclose(sampler.split_log_h(model, st, 0), np.log(a) + f1 + f2 - f12, rtol=1e-13)
    st2 = sampler.suffstats(model, x, np.array([0, 1]), np.array([0, 0]), 2)
    # eq. sample_merges at N1 = N2 = 1: (f12 / (alpha f1 f2)) * alpha / (4 (alpha + 1))
    expect = f12 - np.log(a) - f1 - f2 + np.log(a / (4 * (a + 1)))
    assert np.isclose(sampler.merge_log_h(model, st2, 0, 1), expect, rtol=1e-13)
    model.merge_form = "inverse_split"
    assert np.isclose(sampler.merge_log_h(model, st2, 0, 1), f12 - np.log(a) - f1 - f2, rtol=1e-13)


def test_merge_then_split_restores_statistics(monkeypatch):
    model = _gauss_model(d=2)
    g = np.random.Generator(np.random.PCG64(4))
    # dyadic data: every partial sum is exact, so equality is bit-for-bit
    x = g.integers(-40, 40, size=(300, 2)) / 8.0
    z = g.integers(0, 3, 300)
    zs = g.integers(0, 2, 300)
    state = sampler.State(3, z, zs, np.zeros(3, dtype=np.int64))
    st = sampler.suffstats(model, x, z, zs, 3)
    monkeypatch.setattr(sampler, "split_log_h", lambda *a: -np.inf)
    monkeypatch.setattr(sampler, "merge_log_h", lambda m, s, k1, k2: np.inf if (k1, k2) == (0, 2) else -np.inf)
    merged, info = sampler.split_merge(model, state, st, 1)
    assert info.merges == 1 and merged.K == 2
    stm = sampler.suffstats(model, x, merged.z, merged.zsub, 2)
    # merged cluster's sub-clusters are exactly the two original clusters
    for h, k in ((0, 0), (1, 2)):
        n, s, S = st.cluster(k)
        assert stm.n[0, h] == n and np.array_equal(stm.s[0, h], s) and np.array_equal(stm.S[0, h], S)
    monkeypatch.setattr(sampler, "split_log_h", lambda m, s, k: np.inf if k == 0 else -np.inf)
    monkeypatch.setattr(sampler, "merge_log_h", lambda *a: -np.inf)
    split, info = sampler.split_merge(model, merged, stm, 2)
    assert info.splits == 1 and split.K == 3
    sts = sampler.suffstats(model, x, split.z, split.zsub, 3)
    # cluster 0 keeps the old cluster 0, the appended slot holds the old cluster 2
    for new, old in ((0, 0), (1, 1), (2, 2)):
        a_, b_ = sts.cluster(new), st.cluster(old)
        assert a_[0] == b_[0] and np.array_equal(a_[1], b_[1]) and np.array_equal(a_[2], b_[2])


def test_weights_are_dirichlet():
    model = _gauss_model()
    st = sampler.Stats(n=np.array([[30, 10], [5, 5], [100, 0]]), s=np.zeros((3, 2, 2)), S=np.zeros((3, 2, 2, 2)))
    lps = []
    subs = []
    for t in range(1, 3001):
        lp, lsub = sampler.sample_weights(model, st, t)
        lps.append(np.exp(lp))
        subs.append(np.exp(lsub))
    lps = np.array(lps); subs = np.array(subs)
    conc = np.array([40, 10, 100, model.alpha])
    assert np.allclose(lps.mean(0), conc[:3] / conc.sum(), atol=0.005)
    a = st.n + model.alpha / 2
    assert np.allclose(subs[:, :, 0].mean(0), a[:, 0] / a.sum(1), atol=0.01)
    assert np.allclose(subs.sum(2), 1.0)


def test_multinomial_family_loglik_and_step():
    g = np.random.Generator(np.random.PCG64(8))
    x = g.integers(0, 5, size=(200, 6))
    model = sampler.Model("multinomial", 2.0, dirmult.DirPrior(np.ones(6)), seed=3, burn_out=0)
    st = sampler.initial_state(model, 200)
    for t in range(1, 6):
        st, info = sampler.step(model, x, st, t)
        stats_ = sampler.suffstats(model, x, st.z, st.zsub, st.K)
        assert stats_.n.sum() == 200 and np.all(stats_.n.sum(1) > 0)
        assert stats_.s.sum() == x.sum()


def test_nmi_matches_sklearn():
    skm = pytest.importorskip("sklearn.metrics")
    g = np.random.Generator(np.random.PCG64(1))
    a = g.integers(0, 5, 1000)
    b = np.where(g.random(1000) < 0.7, a, g.integers(0, 7, 1000))
    assert np.isclose(nmi.nmi(a, b), skm.normalized_mutual_info_score(a, b), rtol=1e-12)


def test_chain_finds_clusters_on_separated_data():
    from paper_2204_08988_amd import datagen
    x, lab = datagen.workload("gauss_d2", 1, n=1500)
    x = x.astype(np.float64)
    model = sampler.Model("gaussian", 10.0, niw.NIWPrior(1.0, x.mean(0), 5.0, np.eye(2)), seed=1, burn_out=5)
    st = sampler.initial_state(model, x.shape[0])
    for t in range(1, 121):
        st, info = sampler.step(model, x, st, t)
    assert 4 <= info.K <= 9
    assert nmi.nmi(lab, st.z) > 0.75
