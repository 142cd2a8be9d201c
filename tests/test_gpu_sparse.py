"""GPU parity of count rows in compressed sparse rows (multinomial and
Poisson families, contexts created with sparse=True) against the FP64
oracle, which reads the same rows densified.

Cases: the 20newsgroups-shaped stand-in (V = 20 000) at a few thousand rows
and at its full N = 11 314 (labels on sampled rows, statistics exact);
K = 1, K below one lane group, K above 64 (cluster chunks); rows with no
entry, unsorted and repeated columns; parameter draws and split/merge
decisions over the whole vocabulary; a chain that finds the topics; the
kernels' range checks on bad rows (the row is skipped, the call that
synchronises returns DPMM_E_ARG).  Comparison rules as for the dense rows:
log-likelihoods within 1e-5 M, labels only inside the oracle's margin,
statistics bit-exact."""
import numpy as np
import pytest

from oracle import dirmult, nmi, poisson, rng, sampler
from tests import parity_util as pu

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _news(n, seed=1):
    from paper_2204_08988_amd import datagen
    return datagen.workload("news_v20k", seed, n=n)


def _sparse(x):
    from paper_2204_08988_amd.sampler import SparseCounts
    return SparseCounts.from_numpy(x.indptr, x.indices, x.data, x.shape[1])


def _mult_params(K, V, seed, close):
    """Dirichlet(1) components; close=True: the clusters are small log-scale
    perturbations of one distribution, so many rows fall in the Gumbel range."""
    g = np.random.Generator(np.random.PCG64(seed))
    if close:
        base = np.log(g.dirichlet(np.ones(V)))
        lt = base + g.normal(0, 0.02, size=(K, 3, V))
    else:
        lt = np.log(g.dirichlet(np.ones(V), size=(K, 3)))
    lt -= np.log(np.exp(lt).sum(axis=2, keepdims=True))
    return sampler.Params(np.log(g.dirichlet(np.ones(K))), np.log(g.dirichlet(np.ones(2), size=K)), log_theta=lt)


def _oracle_loglik(model, x, params, rows):
    lc = np.empty((rows.size, params.K))
    ls = np.empty((rows.size, params.K, 2))
    for a in range(0, rows.size, 500):
        r = rows[a:a + 500]
        lc[a:a + 500], ls[a:a + 500] = sampler.loglik(model, x.rows(r), params)
    return lc, ls


def _oracle_stats(model, x, z, zs, K):
    """Statistics are sums over rows: the oracle's, over chunks of dense rows, added."""
    n = np.zeros((K, 2), dtype=np.int64)
    s = np.zeros((K, 2, x.shape[1]), dtype=np.int64)
    for a in range(0, x.shape[0], 1000):
        r = np.arange(a, min(a + 1000, x.shape[0]))
        st = sampler.suffstats(model, x.rows(r), z[r], zs[r], K)
        n += st.n
        s += st.s
    return pu.stats_array(sampler.Stats(n, s=s), "multinomial")


@pytest.mark.parametrize("K,n,close", [(20, 3000, False), (20, 3000, True), (1, 1500, False), (5, 2001, True),
                                       (70, 2500, True), (130, 1200, False)])
def test_sparse_loglik_labels_stats(K, n, close):
    torch = _torch()
    from paper_2204_08988_amd.sampler import Sampler
    x, _ = _news(n, seed=2)
    V = x.shape[1]
    seed = 900 + K
    params = _mult_params(K, V, seed, close)
    model = sampler.Model("multinomial", 2.0, dirmult.DirPrior(np.ones(V)), seed=seed)
    S = Sampler("multinomial", V, K + 2, 2.0, seed, beta=np.ones(V), sparse=True)
    S.set_params(params.log_pi, params.log_pisub, pu.comp_array(params))
    xs = _sparse(x)
    rows = np.arange(n)
    lc, ls = _oracle_loglik(model, x, params, rows)
    dense = x.toarray()
    Mc, Ms = pu.mult_scale(dense, params)
    ll = S.loglik(xs).cpu().numpy().astype(np.float64)
    assert pu.check_loglik(ll, lc, ls, Mc, Ms) <= 1e-5
    for t in (3, 8):
        z, zs = S.sample_labels(xs, t)
        zn, zsn = z.cpu().numpy(), zs.cpu().numpy()
        bad_c, bad_s, tie_c, tie_s = pu.label_mismatches(seed, t, zn, zsn, lc, ls, Mc, Ms)
        assert bad_c.size == 0 and bad_s.size == 0, (bad_c[:10], bad_s[:10])
        # rows of ~230 tokens over V = 20 000 put M near 2 000 nats; with up to
        # 70 clusters inside the Gumbel range a few top-2 margins fall below
        # the FP32 rounding of the sums
        assert tie_c + tie_s <= max(4, n // 400)
    if close and K > 1:
        # the case reaches the exact Gumbel-max over several clusters
        win = (lc > lc.max(axis=1, keepdims=True) - (rng.GUMBEL_MAX - rng.GUMBEL_MIN)).sum(axis=1)
        assert np.any(win >= 2)
    S.suffstats(xs, z, zs)
    assert np.array_equal(S.get_stats(), _oracle_stats(model, x, zn, zsn, K))
    S.close()


def test_sparse_rows_empty_unsorted_repeated():
    """Rows with no entry, columns out of order and a column given twice (its
    counts add): the same labels rule and the same statistics as the dense rows."""
    torch = _torch()
    from paper_2204_08988_amd.sampler import Sampler, SparseCounts
    V, K, n, seed = 300, 6, 4000, 77
    g = np.random.Generator(np.random.PCG64(seed))
    params = _mult_params(K, V, seed, True)
    dense = np.zeros((n, V), dtype=np.int32)
    indptr = [0]
    cols, vals = [], []
    for i in range(n):
        m = 0 if i % 37 == 0 else int(g.integers(1, 90))
        c = g.integers(0, V, m)
        v = g.integers(0, 4, m)  # zero counts stored too
        if m > 3:
            c[1] = c[0]  # a repeated column
        np.add.at(dense[i], c, v)
        cols.append(c)
        vals.append(v)
        indptr.append(indptr[-1] + m)
    xs = SparseCounts.from_numpy(np.array(indptr), np.concatenate(cols), np.concatenate(vals), V)
    model = sampler.Model("multinomial", 2.0, dirmult.DirPrior(np.ones(V)), seed=seed)
    S = Sampler("multinomial", V, K + 2, 2.0, seed, beta=np.ones(V), sparse=True)
    S.set_params(params.log_pi, params.log_pisub, pu.comp_array(params))
    lc, ls = sampler.loglik(model, dense, params)
    Mc, Ms = pu.mult_scale(dense, params)
    assert pu.check_loglik(S.loglik(xs).cpu().numpy().astype(np.float64), lc, ls, Mc, Ms) <= 1e-5
    z, zs = S.sample_labels(xs, 4)
    zn, zsn = z.cpu().numpy(), zs.cpu().numpy()
    bad_c, bad_s, _, _ = pu.label_mismatches(seed, 4, zn, zsn, lc, ls, Mc, Ms)
    assert bad_c.size == 0 and bad_s.size == 0
    S.suffstats(xs, z, zs)
    ref = pu.stats_array(sampler.suffstats(model, dense, zn, zsn, K), "multinomial")
    assert np.array_equal(S.get_stats(), ref)
    S.close()


def test_sparse_poisson_rows():
    torch = _torch()
    from paper_2204_08988_amd.sampler import Sampler, SparseCounts
    d, K, n, seed = 500, 8, 3000, 88
    g = np.random.Generator(np.random.PCG64(seed))
    lam = g.gamma(0.3, 0.5, size=(K, 1, d)) * np.exp(g.normal(0, 0.05, size=(K, 3, d)))
    params = sampler.Params(np.log(g.dirichlet(np.ones(K))), np.log(g.dirichlet(np.ones(2), size=K)),
                            log_theta=np.log(lam))
    lab = g.integers(0, K, n)
    dense = g.poisson(lam[lab, 0]).astype(np.int32)
    r, c = np.nonzero(dense)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=indptr[1:])
    xs = SparseCounts.from_numpy(indptr, c, dense[r, c], d)
    prior = poisson.GammaPrior(np.full(d, 0.5), np.full(d, 0.3))
    model = sampler.Model("poisson", 2.0, prior, seed=seed)
    S = Sampler("poisson", d, K + 2, 2.0, seed, gamma_shape=prior.shape, gamma_rate=prior.rate, sparse=True)
    S.set_params(params.log_pi, params.log_pisub, pu.comp_array(params))
    lc, ls = sampler.loglik(model, dense, params)
    Mc = np.abs(params.log_pi)[None, :] + dense @ np.abs(params.log_theta[:, 0]).T + lam[:, 0].sum(1)[None, :]
    Ms = np.stack([np.abs(params.log_pisub[:, h])[None, :] + dense @ np.abs(params.log_theta[:, 1 + h]).T
                   + np.exp(params.log_theta[:, 1 + h]).sum(1)[None, :] for h in range(2)], axis=2)
    assert pu.check_loglik(S.loglik(xs).cpu().numpy().astype(np.float64), lc, ls, Mc, Ms) <= 1e-5
    z, zs = S.sample_labels(xs, 5)
    zn, zsn = z.cpu().numpy(), zs.cpu().numpy()
    bad_c, bad_s, _, _ = pu.label_mismatches(seed, 5, zn, zsn, lc, ls, Mc, Ms)
    assert bad_c.size == 0 and bad_s.size == 0
    S.suffstats(xs, z, zs)
    ref = pu.stats_array(sampler.suffstats(model, dense, zn, zsn, K), "poisson")
    assert np.array_equal(S.get_stats(), ref)
    S.close()


def test_sparse_params_and_split_merge_full_vocabulary():
    """Dirichlet draws over V = 20 000 words and the split/merge decisions
    from the Dirichlet-multinomial marginals of the same statistics."""
    torch = _torch()
    from paper_2204_08988_amd.sampler import Sampler
    x, lab = _news(3000, seed=4)
    V, seed = x.shape[1], 31
    g = np.random.Generator(np.random.PCG64(6))
    K = 5
    z = (lab % K).astype(np.int64)
    flip = g.random(z.size) < 0.3
    z[flip] = g.integers(0, K, int(flip.sum()))
    zs = g.integers(0, 2, z.size)
    beta = np.full(V, 0.1)
    model = sampler.Model("multinomial", 2.0, dirmult.DirPrior(beta), seed=seed, burn_out=0)
    S = Sampler("multinomial", V, 32, 2.0, seed, beta=beta, burn_out=0, sparse=True)
    st_arr = _oracle_stats(model, x, z, zs, K)
    st = sampler.Stats(st_arr[..., 0], s=st_arr[..., 1:])
    S.set_stats(st_arr)
    S.sample_params(6)
    lp, lps, lt = S.get_params()
    ref = sampler.sample_params(model, st, 6)
    assert np.allclose(lp, ref.log_pi, rtol=1e-10, atol=1e-12)
    assert np.allclose(lt, ref.log_theta, rtol=1e-10, atol=1e-10)
    xs = _sparse(x)
    zt = torch.from_numpy(z.astype(np.int32)).cuda()
    zst = torch.from_numpy(zs.astype(np.uint8)).cuda()
    S.set_state(K, [0] * K)
    S.suffstats(xs, zt, zst)
    gi = S.split_merge(xs, 6, zt, zst)
    state = sampler.State(K, z.astype(np.int64), zs.astype(np.int64), np.zeros(K, dtype=np.int64))
    refs, info = sampler.split_merge(model, state, st, 6)
    assert gi["K"] == refs.K and gi["merges"] == info.merges and gi["splits"] == info.splits
    assert np.array_equal(zt.cpu().numpy(), refs.z) and np.array_equal(zst.cpu().numpy(), refs.zsub)
    ref_st = _oracle_stats(model, x, refs.z, refs.zsub, refs.K)
    assert np.isclose(gi["logpost"], sampler.log_posterior(model, sampler.Stats(ref_st[..., 0], s=ref_st[..., 1:])),
                      rtol=1e-10)
    S.close()


def test_sparse_full_size_sampled_rows():
    """The configuration's N = 11 314: labels of 600 sampled rows against the
    oracle, statistics of every row exact, in the launch the chain uses."""
    torch = _torch()
    from paper_2204_08988_amd.sampler import Sampler
    x, _ = _news(None, seed=1)
    n, V = x.shape
    K, seed = 20, 5
    params = _mult_params(K, V, seed, True)
    model = sampler.Model("multinomial", 2.0, dirmult.DirPrior(np.ones(V)), seed=seed)
    S = Sampler("multinomial", V, 64, 2.0, seed, beta=np.ones(V), sparse=True)
    S.set_params(params.log_pi, params.log_pisub, pu.comp_array(params))
    xs = _sparse(x)
    z, zs = S.sample_labels(xs, 9)
    zn, zsn = z.cpu().numpy(), zs.cpu().numpy()
    rows = np.sort(np.random.Generator(np.random.PCG64(1)).choice(n, 600, replace=False))
    lc, ls = _oracle_loglik(model, x, params, rows)
    dense = x.rows(rows)
    Mc, Ms = pu.mult_scale(dense, params)
    bad_c, bad_s, tie_c, tie_s = pu.label_mismatches(seed, 9, zn[rows], zsn[rows], lc, ls, Mc, Ms, points=rows)
    assert bad_c.size == 0 and bad_s.size == 0
    S.suffstats(xs, z, zs)
    assert np.array_equal(S.get_stats(), _oracle_stats(model, x, zn, zsn, K))
    S.close()


def test_sparse_chain_finds_topics():
    torch = _torch()
    from paper_2204_08988_amd.sampler import Sampler
    x, lab = _news(None, seed=1)
    V = x.shape[1]
    S = Sampler("multinomial", V, 64, 10.0, 3, beta=np.full(V, 0.1), burn_out=5, sparse=True)
    xs = _sparse(x)
    z, zs = S.init_labels(x.shape[0])
    for t in range(1, 151):
        info = S.step(xs, t, z, zs)
    assert 15 <= info["K"] <= 30, info
    assert nmi.nmi(lab, z.cpu().numpy()) > 0.9
    S.close()


def test_sparse_bad_rows_raise():
    """A column past V, a negative count, a row range past nnz: the kernels
    skip the entry or row and the next synchronising call reports it."""
    torch = _torch()
    from paper_2204_08988_amd._lib import DpmmError
    from paper_2204_08988_amd.sampler import Sampler, SparseCounts
    V, K = 40, 3
    params = _mult_params(K, V, 3, False)
    good = (np.array([0, 2, 4, 6]), np.array([1, 5, 2, 3, 7, 9]), np.array([1, 2, 3, 1, 1, 2]))
    bad_cases = [(good[0], np.array([1, 5, 2, 40, 7, 9]), good[2]),      # column = V
                 (good[0], good[1], np.array([1, 2, -3, 1, 1, 2])),       # negative count
                 (np.array([0, 2, 9, 6]), good[1], good[2])]             # row range past nnz
    for ip, c, v in [good] + bad_cases:
        S = Sampler("multinomial", V, K + 2, 2.0, 3, beta=np.ones(V), sparse=True, burn_out=0)
        S.set_params(params.log_pi, params.log_pisub, pu.comp_array(params))
        xs = SparseCounts.from_numpy(ip, c, v, V)
        z, zs = S.sample_labels(xs, 1)
        if ip is good[0] and c is good[1] and v is good[2]:
            S.get_params()
            S.suffstats(xs, z, zs)
            S.split_merge(xs, 1, z, zs)
            S.close()
            continue
        with pytest.raises(DpmmError) as e:  # the label kernel's flag, read back by get_params
            S.get_params()
        assert e.value.status == -1, e.value
        S.get_params()  # the flag was cleared
        z.zero_()
        S.set_state(K, [0] * K)
        S.suffstats(xs, z, zs)
        with pytest.raises(DpmmError) as e:  # the statistics kernel's flag, read back by split_merge
            S.split_merge(xs, 1, z, zs)
        assert e.value.status == -1, e.value
        S.close()
