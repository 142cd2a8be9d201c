"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs and the same (seed, t)."""
import numpy as np
import pytest

from oracle import dirmult, niw, nmi, sampler
from tests import parity_util as pu

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _gauss_sampler(d, k_max, seed, **kw):
    from paper_2204_08988_amd.sampler import Sampler
    return Sampler("gaussian", d, k_max, kw.pop("alpha", 2.0), seed, kappa=1.0, nu=d + 3.0,
                   m=np.zeros(d), psi=np.eye(d), **kw)


# the last two put more than 2^21 points through the d <= 4 label kernel, whose
# 8192 x 256 lanes then each take two or more points of the grid-stride loop
GAUSS_CASES = [(1, 1, 777), (2, 6, 10000), (3, 4, 5000), (8, 12, 4099), (5, 7, 2049),
               (16, 9, 2000), (32, 20, 3001), (2, 70, 1500), (12, 3, 1300), (8, 300, 5000),
               (64, 5, 700), (33, 4, 900), (128, 3, 300), (128, 6, 140000), (32, 20, 200003),
               (2, 6, 2_500_001), (3, 5, 2_300_000)]


def _check_stats(got, x, z, zs, K, d):
    model = sampler.Model("gaussian", 1.0, niw.NIWPrior(1.0, np.zeros(d), d + 3, np.eye(d)), seed=5)
    ref = pu.stats_array(sampler.suffstats(model, x, z, zs, K), "gaussian")
    assert np.array_equal(got[..., 0], ref[..., 0])
    xa = np.abs(x.astype(np.float64))
    seg = 2 * z.astype(np.int64) + zs
    for s_ in range(2 * K):
        xs = xa[seg == s_]
        k, h = divmod(s_, 2)
        assert np.all(np.abs(got[k, h, 1:1 + d] - ref[k, h, 1:1 + d]) <= 1e-6 * xs.sum(0) + 1e-300)
        assert np.all(np.abs(got[k, h, 1 + d:] - ref[k, h, 1 + d:]).reshape(d, d) <= 1e-6 * (xs.T @ xs) + 1e-300)


@pytest.mark.parametrize("d,K,n", GAUSS_CASES)
def test_gauss_loglik_and_labels(d, K, n):
    torch = _torch()
    seed = 1000 + 7 * d + K
    params = pu.random_gauss_params(K, d, seed)
    x = pu.gauss_points(params, n, seed + 1)
    S = _gauss_sampler(d, K + 3, seed)
    S.set_params(params.log_pi, params.log_pisub, pu.comp_array(params))
    xt = torch.from_numpy(x).cuda()
    model = sampler.Model("gaussian", 2.0, niw.NIWPrior(1.0, np.zeros(d), d + 3, np.eye(d)), seed=seed)
    lc, ls = sampler.loglik(model, x.astype(np.float64), params)
    Mc, Ms = pu.gauss_scale(x, params)
    ll = S.loglik(xt).cpu().numpy().astype(np.float64)
    assert pu.check_loglik(ll, lc, ls, Mc, Ms) <= 1e-5
    for t in (1, 9):
        z, zs = S.sample_labels(xt, t)
        torch.cuda.synchronize()
        bad_c, bad_s, tie_c, tie_s = pu.label_mismatches(seed, t, z.cpu().numpy(), zs.cpu().numpy(), lc, ls, Mc, Ms)
        assert bad_c.size == 0, (bad_c[:10], tie_c)
        assert bad_s.size == 0, (bad_s[:10], tie_s)
        assert tie_c <= max(2, n // 1000) and tie_s <= max(2, n // 1000)
        if d < 5:
            S.suffstats(xt, z, zs)
        # d >= 5: the statistics are a by-product of the sorted sub-label pass
        _check_stats(S.get_stats(), x, z.cpu().numpy(), zs.cpu().numpy(), K, d)
    S.close()


@pytest.mark.parametrize("d,K,n", [(1, 2, 1000), (2, 6, 10000), (3, 5, 3001), (5, 4, 2500),
                                   (32, 20, 9000), (20, 3, 70000), (2, 300, 5000), (0, 1, 0),
                                   (8, 500, 3000), (64, 7, 5000), (128, 2, 700), (32, 1, 1)])
def test_gauss_suffstats(d, K, n):
    torch = _torch()
    d = max(d, 1)
    g = np.random.Generator(np.random.PCG64(d * 31 + K))
    x = (g.standard_normal((n, d)) * 3 + 1).astype(np.float32)
    z = g.integers(0, K, n).astype(np.int32)
    zs = g.integers(0, 2, n).astype(np.uint8)
    S = _gauss_sampler(d, K, 5)
    S.set_state(K)
    S.suffstats(torch.from_numpy(x).cuda(), torch.from_numpy(z).cuda(), torch.from_numpy(zs).cuda())
    _check_stats(S.get_stats(), x, z, zs, K, d)
    S.close()


@pytest.mark.parametrize("d,K", [(1, 1), (2, 6), (3, 4), (8, 5), (32, 3), (64, 2), (100, 2), (128, 3)])
def test_gauss_sample_params(d, K):
    torch = _torch()
    seed = 77 + d
    g = np.random.Generator(np.random.PCG64(seed))
    n = 400 * K
    x = (g.standard_normal((n, d)) * 2 + g.integers(-5, 5, size=(n, 1))).astype(np.float32)
    z = g.integers(0, K, n)
    zs = g.integers(0, 2, n)
    zs[z == 0] = 0  # an empty sub-cluster: its parameters come from the prior
    psi = np.eye(d) * 0.7 + 0.1
    model = sampler.Model("gaussian", 3.0, niw.NIWPrior(1.3, np.full(d, 0.2), d + 2.5, psi), seed=seed)
    st = sampler.suffstats(model, x, z, zs, K)
    from paper_2204_08988_amd.sampler import Sampler
    S = Sampler("gaussian", d, K, 3.0, seed, kappa=1.3, nu=d + 2.5, m=np.full(d, 0.2), psi=psi)
    S.set_stats(pu.stats_array(st, "gaussian"))
    for t in (1, 4):
        S.sample_params(t)
        lp, lps, comp = S.get_params()
        ref = sampler.sample_params(model, st, t)
        assert np.allclose(lp, ref.log_pi, rtol=1e-10, atol=1e-12)
        assert np.allclose(lps, ref.log_pisub, rtol=1e-10, atol=1e-12)
        assert np.allclose(comp[:, :, :d], ref.mu, rtol=1e-9, atol=1e-9)
        sig = comp[:, :, d:].reshape(K, 3, d, d)
        scale = np.sqrt(np.einsum("kcii,kcjj->kcij", ref.sigma, ref.sigma))
        assert np.all(np.abs(sig - ref.sigma) <= 1e-9 * scale)
        # the float32 scoring records written by the draw (whitener, constant, mean)
        lc, ls = sampler.loglik(model, x.astype(np.float64), ref)
        Mc, Ms = pu.gauss_scale(x, ref)
        ll = S.loglik(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
        assert pu.check_loglik(ll, lc, ls, Mc, Ms) <= 1e-5
    S.close()


def _split_merge_case():
    """Three separated true groups; cluster 0 holds two of them with sub-labels
    along the true split, clusters 1 and 2 are halves of the third, cluster 3
    is empty: expect one split, one merge, one removal."""
    g = np.random.Generator(np.random.PCG64(3))
    n = 900
    centres = np.array([[-20.0, 0.0], [20.0, 0.0], [0.0, 25.0]])
    grp = np.repeat(np.arange(3), n // 3)
    x = (centres[grp] + g.standard_normal((n, 2))).astype(np.float32)
    z = np.where(grp < 2, 0, 0)
    z[grp == 2] = np.where(g.random(np.sum(grp == 2)) < 0.5, 1, 2)
    zs = np.where(grp == 1, 1, 0)
    zs[grp == 2] = g.integers(0, 2, np.sum(grp == 2))
    return x, z.astype(np.int64), zs.astype(np.int64)


@pytest.mark.parametrize("merge_form", ["paper", "inverse_split"])
def test_gauss_split_merge(merge_form):
    torch = _torch()
    x, z, zs = _split_merge_case()
    seed, t = 11, 5
    model = sampler.Model("gaussian", 1.0, niw.NIWPrior(1.0, np.zeros(2), 5.0, np.eye(2)), seed=seed,
                          burn_out=2, merge_form=merge_form)
    state = sampler.State(4, z.copy(), zs.copy(), np.array([3, 3, 3, 3]))
    st0, stats = sampler.drop_empty(model, x, state)
    ref, info = sampler.split_merge(model, st0, stats, t)
    ref_stats = sampler.suffstats(model, x, ref.z, ref.zsub, ref.K)
    S = _gauss_sampler(2, 8, seed, alpha=1.0, burn_out=2, merge_form=merge_form)
    zt = torch.from_numpy(z.astype(np.int32)).cuda()
    zst = torch.from_numpy(zs.astype(np.uint8)).cuda()
    xt = torch.from_numpy(x).cuda()
    S.set_state(4, [3, 3, 3, 3])
    S.suffstats(xt, zt, zst)
    ginfo = S.split_merge(xt, t, zt, zst)
    assert (ginfo["K"], ginfo["splits"], ginfo["merges"], ginfo["removed"]) == (ref.K, info.splits, info.merges, 1)
    assert np.array_equal(zt.cpu().numpy(), ref.z) and np.array_equal(zst.cpu().numpy(), ref.zsub)
    assert np.isclose(ginfo["logpost"], sampler.log_posterior(model, ref_stats), rtol=1e-10)
    assert list(S.ages()) == list(ref.age)
    if merge_form == "paper":
        assert info.splits == 1 and info.merges == 1
    S.close()


@pytest.mark.parametrize("d", [3, 16, 17, 32, 33, 64, 65, 100])
def test_gauss_log_marginals_across_dimensions(d):
    """Cluster log marginal likelihoods (through the log posterior that the
    split/merge phase reports when no cluster is old enough to move) against
    the oracle, on both sides of every register-tile boundary of the
    marginal-likelihood kernels."""
    torch = _torch()
    g = np.random.Generator(np.random.PCG64(70 + d))
    K, n = 3, 400
    z = np.repeat(np.arange(K), n // K + 1)[:n]
    x = (g.standard_normal((n, d)) * np.linspace(0.5, 2.0, d) + 3.0 * z[:, None]).astype(np.float32)
    zs = g.integers(0, 2, n)
    psi = np.eye(d) * 0.5 + 0.1
    model = sampler.Model("gaussian", 2.0, niw.NIWPrior(0.7, np.full(d, 0.3), d + 4.0, psi), seed=1, burn_out=5)
    ref = sampler.suffstats(model, x.astype(np.float64), z, zs, K)
    from paper_2204_08988_amd.sampler import Sampler
    S = Sampler("gaussian", d, 8, 2.0, 1, kappa=0.7, nu=d + 4.0, m=np.full(d, 0.3), psi=psi, burn_out=5)
    S.set_state(K, [0] * K)
    S.set_stats(pu.stats_array(ref, "gaussian"))
    xt = torch.from_numpy(x).cuda()
    info = S.split_merge(xt, 1, torch.from_numpy(z.astype(np.int32)).cuda(),
                         torch.from_numpy(zs.astype(np.uint8)).cuda())
    assert info["K"] == K and info["splits"] == 0 and info["merges"] == 0
    assert np.isclose(info["logpost"], sampler.log_posterior(model, ref), rtol=1e-10), (info["logpost"],
                                                                                         sampler.log_posterior(model, ref))
    S.close()


def test_gauss_chain_matches_oracle_then_converges():
    torch = _torch()
    from paper_2204_08988_amd import datagen
    x, lab = datagen.workload("gauss_d2", 1)  # the configuration's N = 10 000
    d = 2
    m = x.mean(0).astype(np.float64)
    seed = 1
    model = sampler.Model("gaussian", 10.0, niw.NIWPrior(1.0, m, 5.0, np.eye(2)), seed=seed, burn_out=5)
    from paper_2204_08988_amd.sampler import Sampler
    S = Sampler("gaussian", d, 64, 10.0, seed, kappa=1.0, nu=5.0, m=m, psi=np.eye(2), burn_out=5)
    xt = torch.from_numpy(x).cuda()
    z, zs = S.init_labels(x.shape[0])
    st = sampler.initial_state(model, x.shape[0])
    assert np.array_equal(zs.cpu().numpy(), st.zsub)
    exact_iters = 0
    for t in range(1, 31):
        gi = S.step(xt, t, z, zs)
        st, oi = sampler.step(model, x.astype(np.float64), st, t)
        if gi["K"] == oi.K and np.array_equal(z.cpu().numpy(), st.z) and np.array_equal(zs.cpu().numpy(), st.zsub):
            assert np.isclose(gi["logpost"], oi.logpost, rtol=1e-9)
            exact_iters += 1
        else:
            break
    assert exact_iters >= 5
    for t in range(31, 151):
        gi = S.step(xt, t, z, zs)
    assert 4 <= gi["K"] <= 10
    assert nmi.nmi(lab, z.cpu().numpy()) > 0.8
    S.close()


# ----------------------------------------------------------------------- multinomial


def _mult_params(K, V, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    lt = np.log(g.dirichlet(np.full(V, 0.3), size=(K, 3)))
    return sampler.Params(np.log(g.dirichlet(np.ones(K))), np.log(g.dirichlet(np.ones(2), size=K)), log_theta=lt)


def _mult_points(params, n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    K, _, V = params.log_theta.shape
    lab = g.integers(0, K, n)
    tot = g.integers(5, 60, n)
    x = np.stack([g.multinomial(tot[i], np.exp(params.log_theta[lab[i], 0])) for i in range(n)])
    return x.astype(np.int32)


@pytest.mark.parametrize("V,K,n", [(100, 50, 4000), (7, 3, 3001), (40, 9, 2000), (128, 2, 1500), (33, 70, 6000)])
def test_mult_loglik_labels_stats(V, K, n):
    torch = _torch()
    from paper_2204_08988_amd.sampler import Sampler
    seed = 500 + V + K
    params = _mult_params(K, V, seed)
    x = _mult_points(params, n, seed + 1)
    S = Sampler("multinomial", V, K + 2, 2.0, seed, beta=np.ones(V))
    S.set_params(params.log_pi, params.log_pisub, pu.comp_array(params))
    xt = torch.from_numpy(x).cuda()
    model = sampler.Model("multinomial", 2.0, dirmult.DirPrior(np.ones(V)), seed=seed)
    lc, ls = sampler.loglik(model, x, params)
    Mc, Ms = pu.mult_scale(x, params)
    ll = S.loglik(xt).cpu().numpy().astype(np.float64)
    assert pu.check_loglik(ll, lc, ls, Mc, Ms) <= 1e-5
    z, zs = S.sample_labels(xt, 3)
    zn, zsn = z.cpu().numpy(), zs.cpu().numpy()
    bad_c, bad_s, tie_c, tie_s = pu.label_mismatches(seed, 3, zn, zsn, lc, ls, Mc, Ms)
    assert bad_c.size == 0 and bad_s.size == 0
    S.suffstats(xt, z, zs)
    got = S.get_stats()
    ref = pu.stats_array(sampler.suffstats(model, x, zn, zsn, K), "multinomial")
    assert np.array_equal(got, ref)
    S.close()


def test_mult_params_and_split_merge():
    torch = _torch()
    from paper_2204_08988_amd.sampler import Sampler
    V, K, seed = 30, 4, 21
    params = _mult_params(K, V, seed)
    x = _mult_points(params, 3000, seed + 1)
    g = np.random.Generator(np.random.PCG64(2))
    z = g.integers(0, K, 3000)
    zs = g.integers(0, 2, 3000)
    model = sampler.Model("multinomial", 2.0, dirmult.DirPrior(np.full(V, 0.5)), seed=seed, burn_out=0)
    st = sampler.suffstats(model, x, z, zs, K)
    S = Sampler("multinomial", V, 16, 2.0, seed, beta=np.full(V, 0.5), burn_out=0)
    S.set_stats(pu.stats_array(st, "multinomial"))
    S.sample_params(6)
    lp, lps, lt = S.get_params()
    ref = sampler.sample_params(model, st, 6)
    assert np.allclose(lp, ref.log_pi, rtol=1e-10) and np.allclose(lt, ref.log_theta, rtol=1e-10, atol=1e-10)
    zt = torch.from_numpy(z.astype(np.int32)).cuda()
    zst = torch.from_numpy(zs.astype(np.uint8)).cuda()
    xt = torch.from_numpy(x).cuda()
    S.set_state(K, [0] * K)
    S.suffstats(xt, zt, zst)
    gi = S.split_merge(xt, 6, zt, zst)
    state = sampler.State(K, z.copy(), zs.copy(), np.zeros(K, dtype=np.int64))
    st0, stats = sampler.drop_empty(model, x, state)
    refs, info = sampler.split_merge(model, st0, stats, 6)
    assert gi["K"] == refs.K and gi["merges"] == info.merges and gi["splits"] == info.splits
    assert np.array_equal(zt.cpu().numpy(), refs.z) and np.array_equal(zst.cpu().numpy(), refs.zsub)
    S.close()


@pytest.mark.parametrize("d,K,n", [(2, 12, 3000), (20, 9, 4000), (64, 8, 3000), (128, 6, 2500)])
def test_gauss_merges_with_the_merge_bound(d, K, n):
    """Many clusters over three true groups: the fragments of one group are
    merge candidates, the rest are pruned by the merge bound.  The GPU's split /
    merge phase must take exactly the oracle's decisions (the oracle computes
    every pair's ratio in full)."""
    torch = _torch()
    g = np.random.Generator(np.random.PCG64(600 + d))
    grp = g.integers(0, 3, n)
    centres = g.normal(0, 6.0, size=(3, d))
    x = (centres[grp] + g.standard_normal((n, d))).astype(np.float32)
    # clusters: random fragments of the groups (each cluster within one group)
    z = np.where(grp == 0, g.integers(0, K // 3, n), np.where(grp == 1, K // 3 + g.integers(0, K // 3, n),
                                                                 2 * (K // 3) + g.integers(0, K - 2 * (K // 3), n)))
    zs = g.integers(0, 2, n)
    seed, t = 17 + d, 3
    prior = niw.NIWPrior(1.0, np.zeros(d), d + 3.0, np.eye(d))
    for form in ("paper", "inverse_split"):
        model = sampler.Model("gaussian", 1.0, prior, seed=seed, burn_out=1, merge_form=form)
        state = sampler.State(K, z.copy(), zs.copy(), np.full(K, 2))
        st0, stats = sampler.drop_empty(model, x, state)
        ref, info = sampler.split_merge(model, st0, stats, t)
        S = _gauss_sampler(d, 2 * K, seed, alpha=1.0, burn_out=1, merge_form=form)
        zt = torch.from_numpy(z.astype(np.int32)).cuda()
        zst = torch.from_numpy(zs.astype(np.uint8)).cuda()
        xt = torch.from_numpy(x).cuda()
        S.set_state(K, [2] * K)
        S.suffstats(xt, zt, zst)
        gi = S.split_merge(xt, t, zt, zst)
        assert (gi["K"], gi["splits"], gi["merges"]) == (ref.K, info.splits, info.merges)
        assert np.array_equal(zt.cpu().numpy(), ref.z) and np.array_equal(zst.cpu().numpy(), ref.zsub)
        if form == "paper":
            assert info.merges >= 1
        S.close()
