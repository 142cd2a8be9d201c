"""GPU parity of the Poisson family (a product of independent Poisson counts
with a Gamma prior on each rate): log-likelihoods, labels and statistics,
the conjugate parameter draws, the split/merge decisions (Gamma-Poisson log
marginals), against the FP64 oracle; a chain on Poisson data that finds its
clusters; the user-level fit with checkpoint resume.

Log-likelihood scale (the comparison rule of the other families):
M = |log w| + sum_v x_v |log lambda_v| + sum_v lambda_v."""
import numpy as np
import pytest

from oracle import nmi, poisson, sampler
from tests import parity_util as pu

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _pois_params(K, d, seed, scale=8.0):
    g = np.random.Generator(np.random.PCG64(seed))
    lam = g.gamma(1.5, scale / 1.5, size=(K, 1, d)) * np.exp(g.normal(0, 0.1, size=(K, 3, d)))
    return sampler.Params(np.log(g.dirichlet(np.ones(K))), np.log(g.dirichlet(np.ones(2), size=K)),
                          log_theta=np.log(lam))


def _pois_points(params, n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    K = params.log_theta.shape[0]
    lab = g.integers(0, K, n)
    return g.poisson(np.exp(params.log_theta[lab, 0])).astype(np.int32)


def _pois_scale(x, params):
    K = params.log_theta.shape[0]
    x = np.asarray(x, dtype=np.float64)
    Mc = np.zeros((x.shape[0], K))
    Ms = np.zeros((x.shape[0], K, 2))
    for k in range(K):
        lt = params.log_theta[k]
        Mc[:, k] = abs(params.log_pi[k]) + x @ np.abs(lt[0]) + np.exp(lt[0]).sum()
        for h in range(2):
            Ms[:, k, h] = abs(params.log_pisub[k, h]) + x @ np.abs(lt[1 + h]) + np.exp(lt[1 + h]).sum()
    return Mc, Ms


def _prior(d, seed=0):
    g = np.random.Generator(np.random.PCG64(seed))
    return poisson.GammaPrior(g.uniform(0.5, 2.0, d), g.uniform(0.1, 1.0, d))


def _sampler(d, k_max, seed, prior, **kw):
    from paper_2204_08988_amd.sampler import Sampler
    return Sampler("poisson", d, k_max, kw.pop("alpha", 2.0), seed, gamma_shape=prior.shape,
                   gamma_rate=prior.rate, **kw)


# (d, K, n): one coordinate; the vocabulary-sized tiles of the count kernels
# (several tiles and a ragged tail); the largest d; many clusters
@pytest.mark.parametrize("d,K,n", [(1, 3, 2001), (20, 12, 6000), (37, 5, 4097), (128, 4, 1500), (8, 70, 5000)])
def test_pois_loglik_labels_stats(d, K, n):
    torch = _torch()
    seed = 700 + d + K
    params = _pois_params(K, d, seed)
    x = _pois_points(params, n, seed + 1)
    prior = _prior(d, seed)
    S = _sampler(d, K + 2, seed, prior)
    S.set_params(params.log_pi, params.log_pisub, pu.comp_array(params))
    xt = torch.from_numpy(x).cuda()
    model = sampler.Model("poisson", 2.0, prior, seed=seed)
    lc, ls = sampler.loglik(model, x, params)
    Mc, Ms = _pois_scale(x, params)
    ll = S.loglik(xt).cpu().numpy().astype(np.float64)
    assert pu.check_loglik(ll, lc, ls, Mc, Ms) <= 1e-5
    for t in (3, 4):
        z, zs = S.sample_labels(xt, t)
        zn, zsn = z.cpu().numpy(), zs.cpu().numpy()
        bad_c, bad_s, tie_c, tie_s = pu.label_mismatches(seed, t, zn, zsn, lc, ls, Mc, Ms)
        assert bad_c.size == 0 and bad_s.size == 0, (bad_c[:10], bad_s[:10])
        assert tie_c + tie_s <= max(2, n // 1000)
    S.suffstats(xt, z, zs)
    got = S.get_stats()
    ref = pu.stats_array(sampler.suffstats(model, x, zn, zsn, K), "poisson")
    assert np.array_equal(got, ref)
    S.close()


@pytest.mark.parametrize("d,K", [(1, 2), (6, 4), (50, 3), (128, 2)])
def test_pois_sample_params(d, K):
    """Weights and log rates of one draw from the conjugate posteriors, from the
    same statistics and the same (seed, t): log lambda_v = log Gamma(a_v + c_v)
    variate - log(b_v + n)."""
    _torch()
    seed = 40 + d
    g = np.random.Generator(np.random.PCG64(seed))
    prior = _prior(d, seed)
    n = g.integers(0, 500, size=(K, 2))
    n[0, 1] = 0  # an empty sub-cluster: its rates are prior draws
    s = np.where(n[..., None] > 0, g.poisson(3.0 * n[..., None], size=(K, 2, d)), 0)
    st = sampler.Stats(n, s=s)
    model = sampler.Model("poisson", 2.0, prior, seed=seed, burn_out=0)
    S = _sampler(d, K + 1, seed, prior, burn_out=0)
    S.set_stats(pu.stats_array(st, "poisson"))
    for t in (1, 9):
        S.sample_params(t)
        lp, lps, lt = S.get_params()
        ref = sampler.sample_params(model, st, t)
        assert np.allclose(lp, ref.log_pi, rtol=1e-10, atol=1e-12)
        assert np.allclose(lps, ref.log_pisub, rtol=1e-10, atol=1e-12)
        assert np.allclose(lt, ref.log_theta, rtol=1e-10, atol=1e-10)
    S.close()


@pytest.mark.parametrize("merge_form", ["paper", "inverse_split"])
def test_pois_split_merge(merge_form):
    """Splits and merges from the same statistics and (seed, t): the decisions
    rest on the Gamma-Poisson log marginals, so they must match the oracle's,
    and so must the relabelled (z, zsub)."""
    torch = _torch()
    d, K, seed = 12, 5, 23
    params = _pois_params(K, d, seed, scale=4.0)
    x = _pois_points(params, 4000, seed + 1)
    prior = _prior(d, seed)
    g = np.random.Generator(np.random.PCG64(3))
    z = g.integers(0, K, 4000)
    z[z == 4] = 3  # one cluster empty at the start: dropped before the moves
    zs = g.integers(0, 2, 4000)
    model = sampler.Model("poisson", 2.0, prior, seed=seed, burn_out=0, merge_form=merge_form)
    S = _sampler(d, 16, seed, prior, burn_out=0, merge_form=merge_form)
    xt = torch.from_numpy(x).cuda()
    zt = torch.from_numpy(z.astype(np.int32)).cuda()
    zst = torch.from_numpy(zs.astype(np.uint8)).cuda()
    for t in (6, 7):
        K_now = int(zt.max().item()) + 1
        zn, zsn = zt.cpu().numpy().astype(np.int64), zst.cpu().numpy().astype(np.int64)
        S.set_state(K_now, [0] * K_now)
        S.suffstats(xt, zt, zst)
        gi = S.split_merge(xt, t, zt, zst)
        state = sampler.State(K_now, zn.copy(), zsn.copy(), np.zeros(K_now, dtype=np.int64))
        st0, stats = sampler.drop_empty(model, x, state)
        refs, info = sampler.split_merge(model, st0, stats, t)
        assert gi["K"] == refs.K and gi["merges"] == info.merges and gi["splits"] == info.splits
        assert np.array_equal(zt.cpu().numpy(), refs.z) and np.array_equal(zst.cpu().numpy(), refs.zsub)
        ref_stats = sampler.suffstats(model, x, refs.z, refs.zsub, refs.K)
        assert np.isclose(gi["logpost"], sampler.log_posterior(model, ref_stats), rtol=1e-10)
    S.close()


def test_pois_log_marginals_through_logpost():
    """The log posterior the step reports (Gamma-Poisson marginals of every
    cluster and the CRP prior) against the oracle's on the same labels."""
    torch = _torch()
    d, K, seed = 9, 4, 61
    params = _pois_params(K, d, seed)
    x = _pois_points(params, 3000, seed + 1)
    prior = _prior(d, seed)
    model = sampler.Model("poisson", 2.0, prior, seed=seed, burn_out=50)
    S = _sampler(d, 8, seed, prior, burn_out=50)
    g = np.random.Generator(np.random.PCG64(5))
    z = g.integers(0, K, 3000)
    zs = g.integers(0, 2, 3000)
    xt = torch.from_numpy(x).cuda()
    zt = torch.from_numpy(z.astype(np.int32)).cuda()
    zst = torch.from_numpy(zs.astype(np.uint8)).cuda()
    S.set_state(K, [0] * K)
    info = S.step(xt, 2, zt, zst)
    zn, zsn = zt.cpu().numpy(), zst.cpu().numpy()
    ref = sampler.log_posterior(model, sampler.suffstats(model, x, zn, zsn, info["K"]))
    assert abs(info["logpost"] - ref) <= 1e-9 * abs(ref)
    S.close()


def test_pois_chain_finds_clusters():
    torch = _torch()
    from paper_2204_08988_amd import datagen
    x, lab = datagen.workload("pois_d20", 3, n=40_000)
    d = x.shape[1]
    prior = poisson.GammaPrior(np.ones(d), np.full(d, 0.1))
    S = _sampler(d, 64, 3, prior, alpha=10.0, burn_out=5)
    xt = torch.from_numpy(x).cuda()
    z, zs = S.init_labels(x.shape[0])
    for t in range(1, 101):
        info = S.step(xt, t, z, zs)
    assert 17 <= info["K"] <= 24
    assert nmi.nmi(lab, z.cpu().numpy()) > 0.95
    S.close()


def test_pois_fit_and_checkpoint(tmp_path):
    from paper_2204_08988_amd import datagen, fit
    x, lab = datagen.workload("pois_d20", 2, n=20_000)
    cfg = {"prior_type": "Poisson", "iterations": 30, "burn_out": 3, "seed": 8,
           "hyper_params": {"shape": [1.0] * 20, "rate": [0.1] * 20}}
    full = fit.fit(x, cfg, gt=lab)
    half = dict(cfg, iterations=15)
    a = fit.fit(x, half, checkpoint_path=tmp_path / "c.ckpt")
    b = fit.fit(x, half, resume_path=tmp_path / "c.ckpt")
    assert a["K_trace"] + b["K_trace"] == full["K_trace"]
    assert b["labels"] == full["labels"] and b["weights"] == full["weights"]
    assert max(full["K_trace"]) > 1
