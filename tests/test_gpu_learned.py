"""GPU parity of the learned split proposal (an added form) against the FP64
oracle: network forward / gradient / Adam, set features, the learned move's
Metropolis-Hastings pieces given the GPU's Bernoulli sides, and a chain of
GPU learned moves alone against the enumerated partition posterior.

Tolerances: the network runs in BF16 with FP32 accumulation, so logits and
gradients are compared by relative L2 error (1e-2 for arbitrary operands;
4e-3 when the inputs and weights are BF16-exact and only the hidden
activations are rounded) and gradient cosine >= 0.999; features are FP32
products of float64 frames (atol 1e-4 (1 + |f|)); the float64 marginal
likelihood pieces agree to 1e-7 relative."""
from collections import Counter

import numpy as np
import pytest
from scipy.special import gammaln

from oracle import learned, mlp, niw, partitions, rng, sampler

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _bf16(a):
    torch = _torch()
    return torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _sampler(d, m, seed, k_max=16, **kw):
    from paper_2204_08988_amd.sampler import Sampler
    prior = kw.pop("prior", None)
    if prior is None:
        prior = niw.NIWPrior(1.0, np.zeros(d), d + 3.0, np.eye(d))
    return Sampler("gaussian", d, k_max, kw.pop("alpha", 2.0), seed, kappa=prior.kappa, nu=prior.nu,
                   m=np.asarray(prior.m, dtype=np.float64), psi=np.asarray(prior.psi, dtype=np.float64),
                   learned=m, **kw)


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _forward_error_bound(theta, X, F, exact):
    """First-order bound on |logit_gpu - logit| per row: every BF16 rounding
    (X, W1, H1, W2; none of X, W1, W2 when `exact`) has relative error at most
    2^-9, propagated through the absolute values of the layers (ReLU is
    1-Lipschitz); FP32 accumulation adds 1e-5 of the absolute magnitudes."""
    W1, b1, W2, b2, w3, b3 = mlp.unpack(theta, F)
    u = 2.0 ** -9
    aX, aW1, aW2, aw3 = np.abs(X), np.abs(W1), np.abs(W2), np.abs(w3)
    a1 = np.maximum(X @ W1 + b1, 0)
    e1 = 0.0 if exact else 2 * u * (aX @ aW1)
    ea1 = e1 + u * (np.abs(a1) + e1)
    e2 = ea1 @ aW2 + (0.0 if exact else u * ((np.abs(a1) + ea1) @ aW2))
    scale = (np.abs(a1) @ aW2 + np.abs(b2)) @ aw3 + abs(b3) + (aX @ aW1 + np.abs(b1)) @ aW2 @ aw3
    return 1.05 * (e2 @ aw3) + 1e-5 * scale


@pytest.mark.parametrize("n,exact", [(1, True), (777, True), (777, False), (70001, False)])
def test_mlp_forward_matches_oracle(n, exact):
    torch = _torch()
    m = 3
    F = 2 * m
    S = _sampler(8, m, 1)
    theta = mlp.init(F, 21)
    g = np.random.Generator(np.random.PCG64(n))
    X = g.standard_normal((n, F)) * 1.5
    if exact:
        W1, b1, W2, b2, w3, b3 = mlp.unpack(theta, F)
        theta = mlp.pack(_bf16(W1), b1, _bf16(W2), b2, w3, b3)
        X = _bf16(X)
    S.mlp_set_weights(theta)
    theta = theta.astype(np.float32).astype(np.float64)
    X = X.astype(np.float32).astype(np.float64)
    assert np.array_equal(S.mlp_get_weights(), theta)
    o = S.mlp_forward(torch.tensor(X, dtype=torch.float32).cuda()).cpu().numpy().astype(np.float64)
    ref, _ = mlp.forward(theta, X, F)
    bound = _forward_error_bound(theta, X, F, exact)
    assert np.all(np.abs(o - ref) <= bound), np.max(np.abs(o - ref) / bound)
    assert _rel_l2(o, ref) <= 1e-2


@pytest.mark.parametrize("n", [5, 3000, 70001])
def test_mlp_gradient_matches_oracle(n):
    torch = _torch()
    m = 2
    F = 2 * m
    S = _sampler(4, m, 2)
    theta = mlp.init(F, 22).astype(np.float32).astype(np.float64)
    S.mlp_set_weights(theta)
    g = np.random.Generator(np.random.PCG64(100 + n))
    X = (g.standard_normal((n, F))).astype(np.float32)
    y = (g.random(n) < 1.0 / (1.0 + np.exp(-2.0 * X[:, 0]))).astype(np.float32)
    grad, loss = S.mlp_grad(torch.tensor(X).cuda(), torch.tensor(y).cuda())
    ref = mlp.backward(theta, X.astype(np.float64), y.astype(np.float64), F)
    ref_loss = mlp.loss(theta, X.astype(np.float64), y.astype(np.float64), F)
    assert _rel_l2(grad, ref) <= 1e-2, _rel_l2(grad, ref)
    cos = float(grad @ ref / (np.linalg.norm(grad) * np.linalg.norm(ref)))
    assert cos >= 0.999, cos
    assert abs(loss - ref_loss) <= 1e-2 * abs(ref_loss) + 1e-6
    # each parameter block separately (a dropped or misplaced block fails here)
    of = [0, F * 128, F * 128 + 128, F * 128 + 128 + 128 * 128, F * 128 + 256 + 128 * 128,
          F * 128 + 384 + 128 * 128, F * 128 + 385 + 128 * 128]
    for a, b in zip(of[:-1], of[1:]):
        assert _rel_l2(grad[a:b], ref[a:b]) <= 2e-2, (a, b)


def test_adam_matches_oracle_adam_on_the_gpu_gradient():
    torch = _torch()
    m = 2
    F = 2 * m
    S = _sampler(4, m, 3)
    theta = mlp.init(F, 23).astype(np.float32).astype(np.float64)
    S.mlp_set_weights(theta)
    g = np.random.Generator(np.random.PCG64(7))
    X = torch.tensor(g.standard_normal((500, F)).astype(np.float32)).cuda()
    y = torch.tensor((g.random(500) < 0.3).astype(np.float32)).cuda()
    opt = mlp.Adam(theta.size, lr=1e-2)
    p = theta.copy()
    for _ in range(4):
        grad, _ = S.mlp_grad(X, y)
        S.mlp_adam_step(X, y, 1e-2)
        p = opt.step(p, grad)
        got = S.mlp_get_weights()
        assert np.all(np.abs(got - p) <= 1e-5 * np.abs(p) + 2e-4 * 1e-2), np.max(np.abs(got - p))


def _two_cluster_data(d, seed, n=(900, 700)):
    g = np.random.Generator(np.random.PCG64(seed))
    xs, zs = [], []
    for k, nk in enumerate(n):
        q, _ = np.linalg.qr(g.standard_normal((d, d)))
        ev = np.linspace(3.0, 0.3, d) ** 2 * (k + 1)   # well separated spectrum
        A = q * np.sqrt(ev)
        xs.append(g.standard_normal((nk, d)) @ A.T + g.normal(0, 3, d))
        zs.append(np.full(nk, k))
    x = np.concatenate(xs).astype(np.float32)
    z = np.concatenate(zs)
    perm = g.permutation(z.size)
    return x[perm], z[perm]


@pytest.mark.parametrize("d,m", [(6, 3), (1, 1), (32, 8)])
def test_set_features_match_oracle(d, m):
    torch = _torch()
    x, z = _two_cluster_data(d, 40 + d)
    zs = (np.arange(z.size) % 2).astype(np.uint8)
    S = _sampler(d, m, 4)
    S.set_state(2)
    xt = torch.tensor(x).cuda()
    zt = torch.tensor(z.astype(np.int32)).cuda()
    S.suffstats(xt, zt, torch.tensor(zs).cuda())
    xd = x.astype(np.float64)
    for k1, k2 in ((0, -1), (1, -1), (0, 1)):
        C = np.nonzero((z == k1) | (z == k2))[0]
        feats, idx = S.set_features(xt, zt, k1, k2)
        assert np.array_equal(idx.cpu().numpy(), C)
        ref = learned.features(xd[C], C.size, xd[C].sum(0), xd[C].T @ xd[C], m)
        got = feats.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - ref) <= 1e-4 * (1 + np.abs(ref))), np.max(np.abs(got - ref))


def _move_case(d, m, seed):
    """Three labelled clusters, GPU sampler with current statistics."""
    torch = _torch()
    g = np.random.Generator(np.random.PCG64(seed))
    centers = g.normal(0, 2.5, (3, d))
    n = (300, 200, 250)
    x = np.concatenate([g.standard_normal((nk, d)) + centers[k] for k, nk in enumerate(n)]).astype(np.float32)
    z = np.concatenate([np.full(nk, k) for k, nk in enumerate(n)])
    perm = g.permutation(z.size)
    x, z = x[perm], z[perm]
    prior = niw.NIWPrior(1.0, np.zeros(d), d + 3.0, np.eye(d))
    model = sampler.Model("gaussian", 2.0, prior, seed=seed, burn_out=0)
    S = _sampler(d, m, seed, prior=prior, burn_out=0)
    theta = mlp.init(2 * m, seed).astype(np.float32).astype(np.float64)
    S.mlp_set_weights(theta)
    return torch, x, z, model, S, theta


@pytest.mark.parametrize("d,m", [(2, 2), (8, 3), (40, 4)])
def test_learned_move_pieces_match_oracle_given_gpu_sides(d, m):
    torch, x, z, model, S, theta = _move_case(d, m, 60 + d)
    xd = x.astype(np.float64)
    xt = torch.tensor(x).cuda()
    seen = Counter()
    for t in range(1, 41):
        K = int(z.max()) + 1
        S.set_state(K)
        zt = torch.tensor(z.astype(np.int32)).cuda()
        zst = torch.zeros(z.size, dtype=torch.uint8).cuda()
        S.suffstats(xt, zt, zst)
        side_t = torch.full((z.size,), 7, dtype=torch.uint8).cuda()
        info = S.learned_move(xt, t, zt, zst, side_t)
        # move selection
        w = rng.block(model.seed, t, 0, rng.TAG_MOVE, 0)
        u_type, u_pick, u_acc = (float(rng.uniform(w[j])) for j in range(3))
        split = K == 1 or u_type < 0.5
        assert info["kind"] == (1 if split else 2)
        if split:
            C = np.nonzero(z == min(int(u_pick * K), K - 1))[0]
            assert info["k1"] == z[C[0]]
        else:
            npairs = K * (K - 1) // 2
            k1, k2 = learned.pair_of(min(int(u_pick * npairs), npairs - 1), K)
            assert (info["k1"], info["k2"]) == (k1, k2)
            C = np.nonzero((z == k1) | (z == k2))[0]
        side = side_t.cpu().numpy()
        assert np.all(side[np.setdiff1d(np.arange(z.size), C)] == 7)
        sa = side[C] == 1
        zn = zt.cpu().numpy()
        zs_after = zst.cpu().numpy()
        K_after = S.K
        assert K_after == K + (1 if split else -1) * info["accepted"]
        # the GPU's probabilities, from the same features and network, on the
        # state before the move
        z0 = torch.tensor(z.astype(np.int32)).cuda()
        S.set_state(K)
        S.suffstats(xt, z0, torch.zeros(z.size, dtype=torch.uint8).cuda())
        feats, idx = S.set_features(xt, z0, info["k1"], info["k2"])
        assert np.array_equal(idx.cpu().numpy(), C)
        o = S.mlp_forward(feats).cpu().numpy().astype(np.float64)
        b = np.clip(1.0 / (1.0 + np.exp(-o)), learned.CLIP, 1 - learned.CLIP)
        if split:
            u = rng.uniform(rng.block(model.seed, t, C.astype(np.uint64), rng.TAG_BERN, 0)[0])
            near = np.abs(u - b) <= 1e-5 * (1 + b)
            assert np.array_equal(sa[~near], (u < b)[~near])
            # and the oracle's own float64 network agrees up to the BF16 logit error
            b_ref = learned.probs(theta, learned.features(xd[C], C.size, xd[C].sum(0), xd[C].T @ xd[C], m), 2 * m)
            assert np.mean(sa != (u < b_ref)) <= 0.02
        else:
            assert np.array_equal(sa, z[C] == info["k1"])
        assert info["n_a"] == sa.sum() and info["n_b"] == (~sa).sum()
        assert abs(info["log_q_part"] - learned.log_q_partition(b, sa)) <= 1e-6 * C.size + 1e-9
        seen[(info["kind"], info["skipped"])] += 1
        if info["skipped"]:
            assert info["skipped"] == 1 and (sa.all() or not sa.any())
            continue
        A, B = C[sa], C[~sa]
        lm = lambda r: niw.log_marginal(model.prior, r.size, xd[r].sum(0), xd[r].T @ xd[r])
        target = (np.log(model.alpha) + gammaln(A.size) + lm(A) + gammaln(B.size) + lm(B)
                  - gammaln(C.size) - lm(C))
        assert abs(info["log_target"] - target) <= 1e-7 * (1 + abs(lm(A)) + abs(lm(B)) + abs(lm(C)))
        if split:
            lq_fwd = np.log(1.0 if K == 1 else 0.5) - np.log(K) + info["log_q_part"]
            lq_rev = np.log(0.5) - np.log((K + 1) * K / 2.0)
            lh = info["log_target"] + lq_rev - lq_fwd
        else:
            lq_fwd = np.log(0.5) - np.log(K * (K - 1) / 2.0)
            lq_rev = np.log(1.0 if K - 1 == 1 else 0.5) - np.log(K - 1) + info["log_q_part"]
            lh = -info["log_target"] + lq_rev - lq_fwd
        assert np.isclose(info["log_h"], lh, rtol=1e-12, atol=1e-12)
        # the oracle's Hastings ratio for the same sides, given the GPU's
        # probabilities, is the same number
        assert info["accepted"] == int(np.log(u_acc) < info["log_h"])
        if info["accepted"]:
            if split:
                exp = z.copy()
                exp[A] = K
                assert np.array_equal(zn, exp)
                fresh = rng.block(model.seed, t, C.astype(np.uint64), learned.TAG_LEARNSUB, 0)[0] & np.uint32(1)
                assert np.array_equal(zs_after[C], fresh.astype(np.uint8))
            else:
                exp = z.copy()
                exp[z == info["k2"]] = info["k1"]
                exp[exp > info["k2"]] -= 1
                assert np.array_equal(zn, exp)
                assert np.all(zs_after[z == info["k1"]] == 0) and np.all(zs_after[z == info["k2"]] == 1)
            z = zn.astype(np.int64)
        else:
            assert np.array_equal(zn, z)
    assert seen[(1, 0)] > 0 and seen[(2, 0)] > 0, seen


def test_learned_moves_alone_sample_the_exact_partition_posterior():
    torch = _torch()
    x = np.array([[-1.2], [-0.9], [0.1], [1.5], [1.8]])
    prior = niw.NIWPrior(0.5, np.array([0.0]), 2.0, np.array([[0.5]]))
    lm = lambda rows: niw.log_marginal(prior, len(rows), x[rows].sum(0), x[rows].T @ x[rows])
    ex = partitions.exact_posterior(x, 1.0, lm)
    S = _sampler(1, 1, 11, alpha=1.0, prior=prior, burn_out=0, k_max=8)
    S.mlp_set_weights(mlp.init(2, 13).astype(np.float32).astype(np.float64))
    xt = torch.tensor(x.astype(np.float32)).cuda()
    zt = torch.zeros(5, dtype=torch.int32).cuda()
    zst = torch.zeros(5, dtype=torch.uint8).cuda()
    S.set_state(1)
    S.suffstats(xt, zt, zst)
    h = Counter()
    moves = 40000
    for t in range(1, moves + 1):
        S.learned_move(xt, t, zt, zst)
        h[partitions.canonical(zt.cpu().numpy())] += 1
    tv = partitions.total_variation(h, ex)
    print(f"GPU learned-move chain: TV to exact posterior = {tv:.3f}")
    assert tv < 0.05


def test_training_learns_a_principal_axis_split():
    """One cluster whose sub-labels are the sign of the first principal
    coordinate (the split the set features expose): training on the sampler's
    own sub-labels must learn it."""
    torch = _torch()
    d, m, n = 6, 3, 20000
    g = np.random.Generator(np.random.PCG64(8))
    q, _ = np.linalg.qr(g.standard_normal((d, d)))
    x = ((g.standard_normal((n, d)) * np.array([3.0, 1, 1, 1, 1, 1])) @ q.T + 2.0).astype(np.float32)
    xd = x.astype(np.float64)
    f = learned.features(xd, n, xd.sum(0), xd.T @ xd, m)
    zs = np.where(f[:, 0] > 0, 0, 1).astype(np.uint8)   # l = positive side
    S = _sampler(d, m, 9, burn_out=3)
    S.set_state(1, ages=[10])
    xt = torch.tensor(x).cuda()
    zt = torch.zeros(n, dtype=torch.int32).cuda()
    zst = torch.tensor(zs).cuda()
    S.suffstats(xt, zt, zst)
    l0 = S.mlp_train(xt, zt, zst, 1, 2048, 3e-3)
    loss = S.mlp_train(xt, zt, zst, 300, 2048, 3e-3)
    feats, idx = S.set_features(xt, zt, 0)
    o = S.mlp_forward(feats).cpu().numpy()
    acc = float(np.mean((o > 0) == (zs[idx.cpu().numpy()] == 0)))
    print(f"loss {l0:.3f} -> {loss:.3f}, accuracy {acc:.4f}")
    assert loss < 0.15 and acc > 0.97, (l0, loss, acc)
    # the opposite labelling trains the same network (targets are canonicalised)
    S.suffstats(xt, zt, 1 - zst)
    assert S.mlp_train(xt, zt, 1 - zst, 20, 2048, 3e-3) < 0.15


def test_learned_step_and_training_on_a_mixture():
    """Chain with one learned move per iteration and periodic training on
    clusters with a dominant major axis (their sub-clusters split along it,
    the direction the set features expose): the network must beat chance on
    the sampler's own sub-labels and the chain must recover the mixture."""
    torch = _torch()
    d, K_true, n = 8, 6, 30000
    g = np.random.Generator(np.random.PCG64(5))
    mus = g.normal(0, 10.0, (K_true, d))
    chol = []
    for _ in range(K_true):
        q, _ = np.linalg.qr(g.standard_normal((d, d)))
        chol.append(q * np.array([2.5, 1, 1, 1, 1, 1, 1, 1]))
    zt_true = g.integers(0, K_true, n)
    eps = g.standard_normal((n, d))
    x = np.stack([chol[k] @ e for k, e in zip(zt_true, eps)]) + mus[zt_true]
    x = x.astype(np.float32)
    S = _sampler(d, 4, 77, k_max=32, burn_out=5)
    xt = torch.tensor(x).cuda()
    z, zs = S.init_labels(n)
    kinds = Counter()
    losses = []
    for t in range(1, 101):
        info = S.step(xt, t, z, zs)
        kinds[info["learned_kind"]] += 1
        if t % 20 == 0:
            losses.append(S.mlp_train(xt, z, zs, 100, 2048, 2e-3))
    from oracle import nmi
    score = nmi.nmi(zt_true, z.cpu().numpy())
    print(f"losses {losses}, K {S.K}, NMI {score:.4f}, moves {dict(kinds)}")
    assert kinds[1] + kinds[2] == 100
    # converged single-Gaussian clusters let one sub-cluster take every point,
    # so late training sets are small or empty (NaN) and close to chance
    assert all(np.isnan(l) or 0.0 < l < 1.0 for l in losses), losses
    assert score > 0.9, (score, S.K)


def test_trained_proposal_splits_a_two_component_cluster():
    """The purpose of the learned proposal: a cluster holding two true
    components, whose sub-clusters have found them, is split in one learned
    move once the network has been trained on those sub-labels, while an
    untrained network's proposal is rejected.  (The sub-labels are set to the
    components here: from a symmetric start the restricted Gibbs sweep maps
    the sub-cluster mean gap to about itself while both sub-clusters carry
    the full between-component variance, so finding them can take the
    sampler many iterations.)"""
    torch = _torch()
    from oracle import nmi
    d, n = 8, 20000
    g = np.random.Generator(np.random.PCG64(12))
    v = g.standard_normal(d)
    v /= np.linalg.norm(v)
    truth = g.integers(0, 2, n)
    x = (g.standard_normal((n, d)) + np.outer(np.where(truth == 1, 4.0, -4.0), v) + 1.0).astype(np.float32)
    S = _sampler(d, 4, 31, k_max=8, burn_out=3)
    xt = torch.tensor(x).cuda()
    z = torch.zeros(n, dtype=torch.int32).cuda()
    zs = torch.tensor(truth.astype(np.uint8)).cuda()
    S.set_state(1, ages=[10])
    S.suffstats(xt, z, zs)
    before = S.learned_move(xt, 100, z, zs)
    assert before["kind"] == 1 and not before["accepted"] and before["log_h"] < 0, before
    loss = S.mlp_train(xt, z, zs, 200, 2048, 3e-3)
    assert loss < 0.1, loss
    after = S.learned_move(xt, 101, z, zs)
    print(f"untrained log H {before['log_h']:.1f}, trained log H {after['log_h']:.1f}, loss {loss:.4f}")
    assert after["accepted"] and after["log_h"] > 10, after
    assert S.K == 2 and nmi.nmi(truth, z.cpu().numpy()) > 0.99
