"""Pins of the learned-proposal oracle: MLP gradients against central finite
differences and torch autograd (float64), Adam against torch.optim.Adam, set
features' invariances, the split/merge detailed-balance identity, and a chain
of learned moves alone against the enumerated partition posterior."""
from collections import Counter

import numpy as np
import pytest

from oracle import learned, mlp, niw, partitions, sampler

F = 6


def _batch(n=40, seed=0):
    g = np.random.Generator(np.random.PCG64(seed))
    return g.standard_normal((n, F)), (g.random(n) < 0.4).astype(np.float64)


def test_gradient_matches_central_differences():
    theta = mlp.init(F, 3)
    X, y = _batch()
    g = mlp.backward(theta, X, y, F)
    rs = np.random.Generator(np.random.PCG64(1))
    idx = rs.choice(theta.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss(tp, X, y, F) - mlp.loss(tm, X, y, F)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(fd)), i


def test_forward_backward_match_torch_autograd():
    torch = pytest.importorskip("torch")
    theta = mlp.init(F, 4)
    X, y = _batch(64, 2)
    W1, b1, W2, b2, w3, b3 = (torch.tensor(np.array(a), dtype=torch.float64, requires_grad=True)
                              for a in mlp.unpack(theta, F))
    Xt = torch.tensor(X)
    o = torch.relu(torch.relu(Xt @ W1 + b1) @ W2 + b2) @ w3 + b3
    L = torch.nn.functional.binary_cross_entropy_with_logits(o, torch.tensor(y), reduction="sum")
    L.backward()
    ref = mlp.pack(W1.grad.numpy(), b1.grad.numpy(), W2.grad.numpy(), b2.grad.numpy(), w3.grad.numpy(),
                   float(b3.grad))
    assert np.allclose(mlp.backward(theta, X, y, F), ref, rtol=1e-10, atol=1e-12)
    assert np.isclose(mlp.loss(theta, X, y, F), float(L), rtol=1e-12)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    theta = mlp.init(F, 5)
    X, y = _batch(32, 3)
    opt = mlp.Adam(theta.size, lr=1e-2)
    p = torch.tensor(theta.copy(), requires_grad=True)
    topt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(5):
        g = mlp.backward(theta, X, y, F)
        theta = opt.step(theta, g)
        topt.zero_grad()
        p.grad = torch.tensor(mlp.backward(p.detach().numpy(), X, y, F))
        topt.step()
    assert np.allclose(theta, p.detach().numpy(), rtol=1e-10, atol=1e-12)


def test_features_are_set_functions():
    g = np.random.Generator(np.random.PCG64(7))
    d, m = 4, 3
    x = g.standard_normal((50, d)) @ np.diag([3.0, 2.0, 1.0, 0.5]) + 2.0
    n, s, S = 50, x.sum(0), x.T @ x
    f = learned.features(x, n, s, S, m)
    perm = g.permutation(50)
    xp = x[perm]
    fp = learned.features(xp, n, xp.sum(0), xp.T @ xp, m)
    assert np.allclose(fp, f[perm], rtol=1e-9, atol=1e-9)
    # whitened coordinates of the set's own points: mean 0, identity covariance
    U = f[:, :m]
    assert np.allclose(U.mean(0), 0, atol=1e-9)
    assert np.allclose(U.T @ U / n, np.eye(m), atol=1e-6)
    r = f[0, m:]
    assert np.all(np.diff(r) <= 0) and np.all(f[:, m:] == r)
    mu, P, _ = learned.set_frame(n, s, S, m)
    for j in range(m):
        v = P[j] / np.linalg.norm(P[j])
        assert v[np.argmax(np.abs(v))] > 0


def _tiny():
    x = np.array([[-1.2], [-0.9], [0.1], [1.5], [1.8]])
    model = sampler.Model("gaussian", 1.0, niw.NIWPrior(0.5, [0.0], 2.0, [[0.5]]), seed=11, burn_out=0)
    return x, model


def test_split_merge_detailed_balance_identity():
    x, model = _tiny()
    theta = mlp.init(2, 9)
    z = np.array([0, 0, 1, 1, 1])
    side = np.array([True, False, True])          # split cluster 1 = points 2, 3, 4
    lh_split = learned.split_log_h(model, x, z, 2, 1, theta, 1, side)
    z2 = z.copy(); z2[[2, 4]] = 2                 # side A (points 2 and 4) goes to the new cluster 2
    lh_merge = learned.merge_log_h(model, x, z2, 3, 1, 2, theta, 1)
    assert np.isclose(lh_split, -lh_merge, rtol=1e-12, atol=1e-12)
    z1 = np.zeros(5, dtype=int)
    side1 = np.array([True, True, False, False, True])
    a = learned.split_log_h(model, x, z1, 1, 0, theta, 1, side1)
    zz = np.where(side1, 1, 0)
    assert np.isclose(a, -learned.merge_log_h(model, x, zz, 2, 0, 1, theta, 1), rtol=1e-12)


@pytest.mark.slow
def test_learned_moves_alone_sample_the_exact_partition_posterior():
    x, model = _tiny()
    pr = model.prior
    lm = lambda rows: niw.log_marginal(pr, len(rows), x[rows].sum(0), x[rows].T @ x[rows])
    ex = partitions.exact_posterior(x, model.alpha, lm)
    theta = mlp.init(2, 13)
    st = sampler.State(1, np.zeros(5, dtype=np.int64), np.zeros(5, dtype=np.int64), np.zeros(1, dtype=np.int64))
    h = Counter()
    for t in range(1, 48001):
        st, info = learned.move(model, x, st, theta, 1, t)
        h[partitions.canonical(st.z)] += 1
    tv = partitions.total_variation(h, ex)
    print(f"learned-move chain: TV to exact posterior = {tv:.3f}")
    # Monte-Carlo error at this length is about 0.03 (0.021 at 96 000 moves)
    assert tv < 0.05
