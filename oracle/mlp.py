"""Float64 MLP of the learned split proposal (test-only).

The paper has no learned component; this is the added form.  A network
F -> 128 -> 128 -> 1 with ReLU hidden layers maps a point's set-relative
features to the logit of its probability of going to side A of a proposed
2-way partition.  Training minimises the binary cross-entropy
    L = sum_i [softplus(o_i) - y_i o_i]
(the logistic log-loss written with the logit o_i) with Adam (Kingma & Ba 2015).

Parameter vector layout (float, in this order):
    W1[F][H], b1[H], W2[H][H], b2[H], w3[H], b3[1]      (H = 128)
with layer k computing a_k = a_{k-1} W_k + b_k.
"""
import numpy as np

HIDDEN = 128


def n_params(F, H=HIDDEN):
    return F * H + H + H * H + H + H + 1


def unpack(theta, F, H=HIDDEN):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + F * H].reshape(F, H); o += F * H
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def init(F, seed, H=HIDDEN):
    """He-uniform initial weights from numpy's PCG64(seed); biases zero."""
    g = np.random.Generator(np.random.PCG64(seed))
    W1 = g.uniform(-1, 1, size=(F, H)) * np.sqrt(6.0 / F)
    W2 = g.uniform(-1, 1, size=(H, H)) * np.sqrt(6.0 / H)
    w3 = g.uniform(-1, 1, size=H) * np.sqrt(6.0 / H)
    return pack(W1, np.zeros(H), W2, np.zeros(H), w3, 0.0)


def forward(theta, X, F):
    """Logits o[n] and the activations needed by `backward`."""
    W1, b1, W2, b2, w3, b3 = unpack(theta, F)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1 + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2 + b2
    a2 = np.maximum(z2, 0.0)
    o = a2 @ w3 + b3
    return o, (X, z1, a1, z2, a2)


def softplus(o):
    return np.logaddexp(0.0, o)


def loss(theta, X, y, F):
    o, _ = forward(theta, X, F)
    return float(np.sum(softplus(o) - np.asarray(y, dtype=np.float64) * o))


def backward(theta, X, y, F):
    """Gradient of `loss` with respect to the parameter vector (same layout)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta, F)
    o, (X, z1, a1, z2, a2) = forward(theta, X, F)
    y = np.asarray(y, dtype=np.float64)
    d_o = 1.0 / (1.0 + np.exp(-o)) - y           # dL/do
    gw3 = a2.T @ d_o
    gb3 = np.sum(d_o)
    d2 = np.outer(d_o, w3) * (z2 > 0)            # dL/dz2
    gW2 = a1.T @ d2
    gb2 = d2.sum(0)
    d1 = (d2 @ W2.T) * (z1 > 0)                  # dL/dz1
    gW1 = X.T @ d1
    gb1 = d1.sum(0)
    return pack(gW1, gb1, gW2, gb2, gw3, gb3)


class Adam:
    """Adam with bias correction on the flat parameter vector."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, grad):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad
        self.v = self.b2 * self.v + (1 - self.b2) * grad * grad
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)
