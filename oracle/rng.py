"""Random-number streams and transforms of the oracle (test-only, float64).

Every random quantity the sampler uses is a pure function of
(seed, iteration t, entity, tag, block): the Philox4x32-10 block with

    key     = (seed mod 2**32, seed >> 32)
    counter = (entity, t, tag, block)

so any draw can be recomputed in isolation, by either implementation, in any
order.  The paper draws from std::mt19937-style sequential generators
(Sec. 4.1 step (a)); a counter-based generator is used instead so that the
oracle and the GPU path see identical random numbers.

Tags (the entity named after each tag):
    0  TAG_GUMBEL     point i      cluster-label Gumbels: block k//4, word k%4
    1  TAG_LOGISTIC   point i      sub-label logistic with K a multiple of 4:
                                   block 0, word 0 (otherwise the logistic
                                   takes the first word of the last Gumbel
                                   block that no cluster uses: TAG_GUMBEL
                                   block K//4, word K%4; see sub_label_word)
    2  TAG_SUBINIT    point i      fresh random sub-label: block 0, word 0, bit 0
    3  TAG_BERN       point i      learned-proposal Bernoulli: block 0, word 0
    16 TAG_WEIGHTS    cluster k    Gamma draw for Dir(N_1..N_K, alpha); the
                                   alpha slot uses entity K
    17 TAG_SUBWEIGHTS cluster k    Gamma draws h = 0, 1 for the sub-weights
    18 TAG_NIW        3k + c       NIW draw of component c of cluster k
                                   (c = 0 cluster, 1 sub l, 2 sub r)
    19 TAG_DIRTHETA   3k + c       Dirichlet draw of a multinomial component
    20 TAG_SPLIT      cluster k    split acceptance uniform, word 0
    21 TAG_MERGE      (k1<<16)|k2  merge acceptance uniform, word 0
    22 TAG_MOVE       0            learned move selection, word 0 / 1
For tags >= 16 the draw with index q, attempt a uses block 256*q + a.

Transforms of one 32-bit word w:
    uniform  u = ((w >> 9) + 1/2) * 2**-23, in [2**-24, 1 - 2**-24], exactly
             representable in float32 and float64;
    Gumbel   g = -log(-log u), where -log u is taken as -log1p(u - 1) for
             u > 1/2 (u - 1 is exact), so g lies in [-2.8116, 16.6355];
    logistic L = log u - log1p(-u), |L| <= 16.6355.
Normal: Box-Muller on words (0, 1) of a block (Box & Muller 1958).
Gamma: Marsaglia & Tsang (2000) squeeze-free acceptance test on words 0-2 of
each attempt's block, with the u**(1/a) boost for shape a < 1 taken from
word 3 of the accepted block.  Draws are returned on the log scale so that
tiny shapes cannot underflow.
"""
import numpy as np

from .philox import philox4x32

TAG_GUMBEL = 0
TAG_LOGISTIC = 1
TAG_SUBINIT = 2
TAG_BERN = 3
TAG_WEIGHTS = 16
TAG_SUBWEIGHTS = 17
TAG_NIW = 18
TAG_DIRTHETA = 19
TAG_SPLIT = 20
TAG_MERGE = 21
TAG_MOVE = 22

ATTEMPT_STRIDE = 256
TWO_M23 = 2.0 ** -23


def key_of(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def block(seed, t, entity, tag, blk):
    """Philox block for (entity, t, tag, blk); arrays broadcast."""
    k0, k1 = key_of(seed)
    return philox4x32(entity, t, tag, blk, k0, k1)


def sub_label_word(seed, t, i, K):
    """The word of point i's sub-label logistic at step t with K clusters.  The
    Gumbels of clusters 0..K-1 take words 0..K-1 of blocks 0, 1, ... of
    TAG_GUMBEL; when K is not a multiple of 4 the last of those blocks has a
    word no cluster uses (K % 4), and the logistic takes it, so that a point
    that draws both labels computes one block fewer; otherwise it takes word 0
    of its own block (TAG_LOGISTIC)."""
    if K % 4:
        return block(seed, t, i, TAG_GUMBEL, K // 4)[K % 4]
    return block(seed, t, i, TAG_LOGISTIC, 0)[0]


def uniform(w):
    """Map uint32 words to float64 uniforms ((w >> 9) + 0.5) * 2**-23."""
    w = np.asarray(w, dtype=np.uint32)
    return ((w >> np.uint32(9)).astype(np.float64) + 0.5) * TWO_M23


def neglog_u(u):
    """-log(u) computed as -log1p(u - 1) on the upper half (exact argument)."""
    u = np.asarray(u, dtype=np.float64)
    return np.where(u > 0.5, -np.log1p(u - 1.0), -np.log(u))


def gumbel(w):
    return -np.log(neglog_u(uniform(w)))


def logistic(w):
    u = uniform(w)
    return np.log(u) - np.log1p(-u)


GUMBEL_MAX = float(-np.log(-np.log1p(-(2.0 ** -24))))
GUMBEL_MIN = float(-np.log(-np.log(2.0 ** -24)))
LOGISTIC_MAX = float(np.log1p(-(2.0 ** -24)) - np.log(2.0 ** -24))


def box_muller(w0, w1):
    u0 = uniform(w0)
    u1 = uniform(w1)
    return np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)


def normals(seed, t, entity, tag, q):
    """Standard normal draw number q of (entity, tag): one block per draw."""
    w = block(seed, t, entity, tag, np.asarray(q, dtype=np.uint64) * ATTEMPT_STRIDE)
    return box_muller(w[0], w[1])


def log_gamma_variates(seed, t, entity, tag, q, shape, max_attempts=ATTEMPT_STRIDE):
    """log of Gamma(shape, 1) draws, Marsaglia-Tsang with the shape<1 boost.

    entity, q and shape broadcast to a common 1-D shape; every element is an
    independent draw using blocks 256*q + attempt of its own (entity, tag).
    Attempt a is accepted when, with x = normal(words 0, 1), v = (1 + c x)^3,
    v > 0 and log(uniform(word 2)) < x^2/2 + d - d v + d log v, where
    d = a' - 1/3, c = 1 / sqrt(9 d) and a' = shape (or shape + 1 if shape < 1).
    The result is log(d v) (+ log(uniform(word 3)) / shape if shape < 1).
    If every attempt is rejected (probability below 0.05**256) log(d) is used.
    """
    entity, q, shape = np.broadcast_arrays(np.asarray(entity, dtype=np.uint64),
                                           np.asarray(q, dtype=np.uint64),
                                           np.asarray(shape, dtype=np.float64))
    entity = entity.ravel(); q = q.ravel(); shape = shape.ravel()
    if np.any(~(shape > 0)):
        raise ValueError("gamma shape must be > 0")
    boost = shape < 1.0
    a = np.where(boost, shape + 1.0, shape)
    d = a - 1.0 / 3.0
    c = 1.0 / np.sqrt(9.0 * d)
    out = np.log(d)
    done = np.zeros(shape.shape, dtype=bool)
    chunk = 4
    for a0 in range(0, max_attempts, chunk):
        todo = np.nonzero(~done)[0]
        if todo.size == 0:
            break
        att = np.arange(a0, min(a0 + chunk, max_attempts), dtype=np.uint64)
        blk = q[todo][:, None] * np.uint64(ATTEMPT_STRIDE) + att[None, :]
        w = block(seed, t, entity[todo][:, None], tag, blk)
        x = box_muller(w[0], w[1])
        dd = d[todo][:, None]
        v = 1.0 + c[todo][:, None] * x
        pos = v > 0
        v3 = np.where(pos, v, 1.0) ** 3
        with np.errstate(divide="ignore", invalid="ignore"):
            lhs = np.log(uniform(w[2]))
            rhs = 0.5 * x * x + dd - dd * v3 + dd * np.log(v3)
        acc = pos & (lhs < rhs)
        has = acc.any(axis=1)
        first = np.argmax(acc, axis=1)
        rows = np.nonzero(has)[0]
        sel = first[rows]
        idx = todo[rows]
        lg = np.log(d[idx]) + np.log(v3[rows, sel])
        bst = boost[idx]
        if np.any(bst):
            ub = uniform(w[3][rows, sel])
            lg = np.where(bst, lg + np.log(ub) / shape[idx], lg)
        out[idx] = lg
        done[idx] = True
    return out


def log_chi2_variates(seed, t, entity, tag, q, dof):
    """log of chi-square(dof) draws: chi2(k) = 2 Gamma(k/2)."""
    return np.log(2.0) + log_gamma_variates(seed, t, entity, tag, q, 0.5 * np.asarray(dof, dtype=np.float64))
