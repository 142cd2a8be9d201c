/*
 * dpmm.h -- C ABI of the MI355X (gfx950) DPMM sub-cluster sampler hot path.
 *
 * The sampler is the sub-cluster split/merge sampler of Chang & Fisher III as
 * described in Dinari, Zamir, Fisher III & Freifeld, "CPU- and GPU-based
 * Distributed Sampling in Dirichlet Process Mixtures for Large-scale
 * Analysis" (arXiv 2204.08988): Sec. 2.3 (augmented space, restricted Gibbs
 * sampler, split/merge framework) and Sec. 4.1 (steps (a)-(f), the split and
 * merge proposals).
 *
 * Conventions shared by every entry point
 *   - Ownership: the caller owns the data x and the labels z / zsub (device
 *     memory, e.g. torch tensors).  The context owns everything else (packed
 *     parameters, statistics, scratch) and frees it in dpmm_destroy.
 *   - Layout: x is point-major (row-major) N x d float32 (Gaussian) or
 *     N x V int32 counts (multinomial, Poisson); for a context created with
 *     sparse = 1, x is instead a host pointer to a dpmm_csr that describes
 *     the counts in compressed sparse rows; z is int32[N] with clusters 0..K-1;
 *     zsub is uint8[N] with 0 = left (l), 1 = right (r) sub-cluster.  Every
 *     call taking n accepts 0 <= n < 2^31 (device point indices are int32)
 *     and returns DPMM_E_SHAPE otherwise.
 *   - Streams: every call enqueues on the stream given to dpmm_create and
 *     returns; calls that must read device results back (dpmm_split_merge,
 *     dpmm_step, the dpmm_get_* calls) synchronise that stream.
 *   - Errors: every call returns a dpmm_status; nothing aborts and no C++
 *     exception crosses the ABI.  Argument and shape checks happen before any
 *     HIP call, so they can be exercised on a machine without a GPU.
 *     dpmm_last_error gives a message for the last failure on a context.
 *   - Random numbers: every draw is Philox4x32-10 (Salmon et al., SC'11) at
 *     counter (entity, t, tag, block) under key = seed (low word, high word).
 *     Tags: 0 cluster Gumbels of point i (block k/4, word k%4); the
 *     sub-label logistic of point i takes word K%4 of tag-0 block K/4 when
 *     K % 4 != 0, else word 0 of tag 1; 2 fresh sub-label bit of point i; 16 weight
 *     Gammas (entity k, the alpha slot entity K); 17 sub-weight Gammas
 *     (entity k, draw h); 18 NIW draws and 19 Dirichlet draws of component
 *     3k + c; 20 split uniform (entity k); 21 merge uniform (entity
 *     k1 << 16 | k2).  Draw q, attempt a of tags >= 16 uses block 256 q + a.
 *     The learned split proposal (an added form, not in the paper) uses tag
 *     3 (Bernoulli side of point i, word 0), 4 (fresh sub-label of point i
 *     after an accepted learned split, bit 0 of word 0), 5 (training batch
 *     row j, entity j, t = the training step counter), 22 (move selection:
 *     entity 0, words 0 type / 1 target / 2 acceptance) and 23 (initial
 *     weight q: entity q, t = 0).
 *     The same (seed, t) reproduces the same draws bit for bit.
 *   - Threading: one context per host thread; calls on one context are not
 *     re-entrant.
 */
#ifndef DPMM_H
#define DPMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dpmm_ctx dpmm_ctx;
typedef int32_t dpmm_status;

enum {
  DPMM_OK = 0,
  DPMM_E_ARG = -1,      /* null pointer or scalar argument out of range */
  DPMM_E_SHAPE = -2,    /* n or a buffer size inconsistent with the context */
  DPMM_E_CAPACITY = -3, /* the number of clusters would exceed k_max */
  DPMM_E_NUMERIC = -4,  /* non-finite value or matrix not positive definite */
  DPMM_E_DEVICE = -5,   /* HIP runtime error (no device, launch failure, ...) */
  DPMM_E_OOM = -6,      /* device allocation failed */
  DPMM_E_STATE = -7     /* call out of order (no parameters / statistics yet) */
};

enum { DPMM_GAUSSIAN = 0, DPMM_MULTINOMIAL = 1, DPMM_POISSON = 2 };
enum { DPMM_FP32 = 0, DPMM_BF16 = 1, DPMM_BF16X3 = 2 };
enum { DPMM_MERGE_PAPER = 0, DPMM_MERGE_INVERSE_SPLIT = 1 };

/* Count data in compressed sparse rows (contexts created with sparse = 1):
 * the shape of bag-of-words data with a large vocabulary, such as the
 * 20newsgroups documents of Sec. 5 (N = 11314, V = 20000).  The struct is
 * host memory read during the call; the three arrays are device memory owned
 * by the caller.  Row i is entries row_ptr[i] .. row_ptr[i+1] - 1 of col /
 * val: word col[e] in [0, V) with count val[e] >= 0; the columns of a row
 * need not be sorted, and a repeated column adds its counts.  row_ptr has
 * n + 1 entries, non-decreasing, within [0, nnz].  The kernels check every
 * entry: a row range outside [0, nnz], a column outside [0, V) or a negative
 * count is skipped (the row's labels stay as they were) and makes the next
 * call that synchronises (dpmm_split_merge, dpmm_step, the dpmm_get_* calls)
 * return DPMM_E_ARG. */
typedef struct {
  const int64_t* row_ptr; /* device [n + 1] */
  const int32_t* col;     /* device [nnz] */
  const int32_t* val;     /* device [nnz] */
  int64_t nnz;            /* number of stored entries, >= 0 */
} dpmm_csr;

/* Model and capacity (Sec. 2.2 model; NIW prior of Sec. 2.2 Example;
 * Dirichlet prior for multinomial components, Sec. 2.1).  DPMM_POISSON is a
 * further exponential family on the same template (Sec. 3.4 names Poisson as
 * the example of one): a component is a product of independent Poisson
 * counts with rates lambda_v ~ Gamma(gamma_shape_v, gamma_rate_v). */
typedef struct {
  int32_t family;     /* DPMM_GAUSSIAN, DPMM_MULTINOMIAL or DPMM_POISSON */
  int32_t d;          /* data dimension d (Gaussian, Poisson) or vocabulary
                         size V: 1 <= d <= 128 for dense data, 1 <= d <= 2^20
                         with sparse = 1 */
  int32_t k_max;      /* capacity in clusters, 1 <= k_max <= 4096 */
  int32_t burn_out;   /* a cluster younger than this many iterations may not
                         split or merge (>= 0) */
  double alpha;       /* DP concentration, > 0 */
  double kappa;       /* NIW kappa > 0 (Gaussian) */
  double nu;          /* NIW nu > d - 1 (Gaussian) */
  const double* m;    /* host [d]: NIW mean (Gaussian; copied) */
  const double* psi;  /* host [d*d]: NIW scale, row-major SPD (Gaussian; copied) */
  const double* beta; /* host [V]: Dirichlet prior, > 0 (multinomial; copied) */
  uint64_t seed;      /* Philox key */
  int32_t precision;  /* cluster scoring of the label step: DPMM_FP32 (vector
                         ALUs, any d); DPMM_BF16 or DPMM_BF16X3 (matrix cores,
                         Gaussian with d = 32, 64 or 128 only, else DPMM_E_ARG):
                         BF16 inputs with FP32 accumulation, X3 adding the
                         hi/lo cross terms; points whose BF16 top-2 gap leaves
                         any doubt are re-scored in FP32.  Sub-labels,
                         statistics and parameters are FP32/FP64 in every form */
  int32_t merge_form; /* DPMM_MERGE_PAPER: ratio of Sec. 4.1 eq. sample_merges;
                         DPMM_MERGE_INVERSE_SPLIT: H_merge = 1 / H_split of
                         Sec. 2.3 */
  int32_t learned;    /* learned split proposal (an added form; the paper has
                         none): 0 = off; m > 0 = number of principal axes of
                         the set features, 1 <= m <= min(d, 32), Gaussian
                         family only.  F = 2m network inputs.  When on,
                         dpmm_step makes one learned move after the split /
                         merge phase */
  const double* gamma_shape; /* host [d]: Gamma prior shapes, > 0 (Poisson; copied) */
  const double* gamma_rate;  /* host [d]: Gamma prior rates, > 0 (Poisson; copied) */
  int32_t sparse;     /* 0: dense x; 1: x is a dpmm_csr (multinomial and
                         Poisson families only) */
} dpmm_config;

/* What one iteration did (filled by dpmm_split_merge and dpmm_step). */
typedef struct {
  int32_t K;         /* clusters after the iteration */
  int32_t splits;    /* accepted splits */
  int32_t merges;    /* accepted merges */
  int32_t removed;   /* clusters deleted because they became empty */
  double logpost;    /* log p(z | x) up to a constant: K log alpha
                        + lgamma(alpha) - lgamma(alpha + N)
                        + sum_k [lgamma(N_k) + log f(C_k; lambda)] */
  /* device time of the phases of dpmm_step, milliseconds (HIP events on the
   * context's stream): */
  float ms_params;     /* parameter draws and packing */
  float ms_labels;     /* the label kernel: cluster draw (plus the sub-label
                          draw for d < 5 and the multinomial family) */
  float ms_sort;       /* counting sort by cluster (Gaussian d >= 5) */
  float ms_stats;      /* the statistics kernel (for d >= 5 also the
                          sub-label draw, over the sorted order) */
  float ms_splitmerge; /* split / merge phase */
  int32_t learned_kind;     /* learned move of dpmm_step: 0 none, 1 split, 2 merge */
  int32_t learned_accepted; /* 1 if it was accepted */
  float ms_learned;         /* its device-side time span, milliseconds */
  float ms_label_kernel;    /* the main cluster-draw kernel alone (Gaussian
                               matrix-core path: start and end events taken by
                               its own dispatch, without the candidate pass and
                               the FP32 re-score of deferred points); ms_labels
                               on the other paths */
} dpmm_iter_info;

/* What one learned move did (dpmm_learned_move). */
typedef struct {
  int32_t kind;       /* 1 split, 2 merge */
  int32_t k1, k2;     /* split: k1 = the cluster, k2 = -1; merge: k1 < k2 */
  int32_t accepted;   /* 1 if the labels were changed */
  int32_t skipped;    /* 0 the MH test decided; 1 a side of the split proposal
                         was empty; 2 a split would exceed k_max */
  int32_t reserved;
  int64_t n_a, n_b;   /* side sizes (split: Bernoulli sides; merge: k1, k2) */
  double log_target;  /* split orientation: log alpha + lgamma(n_a) + log f(A)
                         + lgamma(n_b) + log f(B) - lgamma(n_a + n_b) - log f(A u B) */
  double log_q_part;  /* log (q(s) + q(not s)): probability of the unordered
                         partition {A, B} under the per-point Bernoulli proposal */
  double log_h;       /* log Hastings ratio of the move made (split or merge) */
} dpmm_learned_info;

/* Create a context.  hip_stream: a hipStream_t (NULL = default stream).
 * Allocates the device tables for k_max clusters.  On failure *out is NULL. */
dpmm_status dpmm_create(const dpmm_config* cfg, void* hip_stream, dpmm_ctx** out);
void dpmm_destroy(dpmm_ctx* ctx);
const char* dpmm_last_error(const dpmm_ctx* ctx);
const char* dpmm_status_string(dpmm_status s);

/* Initial state (one cluster): z[i] = 0, zsub[i] = bit 0 of Philox word 0 at
 * (entity i, t = 0, tag 2, block 0); K = 1, age 0.  z, zsub: device, [n]. */
dpmm_status dpmm_init_labels(dpmm_ctx* ctx, int64_t n, int32_t* z, uint8_t* zsub);

/* Cluster count and ages.  age: host int32[K] (may be NULL in get to skip). */
dpmm_status dpmm_set_state(dpmm_ctx* ctx, int32_t K, const int32_t* age);
dpmm_status dpmm_get_state(dpmm_ctx* ctx, int32_t* K, int32_t* age);

/* Parameters of K clusters and their 2K sub-clusters (Sec. 4.1 steps (a)-(d)).
 *   log_pi    host double[K]       log cluster weights
 *   log_pisub host double[K][2]    log sub-cluster weights (l, r)
 *   comp      host double[K][3][P] component c = 0 (cluster), 1 (sub l),
 *             2 (sub r) of cluster k; Gaussian P = d + d*d: mean (d) then
 *             covariance Sigma (d*d row-major SPD); multinomial P = V: log theta;
 *             Poisson P = d: log lambda (log rates).
 * dpmm_set_params packs the float32 scoring tables on the device (Cholesky
 * of Sigma in float64, whitener W = L^-1, constant log w - 1/2 log|Sigma|
 * - d/2 log 2 pi); a covariance that is not positive definite gives
 * DPMM_E_NUMERIC.  dpmm_get_params returns the float64 parameters. */
dpmm_status dpmm_set_params(dpmm_ctx* ctx, int32_t K, const double* log_pi, const double* log_pisub,
                            const double* comp);
dpmm_status dpmm_get_params(dpmm_ctx* ctx, double* log_pi, double* log_pisub, double* comp);

/* Sufficient statistics per sub-cluster (Sec. 4.4 statistics update).
 * Gaussian: host double[K][2][1 + d + d*d] = (n, sum x, sum x x^T row-major).
 * Multinomial and Poisson: host int64[K][2][1 + V] = (n, summed counts).
 * A cluster's statistics are the sum of its two sub-clusters'. */
dpmm_status dpmm_set_stats(dpmm_ctx* ctx, int32_t K, const void* stats);
dpmm_status dpmm_get_stats(dpmm_ctx* ctx, void* stats);

/* Weighted component log-likelihoods under the current packed parameters:
 * out device float[n][3K]: out[i][k] = log pi_k + log f(x_i; theta_k) for
 * k < K, out[i][K + 2k + h] = log pi-bar_kh + log f(x_i; theta-bar_kh).
 * Multinomial log-likelihoods omit the multinomial coefficient and Poisson
 * ones the factor prod 1 / x_v! (the same for every component).  Sec. 4.1
 * eqs. sample_labels / sample_sub_labels. */
dpmm_status dpmm_loglik(dpmm_ctx* ctx, const void* x, int64_t n, float* out);

/* Steps (e) and (f) of Sec. 4.1: z_i = argmax_k (log pi_k + log f(x_i; theta_k)
 * + Gumbel(i, t, k)) and zsub_i = l iff the sub-cluster score gap plus a
 * Logistic(i, t) draw is positive (eqs. sample_labels, sample_sub_labels). */
dpmm_status dpmm_sample_labels(dpmm_ctx* ctx, const void* x, int64_t n, uint32_t t, int32_t* z,
                               uint8_t* zsub);

/* Recompute the context's sufficient statistics from (x, z, zsub) with the
 * current K; labels must lie in [0, K) and {0, 1}. */
dpmm_status dpmm_suffstats(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z,
                           const uint8_t* zsub);

/* dpmm_suffstats without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid it).  The same kernels and the same results as dpmm_suffstats
 * (bit for bit), but their scratch (sort tables, permutation, partial sums)
 * comes from a static device array of DPMM_STATIC_SCRATCH_MIB MiB that each
 * GPU holds for the life of the process.  A call needs, at the context's
 * current K: nothing for the multinomial family; 8 (2 K (2 + d + d(d+1)/2))
 * 65536 / L bytes (L = 256, 128 or 64 lanes, the most whose accumulators fit
 * in LDS) for the Gaussian family with d <= 4; else about 8 n bytes for the
 * sort plus the partial sums (2 ranges x 2 (1 + d + d(d+1)/2) doubles, at
 * most 2048 ranges).  A call that needs more than the array returns
 * DPMM_E_CAPACITY (its message gives the size) before touching the device.
 * All calls on one GPU share the array: calls that overlap on one GPU race. */
#define DPMM_STATIC_SCRATCH_MIB 128
dpmm_status dpmm_suffstats_static(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z,
                                  const uint8_t* zsub);

/* Steps (a)-(d) of Sec. 4.1 from the context's statistics, in float64 on the
 * device: (pi_1..pi_K, rest) ~ Dir(N_1..N_K, alpha); (pi-bar_kl, pi-bar_kr) ~
 * Dir(N_kl + alpha/2, N_kr + alpha/2); component parameters from their
 * conjugate posteriors (NIW by Bartlett's construction; Dirichlet; Gamma
 * rates Gamma(a_v + c_v, b_v + n)).  Then the
 * float32 scoring tables are packed.  Every cluster must be non-empty
 * (DPMM_E_STATE otherwise). */
dpmm_status dpmm_sample_params(dpmm_ctx* ctx, uint32_t t);

/* Delete empty clusters (stable), propose a split of every eligible cluster
 * (Sec. 2.3 eq. HastingsRatioSplit / Sec. 4.1 eq. sample_splits) and a merge
 * of every eligible pair in lexicographic order (Sec. 4.1 eq. sample_merges,
 * no cluster in two moves, Sec. 4.3), relabel z / zsub on the device,
 * recompute the statistics and report the log posterior.  info: host, may be
 * NULL. */
dpmm_status dpmm_split_merge(dpmm_ctx* ctx, const void* x, int64_t n, uint32_t t, int32_t* z,
                             uint8_t* zsub, dpmm_iter_info* info);

/* One full iteration t >= 1: dpmm_sample_params, dpmm_sample_labels,
 * statistics, dpmm_split_merge, then every cluster's age grows by one. */
dpmm_status dpmm_step(dpmm_ctx* ctx, const void* x, int64_t n, uint32_t t, int32_t* z, uint8_t* zsub,
                      dpmm_iter_info* info);

/* ---- Learned split proposal (an added form; the paper has no learned
 * component).  A network F -> 128 -> 128 -> 1 (ReLU hidden layers) maps the
 * set features of a point to the logit of its probability b of going to side
 * A of a proposed 2-way partition of the set; b = clip(sigmoid(logit), 1e-6,
 * 1 - 1e-6).  Forward and backward products run on the matrix cores in BF16
 * with FP32 accumulation; the master weights and Adam state are FP32.
 * Parameter vector layout (n_params = F*128 + 128 + 128*128 + 128 + 128 + 1):
 * W1[F][128], b1[128], W2[128][128], b2[128], w3[128], b3, layer k computing
 * a_k = a_(k-1) W_k + b_k.  Every call below needs cfg.learned > 0
 * (DPMM_E_STATE otherwise). */

/* Number of network parameters (0 when the learned proposal is off). */
int64_t dpmm_mlp_n_params(const dpmm_ctx* ctx);

/* Replace (set) or read (get) the FP32 master weights: host double[n_params].
 * Setting also resets the Adam state.  dpmm_create initialises the weights
 * He-uniform: W1, W2, w3 entries (2u - 1) sqrt(6 / fan_in) with u the uniform
 * of Philox word 0 at (entity q, t = 0, tag 23), q = the parameter's index in
 * the vector; biases 0. */
dpmm_status dpmm_mlp_set_weights(dpmm_ctx* ctx, const double* params);
dpmm_status dpmm_mlp_get_weights(dpmm_ctx* ctx, double* params);

/* Logits of n feature rows.  X: device float[n][F] (rounded to BF16 on the
 * way in); logits: device float[n]. */
dpmm_status dpmm_mlp_forward(dpmm_ctx* ctx, const float* X, int64_t n, float* logits);

/* Gradient of the summed binary cross-entropy
 *   L = sum_i [softplus(o_i) - y_i o_i]
 * with respect to the parameter vector.  X: device float[n][F]; y: device
 * float[n] in [0, 1]; grad: host double[n_params] (may be NULL); loss: host
 * (may be NULL).  dpmm_mlp_adam_step then applies one Adam step (Kingma & Ba,
 * betas 0.9 / 0.999, eps 1e-8, bias-corrected) with that gradient. */
dpmm_status dpmm_mlp_grad(dpmm_ctx* ctx, const float* X, const float* y, int64_t n, double* grad, double* loss);
dpmm_status dpmm_mlp_adam_step(dpmm_ctx* ctx, const float* X, const float* y, int64_t n, float lr, double* loss);

/* Set features of the points of cluster k1 (k2 < 0) or of the union of
 * clusters k1 and k2, from the context's statistics: mean mu and covariance
 * Sigma (plus 1e-9 (1 + tr Sigma / d) I) of the set, eigenvalues in
 * decreasing order, each eigenvector's largest-magnitude entry positive;
 * features of point x: v_j^T (x - mu) / sqrt(lambda_j) and lambda_j / sum
 * lambda for j < m.  Points in increasing index order.  feats: device
 * float[n_set][F]; idx: device int32[n_set]; n_set: host.  feats / idx may be
 * NULL to ask for n_set only; capacity: rows the buffers hold
 * (DPMM_E_SHAPE if fewer than n_set). */
dpmm_status dpmm_set_features(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, int32_t k1, int32_t k2,
                              float* feats, int32_t* idx, int64_t capacity, int64_t* n_set);

/* One learned Metropolis-Hastings move in the collapsed space of partitions
 * (Hastings 1970; Jain & Neal 2004): split with probability 1 if K = 1 else
 * 1/2, of the cluster floor(u K); else merge of the floor(u K(K-1)/2)-th pair
 * in lexicographic order.  Split proposal: point i of the cluster goes to
 * side A iff uniform(i, t, tag 3) < b_i; merge: A = k1, B = k2.  Target:
 * alpha^K prod_B Gamma(|B|) f(x_B) (f: the NIW marginal likelihood).  The
 * reverse move's probability uses the same per-point network on the merged
 * set, so the move leaves the posterior invariant for any weights.  An
 * accepted split appends cluster K (side A) with age 0, resets cluster k1's
 * age and draws fresh sub-labels (tag 4) for its points; an accepted merge
 * moves k2 into k1 (sub-labels l = old k1, r = old k2), deletes k2 (stable)
 * and resets k1's age.  The statistics are then recomputed.  Needs current
 * statistics and non-empty clusters.  side_out: optional device uint8[n]
 * receiving 1 (side A) / 0 for the points of the set; info: host, optional. */
dpmm_status dpmm_learned_move(dpmm_ctx* ctx, const void* x, int64_t n, uint32_t t, int32_t* z, uint8_t* zsub,
                              uint8_t* side_out, dpmm_learned_info* info);

/* Train the network on the sampler's own sub-labels: rows are the points of
 * clusters with age >= burn_out and two non-empty sub-clusters, target 1 for
 * sub-label l, flipped per cluster so that side l has the larger mean first
 * principal coordinate.  Each of `steps` Adam steps draws `batch` rows
 * uniformly with replacement (tag 5).  loss: host, the mean loss of the last
 * step (may be NULL).  Returns DPMM_OK without a step when no cluster
 * qualifies (loss = NaN). */
dpmm_status dpmm_mlp_train(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, const uint8_t* zsub,
                           int32_t steps, int32_t batch, float lr, double* loss);

/* The rows dpmm_mlp_train draws its batches from, all of them: the points of
 * every cluster with age >= burn_out and two non-empty sub-clusters, in
 * increasing index order; feats device float[n_rows][F] their set features
 * under their own cluster's frame, y device float[n_rows] their targets (1
 * for sub-label l, flipped per cluster so that side l has the larger mean
 * first principal coordinate), idx device int32[n_rows] their point
 * indices.  Each output may be NULL (all NULL: count only); capacity is the
 * rows each non-NULL output holds (DPMM_E_SHAPE if below n_rows).  n_rows:
 * host.  Needs current statistics (DPMM_E_STATE otherwise). */
dpmm_status dpmm_mlp_training_set(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, const uint8_t* zsub,
                                  float* feats, float* y, int32_t* idx, int64_t capacity, int64_t* n_rows);

/* ---- User-level run (the paper's fit interface, Sec. 3.4) ---- */

/* Normalised mutual information of two labelings a, b (host int32[n]) with
 * the arithmetic-mean normalisation I(a; b) / ((H(a) + H(b)) / 2), the
 * accuracy measure of Sec. 5; 1 when both are constant.  Host code: needs no
 * context and no device. */
dpmm_status dpmm_nmi(const int32_t* a, const int32_t* b, int64_t n, double* out);

/* Options of dpmm_fit. */
typedef struct {
  uint32_t t0;         /* the first iteration's number (>= 1); a run resumed
                          from a checkpoint of iteration t passes t + 1 */
  int32_t iters;       /* iterations to run (>= 0) */
  int32_t train_every; /* learned proposal: train the network on the sampler's
                          sub-labels after every iteration t with
                          t % train_every == 0 and t <= train_until (0: never) */
  int32_t train_until;
  int32_t train_steps; /* dpmm_mlp_train arguments */
  int32_t train_batch;
  float train_lr;
  int32_t reserved;
} dpmm_fit_options;

/* Run iterations t0 ... t0 + iters - 1 of the sampler (dpmm_step each, plus
 * the training schedule of opt), the user-level run of Sec. 3.4 (a fixed
 * iteration count, the state in z / zsub).  trace: host dpmm_iter_info[iters]
 * (optional), seconds: host double[iters] wall-clock time of each iteration
 * (optional).  Stops at the first failing iteration and returns its status. */
dpmm_status dpmm_fit(dpmm_ctx* ctx, const void* x, int64_t n, const dpmm_fit_options* opt, int32_t* z, uint8_t* zsub,
                     dpmm_iter_info* trace, double* seconds);

/* Checkpoint files (the save-model option of Sec. 3.4): the state after
 * iteration t -- K, the cluster ages, z and zsub (device int32[n] / uint8[n]),
 * and with the learned proposal the network's weights, Adam moments and
 * counters -- with the configuration it was written under.  Every draw of a
 * later iteration is a function of (seed, iteration, entity) and of this
 * state, so a run resumed from a checkpoint of iteration t at t + 1 repeats
 * the uninterrupted run bit for bit.  The file is written to path + ".tmp"
 * and renamed.  Loading checks the configuration (family, d, seed, alpha,
 * prior, forms) and n against the context (DPMM_E_ARG / DPMM_E_SHAPE
 * otherwise), writes z / zsub, sets K and the ages (as dpmm_set_state) and
 * returns t. */
dpmm_status dpmm_save_checkpoint(dpmm_ctx* ctx, const char* path, int64_t n, uint32_t t, const int32_t* z,
                                 const uint8_t* zsub);
dpmm_status dpmm_load_checkpoint(dpmm_ctx* ctx, const char* path, int64_t n, uint32_t* t, int32_t* z,
                                 uint8_t* zsub);

#ifdef __cplusplus
}
#endif

#endif /* DPMM_H */
