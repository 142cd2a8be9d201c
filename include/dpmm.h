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
 *     N x V int32 counts (multinomial); z is int32[N] with clusters 0..K-1;
 *     zsub is uint8[N] with 0 = left (l), 1 = right (r) sub-cluster.
 *   - Streams: every call enqueues on the stream given to dpmm_create and
 *     returns; calls that must read device results back (dpmm_split_merge,
 *     dpmm_step, the dpmm_get_* calls) synchronise that stream.
 *   - Errors: every call returns a dpmm_status; nothing aborts and no C++
 *     exception crosses the ABI.  Argument and shape checks happen before any
 *     HIP call, so they can be exercised on a machine without a GPU.
 *     dpmm_last_error gives a message for the last failure on a context.
 *   - Random numbers: every draw is Philox4x32-10 (Salmon et al., SC'11) at
 *     counter (entity, t, tag, block) under key = seed (low word, high word).
 *     Tags: 0 cluster Gumbels of point i (block k/4, word k%4); 1 sub-label
 *     logistic of point i; 2 fresh sub-label bit of point i; 16 weight
 *     Gammas (entity k, the alpha slot entity K); 17 sub-weight Gammas
 *     (entity k, draw h); 18 NIW draws and 19 Dirichlet draws of component
 *     3k + c; 20 split uniform (entity k); 21 merge uniform (entity
 *     k1 << 16 | k2).  Draw q, attempt a of tags >= 16 uses block 256 q + a.
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

enum { DPMM_GAUSSIAN = 0, DPMM_MULTINOMIAL = 1 };
enum { DPMM_FP32 = 0, DPMM_BF16 = 1, DPMM_BF16X3 = 2 };
enum { DPMM_MERGE_PAPER = 0, DPMM_MERGE_INVERSE_SPLIT = 1 };

/* Model and capacity (Sec. 2.2 model; NIW prior of Sec. 2.2 Example;
 * Dirichlet prior for multinomial components, Sec. 2.1). */
typedef struct {
  int32_t family;     /* DPMM_GAUSSIAN or DPMM_MULTINOMIAL */
  int32_t d;          /* data dimension d (Gaussian) or vocabulary size V */
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
                         Gaussian with d = 32 or 64 only, else DPMM_E_ARG):
                         BF16 inputs with FP32 accumulation, X3 adding the
                         hi/lo cross terms; points whose BF16 top-2 gap leaves
                         any doubt are re-scored in FP32.  Sub-labels,
                         statistics and parameters are FP32/FP64 in every form */
  int32_t merge_form; /* DPMM_MERGE_PAPER: ratio of Sec. 4.1 eq. sample_merges;
                         DPMM_MERGE_INVERSE_SPLIT: H_merge = 1 / H_split of
                         Sec. 2.3 */
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
} dpmm_iter_info;

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
 *             covariance Sigma (d*d row-major SPD); multinomial P = V: log theta.
 * dpmm_set_params packs the float32 scoring tables on the device (Cholesky
 * of Sigma in float64, whitener W = L^-1, constant log w - 1/2 log|Sigma|
 * - d/2 log 2 pi); a covariance that is not positive definite gives
 * DPMM_E_NUMERIC.  dpmm_get_params returns the float64 parameters. */
dpmm_status dpmm_set_params(dpmm_ctx* ctx, int32_t K, const double* log_pi, const double* log_pisub,
                            const double* comp);
dpmm_status dpmm_get_params(dpmm_ctx* ctx, double* log_pi, double* log_pisub, double* comp);

/* Sufficient statistics per sub-cluster (Sec. 4.4 statistics update).
 * Gaussian: host double[K][2][1 + d + d*d] = (n, sum x, sum x x^T row-major).
 * Multinomial: host int64[K][2][1 + V] = (n, summed counts).
 * A cluster's statistics are the sum of its two sub-clusters'. */
dpmm_status dpmm_set_stats(dpmm_ctx* ctx, int32_t K, const void* stats);
dpmm_status dpmm_get_stats(dpmm_ctx* ctx, void* stats);

/* Weighted component log-likelihoods under the current packed parameters:
 * out device float[n][3K]: out[i][k] = log pi_k + log f(x_i; theta_k) for
 * k < K, out[i][K + 2k + h] = log pi-bar_kh + log f(x_i; theta-bar_kh).
 * Multinomial log-likelihoods omit the multinomial coefficient (the same for
 * every component).  Sec. 4.1 eqs. sample_labels / sample_sub_labels. */
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

/* Steps (a)-(d) of Sec. 4.1 from the context's statistics, in float64 on the
 * device: (pi_1..pi_K, rest) ~ Dir(N_1..N_K, alpha); (pi-bar_kl, pi-bar_kr) ~
 * Dir(N_kl + alpha/2, N_kr + alpha/2); component parameters from their
 * conjugate posteriors (NIW by Bartlett's construction; Dirichlet).  Then the
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

#ifdef __cplusplus
}
#endif

#endif /* DPMM_H */
