// Kernel declarations of the DPMM HIP library (gfx950).
#pragma once
#include "common.hpp"

namespace dpmm {

#define NIW_SCRATCH(d) ((size_t)3 * (d) * (d) + (d))
// float64 workspaces of the per-component kernels live in LDS up to this d
// candidate clusters kept per point by the matrix-core label kernels
constexpr int RESCORE_CAND = 8;
// candidate pass over few deferred points (d = 64, 128): the clusters split over
// CAND_SPLIT_NG workgroups per point chunk, their lists merged per point; used
// while at most CAND_SPLIT_CAP points are deferred.  CAND_STATE: floats of one
// list (bounds, squared norms, clusters, lo_max, ev_max)
constexpr int CAND_SPLIT_NG = 8;
constexpr int CAND_SPLIT_CAP = 32768;
constexpr int CAND_STATE = 3 * RESCORE_CAND + 2;
constexpr int NIW_LDS_MAX_D = 64;
// above that and up to this d the draw keeps one d x (d + 1) float64 matrix in LDS
constexpr int NIW_BIG_MAX_D = 128;
inline size_t niw_lds_bytes(int d) { return d <= NIW_LDS_MAX_D ? NIW_SCRATCH(d) * sizeof(double) : 0; }
// the marginal-likelihood kernel keeps one d x d matrix in LDS up to this d
constexpr int LOGML_LDS_MAX_D = 128;

struct NiwPriorDev {
  double kappa, nu;
  const double* m;    // device [d]
  const double* psi;  // device [d*d]
};

// ---- parameters (params.hip)
__global__ void k_weights(int K, double alpha, const long long* counts, uint64_t seed, uint32_t t,
                          double* log_pi, double* log_pisub, double* tmp);
__global__ void k_niw_draw(int K, int d, int k_max, NiwPriorDev prior, const long long* counts,
                           const double* moments, const double* log_pi, const double* log_pisub,
                           uint64_t seed, uint32_t t, double* mu_out, double* sigma_out, double* scratch,
                           float* packed, double* logdet_out, int* err);
// k_niw_draw, with one wave per component for d <= 64
hipError_t launch_niw_draw(int K, int d, int k_max, NiwPriorDev prior, const long long* counts,
                           const double* moments, const double* log_pi, const double* log_pisub, uint64_t seed,
                           uint32_t t, double* mu_out, double* sigma_out, double* scratch, float* packed,
                           double* logdet_out, int* err, hipStream_t s);
__global__ void k_dir_draw(int K, int V, const double* beta, const long long* sums, uint64_t seed,
                           uint32_t t, double* log_theta);
__global__ void k_pack_gauss(int K, int d, int k_max, const double* log_pi, const double* log_pisub,
                             const double* mu, const double* sigma, double* scratch, float* packed,
                             double* logdet_out, int* err);
__global__ void k_pack_mult(int K, int V, int k_max, const double* log_pi, const double* log_pisub,
                            const double* log_theta, float* packed, int poisson);
__global__ void k_pois_draw(int K, int V, const double* shape, const double* rate, const long long* counts,
                            const long long* sums, uint64_t seed, uint32_t t, double* log_lambda);
// the Dirichlet draw over word chunks (vocabularies above DIR_CHUNK words)
constexpr int DIR_CHUNK = 2048;
__global__ void k_dir_draw_chunk(int K, int V, const double* beta, const long long* sums, uint64_t seed, uint32_t t,
                                 double* log_theta, double* part);
__global__ void k_dir_norm(int K, int V, const double* part, double* log_theta);

// ---- learned split proposal (mlp.hip)
constexpr int MLP_HIDDEN = 128;
constexpr float MLP_CLIP = 1e-6f;
constexpr int MLP_CHUNK = 65536;      // rows per forward / backward pass
constexpr int SELECT_BLOCKS = 1024;   // blocks of the stable selection
constexpr int SET_STATS_BLOCKS = 128; // blocks of the partition statistics
constexpr uint32_t TAG_LEARNSUB = 4;
constexpr uint32_t TAG_TRAIN = 5;
constexpr uint32_t TAG_MLPINIT = 23;
hipError_t launch_gemm_nt(const void* A, int lda, const void* Bt, int ldb, int M, int N, int K, const float* bias,
                          bool relu, const void* mask, int ldm, float* out32, int ld32, bool accumulate, void* out16,
                          int ld16, void* out16t, int ld16t, hipStream_t s);
hipError_t launch_out_layer(const float* H2, int n, const float* w3, const float* b3, float* o, hipStream_t s);
// red: float64 row buffers of the fixed-order reductions below, MLP_RED_DOUBLES
constexpr size_t MLP_RED_DOUBLES = (size_t)1024 * (MLP_HIDDEN + 2);
// gw3, gb3 adjacent (gb3 = gw3 + 128); adds the block sums in block order
hipError_t launch_out_backward(const float* o, const float* y, const float* H2, int n, int npad, const float* w3,
                               void* D2, void* D2t, float* gw3, float* gb3, double* loss, double* red, hipStream_t s);
hipError_t launch_colsum(const void* A, int lda, int n, int ncol, float* out, double* red, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);
hipError_t launch_refresh_weights(const float* p, int F, int Fp, void* w1t, void* w2t, void* w2, hipStream_t s);
// rows whose idx is outside [0, npts) are zero / skipped by the set kernels;
// the frame (and flip) of row q is cl[q], or cl[idx[q]] with cl_by_point
// (cl = z: the row's own cluster), or 0 without cl
hipError_t launch_features(const float* x, int d, long long npts, const int* idx, const int* cl, int n,
                           const float* frames, int m, int F, int Fp, void* X16, void* X16t, int npad, float* X32,
                           hipStream_t s, bool cl_by_point = false);
hipError_t launch_convert(const float* X32, int n, int F, int Fp, void* X16, void* X16t, int npad, hipStream_t s);
hipError_t launch_targets(const int* idx, const int* cl, int n, const unsigned char* zsub, const int* flip, float* y,
                          hipStream_t s, bool cl_by_point = false);
hipError_t launch_proposal(const float* o, long long npts, const int* idx, int n, int merge_k1, const int* z,
                           uint64_t seed, uint32_t t, unsigned char* side, double* sums, double* red, hipStream_t s);
hipError_t launch_apply_split(long long npts, const int* idx, int n, const unsigned char* side, int k_new,
                              uint64_t seed, uint32_t t, int* z, unsigned char* zsub, hipStream_t s);
// stable selection of {i : z_i in {k1, k2}} (elig == nullptr) or {i : elig[z_i]};
// cnt: int[SELECT_BLOCKS + 1], the count lands in cnt[SELECT_BLOCKS]
hipError_t launch_select(const int* z, long long n, int k1, int k2, const int* elig, int K, int* cnt, int* out,
                         hipStream_t s);
// float64 statistics of the sides (side[i] = 1: A, 0: B) of the points idx[0..n)
// into counts / moments slots slot (A) and slot + 1 (B); part: double
// [SET_STATS_BLOCKS][2][1 + d + d(d+1)/2]
hipError_t launch_set_stats(const float* x, int d, long long npts, const int* idx, int n, const unsigned char* side,
                            double* part, int slot, long long* counts, double* moments, hipStream_t s);
hipError_t launch_batch_pick(const int* sel, long long n_sel, int batch, uint64_t seed, uint32_t counter, const int* z,
                             int* bidx, int* bcl, hipStream_t s);

// ---- host launchers of the templated hot kernels
hipError_t launch_label_gauss(int d, const float* x, long long n, const float* packed, int K, int k_max,
                              uint32_t t, uint64_t seed, int* z, unsigned char* zsub, hipStream_t s);
// cluster-sorted path (d >= 5): z + per-block histogram, sort by z, sub-labels
// and statistics over sorted tiles
constexpr int SORTED_MIN_D = 5;
hipError_t launch_label_gauss_z(int d, const float* x, long long n, int G, long long per_block, const float* packed,
                                int K, uint32_t t, uint64_t seed, int* z, int* hist, int* tot, hipStream_t s);
hipError_t sorted_plan(long long n, int K, long long hist_cap, int* G, long long* per_block);
hipError_t launch_sort_by_z(const int* z, long long n, int K, int G, long long per_block, bool have_hist, int* hist,
                            int* tot, int* offs, int* perm, int* zsort, hipStream_t s);
// waves of the d <= 32 statistics kernel.  In slot mode (cstart = the
// clusters' first sorted rows, ctot their sizes, part =
// sub_stats_part_doubles(d, n) doubles) every cluster's statistics are
// written, with no float atomics: the sums are taken in a fixed order
constexpr int SUBW_WAVES = 2048;
size_t sub_stats_part_doubles(int d, long long n);
size_t sub_stats_part_doubles_max(int d);  // over every n
struct SubX3;
// x3 (may be null; d = 64, 128 with sample): the bf16x3 sub-label pass and its buffers
hipError_t launch_sub_stats(int d, bool sample, const float* x, long long n, const int* perm, const int* z,
                            const int* zrow, unsigned char* zsub, const float* packed, int K, int k_max, uint32_t t,
                            uint64_t seed, long long* counts, double* moments, const int* cstart, const int* ctot,
                            double* part, hipStream_t s, const SubX3* x3 = nullptr);
// statistics of a listed set of cluster k1's points split by side[i] into
// segments slot, slot + 1 (slot >= 2 k1; d in {8, 16, 32, 64, 128});
// cspan: device int[2] = {0, nsel}; part: sub_stats_part_doubles(d, nsel)
bool partition_stats_supported(int d);
hipError_t launch_partition_stats(int d, const float* x, long long npts, const int* idx, long long nsel,
                                  const int* z, int k1, int K, const unsigned char* side, int slot,
                                  long long* counts, double* moments, const int* cspan, double* part, hipStream_t s);
// BF16 matrix-core cluster draw (d in {32, 64}) and its whitener fragments
bool mfma_supported(int d);
// wbias (d = 64, 128; may be null): [k_max][d] offsets beta = -W (mu - c) in the
// accumulator layout, [k_max][4] constants, [d] the common centre c, for the
// uncentred BF16 main pass; wbias_floats(d, k_max) floats (0 for other d)
size_t wbias_floats(int d, int k_max);
// shi, slo (may be null): the same fragment tables for the 2K sub-clusters
hipError_t launch_pack_wfrag(int K, int d, int k_max, const float* packed, void* whi, void* wlo, float* wbias,
                             void* shi, void* slo, hipStream_t s);
// bf16x3 sub-label pass over cluster-sorted rows (d = 64, 128) in front of the
// FP32 one: the rows it cannot decide are listed, in sorted order, in
// perm_c / zrow_c, their number in offs[SUBX_GROUPS]
constexpr int SUBX_GROUPS = 1024;
struct SubX3 {
  const void* hi;       // [2 k_max][d / 32][d / 16][64][8] BF16 fragments of the sub-cluster whiteners
  const void* lo;       // their low parts
  unsigned char* flag;  // [n] per sorted row
  int* cnt;             // [SUBX_GROUPS]
  int* offs;            // [SUBX_GROUPS + 1]
  int* perm_c;          // [n]
  int* zrow_c;          // [n]
};
hipError_t launch_sub_labels_x3(int d, const float* x, long long n, const int* perm, const int* z, const int* zrow,
                                unsigned char* zsub, const float* packed, int K, int k_max, uint32_t t, uint64_t seed,
                                const SubX3& b, hipStream_t s);
// flagged: int[n] (the points whose draw is deferred to FP32); cand:
// int[n][RESCORE_CAND], each deferred point's candidate clusters (-1: empty
// slot, -2 in slot 0: all clusters); n_flagged: one device int
hipError_t launch_label_gauss_mfma(int d, bool x3, const float* x, long long n, int G, long long per_block,
                                   const float* packed, const void* whi, const void* wlo, const float* wbias, int K,
                                   int k_max, uint32_t t, uint64_t seed, int* z, int* hist, int* tot, int* flagged,
                                   int* cand, int* n_flagged, hipStream_t s, hipEvent_t ev_main0 = nullptr,
                                   hipEvent_t ev_main1 = nullptr, float* cst = nullptr);
hipError_t launch_loglik_gauss(int d, const float* x, long long n, const float* packed, int K, int k_max,
                               float* out, hipStream_t s);
// ---- count data in compressed sparse rows (label_csr.hip)
// bit of the device error flag: an entry of the sparse rows was out of range
constexpr int ERR_SPARSE_INPUT = 8;
struct SparseRows {
  const long long* row_ptr;  // device [n + 1]
  const int* col;            // device [nnz]
  const int* val;            // device [nnz]
  long long nnz;
};
hipError_t launch_pack_csr(int K, int V, int k_max, const float* packed, float* tcl, float* tsub, float* cw,
                           hipStream_t s);
hipError_t launch_label_csr(const SparseRows& x, long long n, int V, const float* tcl, const float* tsub,
                            const float* cw, int K, uint32_t t, uint64_t seed, int* z, unsigned char* zsub, int* err,
                            hipStream_t s);
hipError_t launch_loglik_csr(const SparseRows& x, long long n, int V, const float* tcl, const float* tsub,
                             const float* cw, int K, float* out, int* err, hipStream_t s);
hipError_t launch_stats_csr(const SparseRows& x, long long n, int V, const int* z, const unsigned char* zsub, int K,
                            long long* counts, long long* sums, int* err, hipStream_t s);

hipError_t launch_label_mult(int V, const int* x, long long n, const float* packed, int K, int k_max,
                             uint32_t t, uint64_t seed, int* z, unsigned char* zsub, hipStream_t s);
hipError_t launch_loglik_mult(int V, const int* x, long long n, const float* packed, int K, int k_max,
                              float* out, hipStream_t s);
// Gaussian statistics for d <= 4 (when stats_small_lanes(d, K) > 0): part
// holds stats_small_part_doubles(d, K) doubles of per-workgroup rows
constexpr int STATS_SMALL_LANES = 65536;
int stats_small_lanes(int d, int K);
size_t stats_small_part_doubles(int d, int K);
hipError_t launch_stats_gauss(int d, const float* x, long long n, const int* z, const unsigned char* zsub,
                              int K, long long* counts, double* moments, double* part, hipStream_t s);
// device p[0] = a, p[1] = b
hipError_t launch_set_pair(int* p, int a, int b, hipStream_t s);
hipError_t launch_stats_mult(int V, const int* x, long long n, const int* z, const unsigned char* zsub,
                             int K, long long* counts, long long* sums, hipStream_t s);

// ---- split / merge (splitmerge.hip)
struct LogmlItem {
  int seg[4];  // up to four sub-cluster segments summed; -1 = unused; seg[3] = LOGML_BOUND: see below
};
// a Gaussian item whose seg[3] is LOGML_BOUND yields log|Psi / 2 + C| (C the
// scatter of its segments about their mean) instead of the log marginal: the
// per-cluster term of the merge bound
constexpr int LOGML_BOUND = -3;
// the merge bound is used up to this d: it relies on Minkowski's inequality
// |X + Y|^(1/d) >= |X|^(1/d) + |Y|^(1/d), whose gap grows with d when the two
// clusters' covariances are ill-conditioned in different directions
constexpr int MERGE_BOUND_MAX_D = 16;
// list mode (list != nullptr): the items list_base + list[q] for q < *list_count
// (n_items bounds the grid)
// cmom (may be null; 64 < d <= 128): (K + 1) x CMOM_TILE_ENTRIES doubles of
// scratch for the clusters' summed scatter matrices, rebuilt by the call
constexpr int CMOM_TILE_ENTRIES = 136 * 64;
hipError_t launch_logml_gauss(int n_items, const LogmlItem* items, int d, NiwPriorDev prior,
                              double logdet_psi, const long long* counts, const double* moments,
                              double* scratch, double* out, int* err, hipStream_t s, const int* list = nullptr,
                              const int* list_count = nullptr, int list_base = 0, double* cmom = nullptr,
                              int K = 0);
// the merge bound: accept[p] = 0 for the pairs it rejects, the others listed
// (list, *list_count) for their log marginal and k_merge_decide
hipError_t launch_merge_prune(int n_pairs, const LogmlItem* pairs, int d, NiwPriorDev prior, double logdet_psi,
                              double lam_psi, const long long* counts, const double* moments, const double* lml_cluster,
                              const double* logdet_half, double alpha, bool paper_form, uint64_t seed, uint32_t t,
                              unsigned char* accept, int* list, int* list_count, hipStream_t s);
// accept[p] = merge test of pair item pairs[p] (see k_merge_decide); list mode as above
hipError_t launch_merge_decide(int n_pairs, const LogmlItem* pairs, const long long* counts, const double* lml_cluster,
                               const double* lml_pair, double alpha, bool paper_form, uint64_t seed, uint32_t t,
                               unsigned char* accept, hipStream_t s, const int* list = nullptr,
                               const int* list_count = nullptr);
// [error flag, 8 bytes][counts 2K int64][3K log marginals float64][P merge decisions] in one buffer
size_t readback_bytes(int K, int P);
hipError_t launch_pack_readback(int K, int P, const long long* counts, const double* lml, const unsigned char* mflag,
                                const int* err, unsigned char* out, hipStream_t s);
hipError_t launch_logml_mult(int n_items, const LogmlItem* items, int V, const double* beta,
                             double beta_sum, double lgamma_beta_sum, const double* lgamma_beta,
                             const long long* counts, const long long* sums, double* out, hipStream_t s);
// Gamma-Poisson log marginal: pconst = sum_v (a_v log b_v - lgamma(a_v))
hipError_t launch_logml_pois(int n_items, const LogmlItem* items, int V, const double* shape, const double* rate,
                             double pconst, const long long* counts, const long long* sums, double* out,
                             hipStream_t s);

// relabel table entry for old segment s = 2 z + zsub
struct RelabelEntry {
  int new_z;
  int mode;  // 0 keep zsub, 1 zsub = l, 2 zsub = r, 3 fresh random (TAG_SUBINIT)
};
hipError_t launch_relabel(long long n, const RelabelEntry* table, int n_entries, uint32_t t, uint64_t seed, int* z,
                          unsigned char* zsub, hipStream_t s);
// zero a buffer of 8-byte words with a kernel (no memset nodes, so the call
// stays safe inside captured graphs)
hipError_t launch_zero64(void* p, size_t n_words, hipStream_t s);
hipError_t launch_init_labels(long long n, uint64_t seed, int* z, unsigned char* zsub, hipStream_t s);

}  // namespace dpmm
