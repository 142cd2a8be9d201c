// Kernel declarations of the DPMM HIP library (gfx950).
#pragma once
#include "common.hpp"

namespace dpmm {

#define NIW_SCRATCH(d) ((size_t)3 * (d) * (d) + (d))
// float64 workspaces of the per-component kernels live in LDS up to this d
constexpr int NIW_LDS_MAX_D = 64;
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
__global__ void k_dir_draw(int K, int V, const double* beta, const long long* sums, uint64_t seed,
                           uint32_t t, double* log_theta);
__global__ void k_pack_gauss(int K, int d, int k_max, const double* log_pi, const double* log_pisub,
                             const double* mu, const double* sigma, double* scratch, float* packed,
                             double* logdet_out, int* err);
__global__ void k_pack_mult(int K, int V, int k_max, const double* log_pi, const double* log_pisub,
                            const double* log_theta, float* packed);

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
                            int* tot, int* offs, int* perm, hipStream_t s);
hipError_t launch_sub_stats(int d, bool sample, const float* x, long long n, const int* perm, const int* z,
                            unsigned char* zsub, const float* packed, int K, int k_max, uint32_t t, uint64_t seed,
                            long long* counts, double* moments, hipStream_t s);
// BF16 matrix-core cluster draw (d in {32, 64}) and its whitener fragments
bool mfma_supported(int d);
hipError_t launch_pack_wfrag(int K, int d, int k_max, const float* packed, void* whi, void* wlo, hipStream_t s);
hipError_t launch_label_gauss_mfma(int d, bool x3, const float* x, long long n, int G, long long per_block,
                                   const float* packed, const void* whi, const void* wlo, int K, uint32_t t,
                                   uint64_t seed, int* z, int* hist, int* tot, hipStream_t s);
hipError_t launch_loglik_gauss(int d, const float* x, long long n, const float* packed, int K, int k_max,
                               float* out, hipStream_t s);
hipError_t launch_label_mult(int V, const int* x, long long n, const float* packed, int K, int k_max,
                             uint32_t t, uint64_t seed, int* z, unsigned char* zsub, hipStream_t s);
hipError_t launch_loglik_mult(int V, const int* x, long long n, const float* packed, int K, int k_max,
                              float* out, hipStream_t s);
hipError_t launch_stats_gauss(int d, const float* x, long long n, const int* z, const unsigned char* zsub,
                              int K, long long* counts, double* moments, hipStream_t s);
hipError_t launch_stats_mult(int V, const int* x, long long n, const int* z, const unsigned char* zsub,
                             int K, long long* counts, long long* sums, hipStream_t s);

// ---- split / merge (splitmerge.hip)
struct LogmlItem {
  int seg[4];  // up to four sub-cluster segments summed; -1 = unused
};
hipError_t launch_logml_gauss(int n_items, const LogmlItem* items, int d, NiwPriorDev prior,
                              double logdet_psi, const long long* counts, const double* moments,
                              double* scratch, double* out, int* err, hipStream_t s);
hipError_t launch_logml_mult(int n_items, const LogmlItem* items, int V, const double* beta,
                             double beta_sum, double lgamma_beta_sum, const double* lgamma_beta,
                             const long long* counts, const long long* sums, double* out, hipStream_t s);

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
