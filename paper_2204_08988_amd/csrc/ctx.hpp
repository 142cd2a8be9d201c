// Private definition of the library context and the host helpers shared by
// the C ABI translation units (api.cpp: the sampler; learned.cpp: the learned
// split proposal).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dpmm.h"
#include "kernels.hpp"

using dpmm::LogmlItem;
using dpmm::NiwPriorDev;
using dpmm::RelabelEntry;

// pinned read-back slots of the learned move
struct LearnedBack {
  int sel_count;
  int pad;
  long long side_cnt[2];
  double sums[4];
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct dpmm_ctx {
  dpmm_config cfg{};
  std::vector<double> m, psi, beta, lgamma_beta, gshape, grate;
  double pois_const = 0.0;  // sum_v (a_v log b_v - lgamma(a_v)) of the Gamma prior
  double logdet_psi = 0.0, beta_sum = 0.0, lgamma_beta_sum = 0.0;
  hipStream_t stream = nullptr;
  int device = 0;  // the HIP device current at dpmm_create
  int K = 0;
  std::vector<int> age;
  bool have_params = false;
  bool have_stats = false;
  std::string err;
  int d = 0, E = 0, stride = 0;
  std::vector<DevBuf> bufs;
  // device tables
  double *d_m = nullptr, *d_psi = nullptr, *d_beta = nullptr, *d_lgamma_beta = nullptr;
  double *d_gshape = nullptr, *d_grate = nullptr;  // Poisson: Gamma prior
  // sparse rows: word-major scoring tables [V][K], [V][2K] and the 3K constants
  float *d_tcl = nullptr, *d_tsub = nullptr, *d_cw = nullptr;
  double* d_dpart = nullptr;  // per-chunk (max, sum) of the chunked Dirichlet draw
  long long* d_counts = nullptr;  // [2 k_max]
  double* d_moments = nullptr;    // Gaussian [2 k_max][E]
  long long* d_sums = nullptr;    // multinomial [2 k_max][V]
  double *d_log_pi = nullptr, *d_log_pisub = nullptr, *d_tmp = nullptr;
  double *d_mu = nullptr, *d_sigma = nullptr, *d_log_theta = nullptr, *d_logdet = nullptr;
  float* d_packed = nullptr;
  // one split/merge round's read-back: device buffer and its pinned copy (grown with the items)
  unsigned char* d_rb = nullptr;
  unsigned char* h_rb = nullptr;
  double* d_scratch = nullptr;  // NIW_SCRATCH(d) per workgroup slot
  int scratch_slots = 0;
  int* d_err = nullptr;
  // marginal-likelihood items: device lists and pinned staging, grown by
  // ensure_items (outside bufs)
  LogmlItem* d_items = nullptr;
  double* d_logml = nullptr;
  unsigned char* d_mflag = nullptr;
  int* d_plist = nullptr;   // pairs the merge bound leaves for the exact test
  int* d_pcount = nullptr;  // their number
  double lam_psi = 0.0;     // an upper bound on lambda_max(Psi) (Gershgorin)
  LogmlItem* h_items = nullptr;
  double* h_lml = nullptr;
  unsigned char* h_mflag = nullptr;
  size_t items_cap = 0;
  long long* h_cnt = nullptr;  // pinned [2 k_max]
  int* h_flag = nullptr;       // pinned
  RelabelEntry* d_table = nullptr;
  // cluster-sorted path (Gaussian, d >= dpmm::SORTED_MIN_D)
  int *d_hist = nullptr, *d_offs = nullptr, *d_tot = nullptr, *d_perm = nullptr;
  int* d_zsort = nullptr;  // [perm_cap] the cluster of each row of the sorted order
  double* d_part = nullptr;  // partial statistics slots of the sorted-order statistics kernels
  size_t part_cap = 0;       // doubles in d_part
  double* d_spart = nullptr; // per-workgroup rows of the d <= 4 statistics kernel
  int* d_cspan = nullptr;    // {0, n} of a partition's one cluster (learned split statistics)
  long long hist_cap = 0, perm_cap = 0;
  bool labels_gave_stats = false;
  // BF16 whitener fragments of the cluster components (precision != FP32)
  uint16_t *d_whi = nullptr, *d_wlo = nullptr;
  // offsets, constants and the common centre of the uncentred BF16 main pass (d = 64, 128)
  float* d_wbias = nullptr;
  // the clusters' summed scatter matrices plus Psi / 2 for the log marginals at 64 < d <= 128
  double* d_cmom = nullptr;
  // BF16 fragments of the sub-cluster whiteners and the buffers of the bf16x3
  // sub-label pass (d = 64, 128): per-workgroup counts and offsets, and per
  // sorted row (sized with the permutation) the undecided flags and list
  uint16_t *d_shi = nullptr, *d_slo = nullptr;
  int *d_scnt = nullptr, *d_soffs = nullptr;
  unsigned char* d_sflag = nullptr;
  int *d_perm_c = nullptr, *d_zrow_c = nullptr;
  int* d_nflag = nullptr;  // count of the points deferred to FP32 (matrix-core label kernels)
  int* d_cand = nullptr;   // [perm_cap][RESCORE_CAND] their candidate clusters
  float* d_cst = nullptr;  // [CAND_SPLIT_CAP][CAND_SPLIT_NG][CAND_STATE] split candidate pass lists (d = 64, 128)
  hipEvent_t ev[9] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  bool timing = false;  // record ev[3] between the sort and the statistics kernel
  // record ev[7], ev[8] around the main cluster-draw kernel (matrix-core path);
  // label_kernel_timed tells whether the last label phase did
  bool label_timing = false, label_kernel_timed = false;
  // learned split proposal (cfg.learned = m > 0 principal axes, F = 2m features)
  int lm = 0, F = 0, Fp = 0, n_mlp = 0;
  float *d_p = nullptr, *d_g = nullptr, *d_am = nullptr, *d_av = nullptr;  // FP32 master weights, gradient, Adam
  int adam_t = 0;
  uint32_t train_counter = 0;
  uint16_t *d_w1t = nullptr, *d_w2t = nullptr, *d_w2 = nullptr;  // BF16 operand copies
  bool weights_fresh = false;
  // per-chunk activations (MLP_CHUNK rows)
  uint16_t *d_x16 = nullptr, *d_x16t = nullptr, *d_h1 = nullptr, *d_h1t = nullptr;
  uint16_t *d_d2 = nullptr, *d_d2t = nullptr, *d_d1 = nullptr, *d_d1t = nullptr;
  float *d_h2 = nullptr, *d_o = nullptr, *d_y = nullptr;
  int *d_bidx = nullptr, *d_bcl = nullptr;
  float* d_frames = nullptr;  // [k_max][d + m d + m]
  int *d_flip = nullptr, *d_elig = nullptr;
  double* d_lsums = nullptr;     // proposal sums [4], loss [1]
  double* d_red = nullptr;       // rows of the fixed-order reductions (MLP_RED_DOUBLES)
  double* d_setpart = nullptr;   // set-statistics partials [SET_STATS_BLOCKS][2][E + 1]
  int* d_selcnt = nullptr;       // selection block counts [SELECT_BLOCKS + 1]
  int* d_sel = nullptr;          // selected point indices [sel_cap]
  unsigned char* d_side = nullptr;  // side of each point [sel_cap]
  long long sel_cap = 0;
  float* h_frame = nullptr;       // pinned staging of one set frame
  LearnedBack* h_back = nullptr;  // pinned read-back slots

  dpmm_status fail(dpmm_status s, const std::string& msg) {
    err = msg;
    return s;
  }
  dpmm_status hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return DPMM_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? DPMM_E_OOM : DPMM_E_DEVICE;
  }
  template <typename T>
  hipError_t alloc(T** p, size_t count) {
    DevBuf b;
    b.bytes = std::max<size_t>(count * sizeof(T), 16);
    hipError_t e = hipMalloc(&b.p, b.bytes);
    if (e != hipSuccess) return e;
    bufs.push_back(b);
    *p = static_cast<T*>(b.p);
    return hipSuccess;
  }
  bool gaussian() const { return cfg.family == DPMM_GAUSSIAN; }
  bool poisson() const { return cfg.family == DPMM_POISSON; }
  bool sparse() const { return cfg.sparse != 0; }
  bool sorted_path() const { return gaussian() && d >= dpmm::SORTED_MIN_D; }
};

#define DPMM_TRY(expr)                         \
  do {                                         \
    dpmm_status _s = (expr);                   \
    if (_s != DPMM_OK) return _s;              \
  } while (0)
#define DPMM_HIP(ctx, expr, what) DPMM_TRY((ctx)->hip((expr), (what)))

namespace dpmm::host {

// device scratch of the statistics kernels: sort tables (hist, offs [G][K],
// tot [K + 2]), permutation and sorted labels [n], partial slots of the
// sorted-order kernels, per-workgroup rows of the d <= 4 kernel
struct StatsBufs {
  int *hist, *offs, *tot, *perm, *zsort;
  double *part, *spart;
};

inline int tri_index(int a, int b, int d) { return a * d - (a * (a - 1)) / 2 + (b - a); }
dpmm_status check_n(dpmm_ctx* ctx, const void* x, int64_t n);
NiwPriorDev prior_dev(dpmm_ctx* ctx);
dpmm_status launch_stats(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, const uint8_t* zsub);
dpmm_status ensure_part(dpmm_ctx* ctx, int64_t n);
// the statistics with the scratch b; whether they take the cluster-sorted kernels
dpmm_status stats_with(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, const uint8_t* zsub,
                       const StatsBufs& b);
bool stats_sorted(const dpmm_ctx* ctx);
// static_scratch.cpp: resolve this device's static scratch (dpmm_create)
dpmm_status static_scratch_init(dpmm_ctx* ctx);
// log marginal likelihoods of segment unions, read back (synchronises);
// *flag_out (optional) receives the device error flag
dpmm_status logml(dpmm_ctx* ctx, const std::vector<LogmlItem>& items, std::vector<double>& out,
                  int* flag_out = nullptr);
dpmm_status check_device_error(dpmm_ctx* ctx);
dpmm_status flag_fail(dpmm_ctx* ctx, int flag);
SparseRows sparse_rows(const void* x);
dpmm_status ensure_items(dpmm_ctx* ctx, size_t count);
dpmm_status apply_relabel(dpmm_ctx* ctx, const std::vector<RelabelEntry>& table, int64_t n, uint32_t t, int32_t* z,
                          uint8_t* zsub);
// learned.cpp: buffers of the learned proposal (called by dpmm_create)
dpmm_status learned_alloc(dpmm_ctx* ctx);
dpmm_status learned_move(dpmm_ctx* ctx, const void* x, int64_t n, uint32_t t, int32_t* z, uint8_t* zsub,
                         uint8_t* side_out, dpmm_learned_info* info);

}  // namespace dpmm::host
