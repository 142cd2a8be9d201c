// Host runtime of the DPMM HIP library: the C ABI declared in include/dpmm.h.
//
// The context owns every device table sized by k_max; the caller owns the
// data and the labels.  Per iteration the device does all O(N) work (labels,
// statistics, relabelling) and all float64 linear algebra (posterior draws,
// marginal likelihoods); the host only runs the O(K^2) accept/reject
// bookkeeping of splits and merges on a few hundred doubles read back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.hpp"

using namespace dpmm;
using namespace dpmm::host;

namespace {

thread_local std::string g_create_error;

}  // namespace


namespace {

bool host_cholesky_logdet(std::vector<double> a, int d, double* logdet) {
  for (int j = 0; j < d; ++j) {
    double s = a[j * d + j];
    for (int k = 0; k < j; ++k) s -= a[j * d + k] * a[j * d + k];
    if (!(s > 0.0) || !std::isfinite(s)) return false;
    a[j * d + j] = std::sqrt(s);
    for (int i = j + 1; i < d; ++i) {
      double t = a[i * d + j];
      for (int k = 0; k < j; ++k) t -= a[i * d + k] * a[j * d + k];
      a[i * d + j] = t / a[j * d + j];
    }
  }
  double ld = 0.0;
  for (int j = 0; j < d; ++j) ld += std::log(a[j * d + j]);
  *logdet = 2.0 * ld;
  return true;
}

}  // namespace

namespace dpmm::host {

dpmm_status check_n(dpmm_ctx* ctx, const void* x, int64_t n) {
  if (!x && n > 0) return ctx->fail(DPMM_E_ARG, "x is NULL");
  if (ctx->sparse() && x) {
    const dpmm_csr* c = static_cast<const dpmm_csr*>(x);
    if (c->nnz < 0) return ctx->fail(DPMM_E_SHAPE, "nnz must be >= 0");
    if (n > 0 && !c->row_ptr) return ctx->fail(DPMM_E_ARG, "row_ptr is NULL");
    if (c->nnz > 0 && (!c->col || !c->val)) return ctx->fail(DPMM_E_ARG, "col / val is NULL");
  }
  // point indices are int32 on the device (the cluster-sorted permutation, the
  // deferred-draw list, the learned proposal's selection)
  if (n < 0 || n > (int64_t)0x7FFFFFFFLL) return ctx->fail(DPMM_E_SHAPE, "n must lie in [0, 2^31)");
  return DPMM_OK;
}

SparseRows sparse_rows(const void* x) {
  const dpmm_csr* c = static_cast<const dpmm_csr*>(x);
  SparseRows r;
  r.row_ptr = reinterpret_cast<const long long*>(c->row_ptr);
  r.col = c->col;
  r.val = c->val;
  r.nnz = c->nnz;
  return r;
}

// the status of a non-zero device error flag (and the flag cleared)
dpmm_status flag_fail(dpmm_ctx* ctx, int flag) {
  DPMM_HIP(ctx, hipMemsetAsync(ctx->d_err, 0, sizeof(int), ctx->stream), "clear flag");
  if (flag & ERR_SPARSE_INPUT)
    return ctx->fail(DPMM_E_ARG, "sparse rows: a row range outside [0, nnz], a column outside [0, V) or a "
                                 "negative count");
  return ctx->fail(DPMM_E_NUMERIC, "a float64 Cholesky factorisation met a non-positive pivot (flag " +
                                       std::to_string(flag) + ")");
}

NiwPriorDev prior_dev(dpmm_ctx* ctx) {
  NiwPriorDev p;
  p.kappa = ctx->cfg.kappa;
  p.nu = ctx->cfg.nu;
  p.m = ctx->d_m;
  p.psi = ctx->d_psi;
  return p;
}

dpmm_status ensure_perm(dpmm_ctx* ctx, int64_t n) {
  if (n > 0x7FFFFFFFLL) return ctx->fail(DPMM_E_SHAPE, "the Gaussian path for d >= 5 takes n < 2^31 points");
  if (n <= ctx->perm_cap) return DPMM_OK;
  if (ctx->d_perm) {
    DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    hipFree(ctx->d_perm);
    hipFree(ctx->d_zsort);
    hipFree(ctx->d_cand);
    hipFree(ctx->d_sflag);
    hipFree(ctx->d_perm_c);
    hipFree(ctx->d_zrow_c);
    ctx->d_perm = nullptr;
    ctx->d_zsort = nullptr;
    ctx->d_cand = nullptr;
    ctx->d_sflag = nullptr;
    ctx->d_perm_c = nullptr;
    ctx->d_zrow_c = nullptr;
    ctx->perm_cap = 0;
  }
  DPMM_HIP(ctx, hipMalloc(&ctx->d_perm, (size_t)n * sizeof(int)), "allocate permutation");
  DPMM_HIP(ctx, hipMalloc(&ctx->d_zsort, (size_t)n * sizeof(int)), "allocate sorted labels");
  // candidate lists of the points the matrix-core label kernels defer
  if (ctx->d_nflag)
    DPMM_HIP(ctx, hipMalloc(&ctx->d_cand, (size_t)n * RESCORE_CAND * sizeof(int)), "allocate candidate lists");
  if (ctx->d_shi) {  // the bf16x3 sub-label pass: flags and the undecided rows' list
    DPMM_HIP(ctx, hipMalloc(&ctx->d_sflag, (size_t)n), "allocate sub-label flags");
    DPMM_HIP(ctx, hipMalloc(&ctx->d_perm_c, (size_t)n * sizeof(int)), "allocate sub-label list");
    DPMM_HIP(ctx, hipMalloc(&ctx->d_zrow_c, (size_t)n * sizeof(int)), "allocate sub-label list");
  }
  ctx->perm_cap = n;
  return ensure_part(ctx, n);
}

// partial-slot buffer of the sorted-order statistics kernels, sized for any
// number of rows (allocated once)
dpmm_status ensure_part(dpmm_ctx* ctx, int64_t n) {
  const size_t need = sub_stats_part_doubles(ctx->d, n);
  if (need <= ctx->part_cap) return DPMM_OK;
  const size_t cap = std::max(need, sub_stats_part_doubles_max(ctx->d));
  if (ctx->d_part) {
    DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    hipFree(ctx->d_part);
    ctx->d_part = nullptr;
    ctx->part_cap = 0;
  }
  DPMM_HIP(ctx, hipMalloc(&ctx->d_part, cap * sizeof(double)), "allocate partial statistics");
  ctx->part_cap = cap;
  return DPMM_OK;
}

// statistics over the cluster-sorted order with the given scratch; with
// sample = true also draws zsub
dpmm_status sorted_pass_with(dpmm_ctx* ctx, const void* x, int64_t n, bool labels_done_hist, bool sample, uint32_t t,
                             const int32_t* z, uint8_t* zsub, int G, long long per_block, const StatsBufs& b) {
  DPMM_HIP(ctx, launch_sort_by_z(z, n, ctx->K, G, per_block, labels_done_hist, b.hist, b.tot, b.offs, b.perm, b.zsort,
                                 ctx->stream), "sort by cluster");
  if (ctx->timing) DPMM_HIP(ctx, hipEventRecord(ctx->ev[3], ctx->stream), "event");
  // BF16 tables at d = 64, 128: the sub-labels in bf16x3 first, the FP32 kernel on the rows left
  SubX3 x3{ctx->d_shi, ctx->d_slo, ctx->d_sflag, ctx->d_scnt, ctx->d_soffs, ctx->d_perm_c, ctx->d_zrow_c};
  const bool use_x3 = sample && ctx->d_shi && ctx->d_sflag && b.perm == ctx->d_perm;
  DPMM_HIP(ctx, launch_sub_stats(ctx->d, sample, (const float*)x, n, b.perm, z, b.zsort, zsub, ctx->d_packed, ctx->K,
                                 ctx->cfg.k_max, t, ctx->cfg.seed, ctx->d_counts, ctx->d_moments, b.offs, b.tot, b.part,
                                 ctx->stream, use_x3 ? &x3 : nullptr),
           "sub-label / statistics kernel");
  ctx->have_stats = true;
  return DPMM_OK;
}

StatsBufs ctx_bufs(dpmm_ctx* ctx) {
  return StatsBufs{ctx->d_hist, ctx->d_offs, ctx->d_tot, ctx->d_perm, ctx->d_zsort, ctx->d_part, ctx->d_spart};
}

// statistics over the cluster-sorted order; with sample = true also draws zsub
dpmm_status sorted_pass(dpmm_ctx* ctx, const void* x, int64_t n, bool labels_done_hist, bool sample, uint32_t t,
                        const int32_t* z, uint8_t* zsub, int G, long long per_block) {
  DPMM_TRY(ensure_perm(ctx, n));
  DPMM_TRY(ensure_part(ctx, n));
  return sorted_pass_with(ctx, x, n, labels_done_hist, sample, t, z, zsub, G, per_block, ctx_bufs(ctx));
}

bool stats_sorted(const dpmm_ctx* ctx) {
  return ctx->gaussian() && (ctx->sorted_path() || !stats_small_lanes(ctx->d, ctx->K));
}

dpmm_status stats_with(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, const uint8_t* zsub,
                       const StatsBufs& b) {
  hipError_t e;
  // Gaussian: per-lane accumulators for d <= 4 while they fit in LDS, else
  // the cluster-sorted kernels (both take their sums in a fixed order)
  if (stats_sorted(ctx)) {
    int G;
    long long per;
    sorted_plan(n, ctx->K, ctx->hist_cap, &G, &per);
    return sorted_pass_with(ctx, x, n, false, false, 0, z, const_cast<uint8_t*>(zsub), G, per, b);
  }
  if (ctx->gaussian())
    e = launch_stats_gauss(ctx->d, (const float*)x, n, z, zsub, ctx->K, ctx->d_counts, ctx->d_moments, b.spart,
                           ctx->stream);
  else if (ctx->sparse())
    e = launch_stats_csr(sparse_rows(x), n, ctx->d, z, zsub, ctx->K, ctx->d_counts, ctx->d_sums, ctx->d_err,
                         ctx->stream);
  else
    e = launch_stats_mult(ctx->d, (const int*)x, n, z, zsub, ctx->K, ctx->d_counts, ctx->d_sums, ctx->stream);
  DPMM_HIP(ctx, e, "statistics kernel");
  ctx->have_stats = true;
  return DPMM_OK;
}

dpmm_status launch_stats(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, const uint8_t* zsub) {
  if (stats_sorted(ctx)) {
    DPMM_TRY(ensure_perm(ctx, n));
    DPMM_TRY(ensure_part(ctx, n));
  }
  return stats_with(ctx, x, n, z, zsub, ctx_bufs(ctx));
}

// capacity of the item lists and their pinned staging (synchronises when it grows)
dpmm_status ensure_items(dpmm_ctx* ctx, size_t count) {
  if (count <= ctx->items_cap) return DPMM_OK;
  const size_t cap = std::max(count, 2 * ctx->items_cap);
  if (ctx->items_cap) DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  hipFree(ctx->d_items);
  hipFree(ctx->d_logml);
  hipFree(ctx->d_mflag);
  hipFree(ctx->d_plist);
  hipHostFree(ctx->h_items);
  hipHostFree(ctx->h_lml);
  hipHostFree(ctx->h_mflag);
  hipFree(ctx->d_rb);
  hipHostFree(ctx->h_rb);
  ctx->d_plist = nullptr;
  ctx->d_rb = nullptr;
  ctx->h_rb = nullptr;
  ctx->d_items = nullptr;
  ctx->d_logml = nullptr;
  ctx->d_mflag = nullptr;
  ctx->h_items = nullptr;
  ctx->h_lml = nullptr;
  ctx->h_mflag = nullptr;
  ctx->items_cap = 0;
  DPMM_HIP(ctx, hipMalloc(&ctx->d_items, cap * sizeof(LogmlItem)), "allocate items");
  DPMM_HIP(ctx, hipMalloc(&ctx->d_logml, cap * sizeof(double)), "allocate items");
  DPMM_HIP(ctx, hipMalloc(&ctx->d_mflag, cap), "allocate items");
  DPMM_HIP(ctx, hipMalloc(&ctx->d_plist, cap * sizeof(int)), "allocate items");
  DPMM_HIP(ctx, hipHostMalloc((void**)&ctx->h_items, cap * sizeof(LogmlItem), hipHostMallocDefault), "pin items");
  DPMM_HIP(ctx, hipHostMalloc((void**)&ctx->h_lml, cap * sizeof(double), hipHostMallocDefault), "pin items");
  DPMM_HIP(ctx, hipHostMalloc((void**)&ctx->h_mflag, cap, hipHostMallocDefault), "pin items");
  const size_t rb = readback_bytes(ctx->cfg.k_max, (int)cap);
  DPMM_HIP(ctx, hipMalloc(&ctx->d_rb, rb), "allocate read-back");
  DPMM_HIP(ctx, hipHostMalloc((void**)&ctx->h_rb, rb, hipHostMallocDefault), "pin read-back");
  ctx->items_cap = cap;
  return DPMM_OK;
}

// copy items to d_items (through pinned staging)
dpmm_status logml_upload(dpmm_ctx* ctx, const LogmlItem* items, size_t count) {
  DPMM_TRY(ensure_items(ctx, count));
  if (count == 0) return DPMM_OK;
  std::memcpy(ctx->h_items, items, count * sizeof(LogmlItem));
  DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_items, ctx->h_items, count * sizeof(LogmlItem), hipMemcpyHostToDevice,
                               ctx->stream), "copy items");
  return DPMM_OK;
}

// the log marginal likelihoods of the uploaded items [first, first + count)
// into d_logml[first ...]
dpmm_status logml_range(dpmm_ctx* ctx, size_t first, size_t count) {
  if (count == 0) return DPMM_OK;
  hipError_t e;
  if (ctx->gaussian())
    e = launch_logml_gauss((int)count, ctx->d_items + first, ctx->d, prior_dev(ctx), ctx->logdet_psi, ctx->d_counts,
                           ctx->d_moments, ctx->d_scratch, ctx->d_logml + first, ctx->d_err, ctx->stream, nullptr,
                           nullptr, 0, ctx->d_cmom, ctx->K);
  else if (ctx->poisson())
    e = launch_logml_pois((int)count, ctx->d_items + first, ctx->d, ctx->d_gshape, ctx->d_grate, ctx->pois_const,
                          ctx->d_counts, ctx->d_sums, ctx->d_logml + first, ctx->stream);
  else
    e = launch_logml_mult((int)count, ctx->d_items + first, ctx->d, ctx->d_beta, ctx->beta_sum, ctx->lgamma_beta_sum,
                          ctx->d_lgamma_beta, ctx->d_counts, ctx->d_sums, ctx->d_logml + first, ctx->stream);
  DPMM_HIP(ctx, e, "log marginal likelihood kernel");
  return DPMM_OK;
}

// enqueue the log marginal likelihoods of items (copied through pinned staging)
dpmm_status logml_launch(dpmm_ctx* ctx, const LogmlItem* items, size_t count) {
  DPMM_TRY(logml_upload(ctx, items, count));
  return logml_range(ctx, 0, count);
}

// log marginal likelihoods of a list of segment unions (device), read back
// with one synchronisation.  *flag_out (optional) receives the device error
// flag after the launch.
dpmm_status logml(dpmm_ctx* ctx, const std::vector<LogmlItem>& items, std::vector<double>& out, int* flag_out) {
  out.assign(items.size(), 0.0);
  DPMM_TRY(logml_launch(ctx, items.data(), items.size()));
  if (!items.empty())
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->h_lml, ctx->d_logml, items.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 ctx->stream), "copy log marginals");
  if (flag_out)
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->h_flag, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream),
             "copy flag");
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  std::memcpy(out.data(), ctx->h_lml, items.size() * sizeof(double));
  if (flag_out) *flag_out = *ctx->h_flag;
  return DPMM_OK;
}

dpmm_status read_counts(dpmm_ctx* ctx, std::vector<long long>& cnt) {
  cnt.assign(2 * (size_t)ctx->K, 0);
  DPMM_HIP(ctx, hipMemcpyAsync(cnt.data(), ctx->d_counts, cnt.size() * sizeof(long long), hipMemcpyDeviceToHost,
                               ctx->stream), "copy counts");
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  return DPMM_OK;
}

dpmm_status check_device_error(dpmm_ctx* ctx) {
  int flag = 0;
  DPMM_HIP(ctx, hipMemcpyAsync(&flag, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "copy flag");
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  if (flag) return flag_fail(ctx, flag);
  return DPMM_OK;
}

dpmm_status apply_relabel(dpmm_ctx* ctx, const std::vector<RelabelEntry>& table, int64_t n, uint32_t t,
                          int32_t* z, uint8_t* zsub) {
  DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_table, table.data(), table.size() * sizeof(RelabelEntry),
                               hipMemcpyHostToDevice, ctx->stream), "copy relabel table");
  DPMM_HIP(ctx, launch_relabel(n, ctx->d_table, (int)table.size(), t, ctx->cfg.seed, z, zsub, ctx->stream),
           "relabel kernel");
  return DPMM_OK;
}

double log_posterior(const dpmm_ctx* ctx, const std::vector<long long>& cnt, const std::vector<double>& lml) {
  const double a = ctx->cfg.alpha;
  long long N = 0;
  for (long long c : cnt) N += c;
  double lp = ctx->K * std::log(a) + std::lgamma(a) - std::lgamma(a + (double)N);
  for (int k = 0; k < ctx->K; ++k) lp += std::lgamma((double)(cnt[2 * k] + cnt[2 * k + 1])) + lml[k];
  return lp;
}

dpmm_status pack_params(dpmm_ctx* ctx) {
  const int K = ctx->K;
  if (ctx->gaussian()) {
    hipLaunchKernelGGL(k_pack_gauss, dim3(3 * K), dim3(256), niw_lds_bytes(ctx->d), ctx->stream, K, ctx->d,
                       ctx->cfg.k_max,
                       ctx->d_log_pi, ctx->d_log_pisub, ctx->d_mu, ctx->d_sigma, ctx->d_scratch, ctx->d_packed,
                       ctx->d_logdet, ctx->d_err);
  } else {
    hipLaunchKernelGGL(k_pack_mult, dim3(3 * K), dim3(256), 0, ctx->stream, K, ctx->d, ctx->cfg.k_max,
                       ctx->d_log_pi, ctx->d_log_pisub, ctx->d_log_theta, ctx->d_packed, ctx->poisson() ? 1 : 0);
  }
  DPMM_HIP(ctx, hipGetLastError(), "pack kernel");
  if (ctx->sparse())
    DPMM_HIP(ctx, launch_pack_csr(K, ctx->d, ctx->cfg.k_max, ctx->d_packed, ctx->d_tcl, ctx->d_tsub, ctx->d_cw,
                                  ctx->stream), "sparse table pack kernel");
  if (ctx->d_whi)
    DPMM_HIP(ctx, launch_pack_wfrag(K, ctx->d, ctx->cfg.k_max, ctx->d_packed, ctx->d_whi, ctx->d_wlo, ctx->d_wbias,
                                    ctx->d_shi, ctx->d_slo, ctx->stream),
             "fragment pack kernel");
  ctx->have_params = true;
  return DPMM_OK;
}

}  // namespace dpmm::host

extern "C" {

const char* dpmm_status_string(dpmm_status s) {
  switch (s) {
    case DPMM_OK: return "ok";
    case DPMM_E_ARG: return "invalid argument";
    case DPMM_E_SHAPE: return "shape mismatch";
    case DPMM_E_CAPACITY: return "capacity exceeded";
    case DPMM_E_NUMERIC: return "numerical error";
    case DPMM_E_DEVICE: return "device error";
    case DPMM_E_OOM: return "out of device memory";
    case DPMM_E_STATE: return "invalid state";
    default: return "unknown status";
  }
}

const char* dpmm_last_error(const dpmm_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

dpmm_status dpmm_create(const dpmm_config* cfg, void* hip_stream, dpmm_ctx** out) {
  if (!out) {
    g_create_error = "out is NULL";
    return DPMM_E_ARG;
  }
  *out = nullptr;
  auto bad = [](dpmm_status s, const char* msg) {
    g_create_error = msg;
    return s;
  };
  if (!cfg) return bad(DPMM_E_ARG, "cfg is NULL");
  if (cfg->family != DPMM_GAUSSIAN && cfg->family != DPMM_MULTINOMIAL && cfg->family != DPMM_POISSON)
    return bad(DPMM_E_ARG, "unknown family");
  if (cfg->family == DPMM_GAUSSIAN && (cfg->d < 1 || cfg->d > 128))
    return bad(DPMM_E_ARG, "Gaussian dimension must lie in [1, 128]");
  if (cfg->sparse != 0 && cfg->sparse != 1) return bad(DPMM_E_ARG, "sparse must be 0 or 1");
  if (cfg->sparse && cfg->family == DPMM_GAUSSIAN)
    return bad(DPMM_E_ARG, "sparse rows need the multinomial or Poisson family");
  const int max_v = cfg->sparse ? (1 << 20) : 128;
  if (cfg->family == DPMM_MULTINOMIAL && (cfg->d < 1 || cfg->d > max_v))
    return bad(DPMM_E_ARG, cfg->sparse ? "vocabulary size must lie in [1, 2^20]" : "vocabulary size must lie in [1, 128]");
  if (cfg->family == DPMM_POISSON && (cfg->d < 1 || cfg->d > max_v))
    return bad(DPMM_E_ARG, cfg->sparse ? "Poisson dimension must lie in [1, 2^20]" : "Poisson dimension must lie in [1, 128]");
  if (cfg->k_max < 1 || cfg->k_max > 4096) return bad(DPMM_E_ARG, "k_max must lie in [1, 4096]");
  if (cfg->burn_out < 0) return bad(DPMM_E_ARG, "burn_out must be >= 0");
  if (!(cfg->alpha > 0.0) || !std::isfinite(cfg->alpha)) return bad(DPMM_E_ARG, "alpha must be > 0");
  if (cfg->precision != DPMM_FP32 && cfg->precision != DPMM_BF16 && cfg->precision != DPMM_BF16X3)
    return bad(DPMM_E_ARG, "unknown precision");
  if (cfg->precision != DPMM_FP32 && !(cfg->family == DPMM_GAUSSIAN && mfma_supported(cfg->d)))
    return bad(DPMM_E_ARG, "BF16 matrix-core scoring needs the Gaussian family with d = 32, 64 or 128");
  if (cfg->merge_form != DPMM_MERGE_PAPER && cfg->merge_form != DPMM_MERGE_INVERSE_SPLIT)
    return bad(DPMM_E_ARG, "unknown merge_form");
  if (cfg->learned < 0) return bad(DPMM_E_ARG, "learned must be >= 0");
  if (cfg->learned > 0 && cfg->family != DPMM_GAUSSIAN)
    return bad(DPMM_E_ARG, "the learned proposal needs the Gaussian family");
  if (cfg->learned > 0 && (cfg->learned > cfg->d || cfg->learned > 32))
    return bad(DPMM_E_ARG, "learned (principal axes) must lie in [1, min(d, 32)]");
  const int d = cfg->d;
  std::unique_ptr<dpmm_ctx> ctx(new dpmm_ctx());
  ctx->cfg = *cfg;
  ctx->d = d;
  if (cfg->family == DPMM_GAUSSIAN) {
    if (!(cfg->kappa > 0.0)) return bad(DPMM_E_ARG, "kappa must be > 0");
    if (!(cfg->nu > d - 1)) return bad(DPMM_E_ARG, "nu must be > d - 1");
    if (!cfg->m || !cfg->psi) return bad(DPMM_E_ARG, "m and psi are required");
    ctx->m.assign(cfg->m, cfg->m + d);
    ctx->psi.assign(cfg->psi, cfg->psi + (size_t)d * d);
    for (double v : ctx->m)
      if (!std::isfinite(v)) return bad(DPMM_E_NUMERIC, "m is not finite");
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j)
        if (ctx->psi[i * d + j] != ctx->psi[j * d + i]) return bad(DPMM_E_NUMERIC, "psi is not symmetric");
    if (!host_cholesky_logdet(ctx->psi, d, &ctx->logdet_psi)) return bad(DPMM_E_NUMERIC, "psi is not positive definite");
    // Gershgorin: the largest absolute row sum bounds lambda_max(Psi) (the merge bound)
    for (int i = 0; i < d; ++i) {
      double r = 0.0;
      for (int j = 0; j < d; ++j) r += std::fabs(ctx->psi[i * d + j]);
      ctx->lam_psi = std::max(ctx->lam_psi, r);
    }
    ctx->E = d + d * (d + 1) / 2;
    ctx->stride = gauss_rec_stride(d);
  } else if (cfg->family == DPMM_POISSON) {
    if (!cfg->gamma_shape || !cfg->gamma_rate) return bad(DPMM_E_ARG, "gamma_shape and gamma_rate are required");
    ctx->gshape.assign(cfg->gamma_shape, cfg->gamma_shape + d);
    ctx->grate.assign(cfg->gamma_rate, cfg->gamma_rate + d);
    for (int v = 0; v < d; ++v) {
      const double a = ctx->gshape[v], b = ctx->grate[v];
      if (!(a > 0.0) || !std::isfinite(a) || !(b > 0.0) || !std::isfinite(b))
        return bad(DPMM_E_ARG, "the Gamma prior needs shape > 0 and rate > 0");
      ctx->pois_const += a * std::log(b) - std::lgamma(a);
    }
    ctx->E = 0;
    ctx->stride = mult_rec_stride(d);
  } else {
    if (!cfg->beta) return bad(DPMM_E_ARG, "beta is required");
    ctx->beta.assign(cfg->beta, cfg->beta + d);
    for (double b : ctx->beta) {
      if (!(b > 0.0) || !std::isfinite(b)) return bad(DPMM_E_ARG, "beta must be > 0");
      ctx->beta_sum += b;
      ctx->lgamma_beta.push_back(std::lgamma(b));
    }
    ctx->lgamma_beta_sum = std::lgamma(ctx->beta_sum);
    ctx->E = 0;
    ctx->stride = mult_rec_stride(d);
  }
  ctx->cfg.m = ctx->cfg.psi = ctx->cfg.beta = ctx->cfg.gamma_shape = ctx->cfg.gamma_rate = nullptr;
  ctx->stream = (hipStream_t)hip_stream;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return bad(DPMM_E_DEVICE, "no HIP device");
  if (hipGetDevice(&ctx->device) != hipSuccess) return bad(DPMM_E_DEVICE, "no current HIP device");
  if (static_scratch_init(ctx.get()) != DPMM_OK) {
    g_create_error = ctx->err;
    return DPMM_E_DEVICE;
  }
  const int km = cfg->k_max;
  dpmm_ctx* c = ctx.get();
  auto chk = [&](hipError_t e) { return e == hipSuccess; };
  bool ok = true;
  ok = ok && chk(c->alloc(&c->d_counts, 2 * (size_t)km));
  ok = ok && chk(c->alloc(&c->d_log_pi, (size_t)km + 1));
  ok = ok && chk(c->alloc(&c->d_log_pisub, 2 * (size_t)km));
  ok = ok && chk(c->alloc(&c->d_tmp, (size_t)3 * km + 1));  // the K + 1 + 2K log-gamma draws of k_weights
  ok = ok && chk(c->alloc(&c->d_logdet, 3 * (size_t)km));
  ok = ok && chk(c->alloc(&c->d_packed, 3 * (size_t)km * c->stride));
  ok = ok && chk(c->alloc(&c->d_err, 1));
  ok = ok && chk(c->alloc(&c->d_table, 4 * (size_t)km));
  ok = ok && chk(c->alloc(&c->d_pcount, 2));
  if (c->gaussian()) {
    ok = ok && chk(c->alloc(&c->d_m, (size_t)d));
    ok = ok && chk(c->alloc(&c->d_psi, (size_t)d * d));
    ok = ok && chk(c->alloc(&c->d_moments, 2 * (size_t)km * c->E));
    ok = ok && chk(c->alloc(&c->d_mu, 3 * (size_t)km * d));
    ok = ok && chk(c->alloc(&c->d_sigma, 3 * (size_t)km * d * d));
    c->scratch_slots = std::max(3 * km, 256);
    ok = ok && chk(c->alloc(&c->d_scratch, (size_t)c->scratch_slots * NIW_SCRATCH(d)));
    if (d > 64 && d <= 128) ok = ok && chk(c->alloc(&c->d_cmom, ((size_t)km + 1) * CMOM_TILE_ENTRIES));
    if (cfg->precision != DPMM_FP32) {
      ok = ok && chk(c->alloc(&c->d_whi, (size_t)km * d * d));
      ok = ok && chk(c->alloc(&c->d_nflag, 2));
      // low parts: the bf16x3 form, and the candidate pass of either matrix-core form
      ok = ok && chk(c->alloc(&c->d_wlo, (size_t)km * d * d));
      if (wbias_floats(d, km)) ok = ok && chk(c->alloc(&c->d_wbias, wbias_floats(d, km)));
      if (d == 64 || d == 128) {
        ok = ok && chk(c->alloc(&c->d_shi, (size_t)2 * km * d * d));
        ok = ok && chk(c->alloc(&c->d_slo, (size_t)2 * km * d * d));
        ok = ok && chk(c->alloc(&c->d_scnt, (size_t)SUBX_GROUPS));
        ok = ok && chk(c->alloc(&c->d_soffs, (size_t)SUBX_GROUPS + 1));
        // the split candidate pass's per-group lists of up to CAND_SPLIT_CAP deferred points
        ok = ok && chk(c->alloc(&c->d_cst, (size_t)CAND_SPLIT_CAP * CAND_SPLIT_NG * CAND_STATE));
      }
    }
    // counting sort by cluster: the label path for d >= 5, the statistics of
    // any d once K outgrows the small-d kernel's LDS accumulators
    c->hist_cap = 2048LL * km;
    ok = ok && chk(c->alloc(&c->d_hist, (size_t)c->hist_cap));
    ok = ok && chk(c->alloc(&c->d_offs, (size_t)c->hist_cap));
    ok = ok && chk(c->alloc(&c->d_tot, (size_t)km + 2));
    ok = ok && chk(c->alloc(&c->d_cspan, 2));
    if (d <= 4) {
      size_t sp = 0;
      for (int k = 1; k <= km; ++k) sp = std::max(sp, stats_small_part_doubles(d, k));
      ok = ok && chk(c->alloc(&c->d_spart, std::max<size_t>(sp, 1)));
    }
  } else {
    if (c->poisson()) {
      ok = ok && chk(c->alloc(&c->d_gshape, (size_t)d));
      ok = ok && chk(c->alloc(&c->d_grate, (size_t)d));
    } else {
      ok = ok && chk(c->alloc(&c->d_beta, (size_t)d));
      ok = ok && chk(c->alloc(&c->d_lgamma_beta, (size_t)d));
    }
    ok = ok && chk(c->alloc(&c->d_sums, 2 * (size_t)km * d));
    ok = ok && chk(c->alloc(&c->d_log_theta, 3 * (size_t)km * d));
    if (d > DIR_CHUNK && !c->poisson())
      ok = ok && chk(c->alloc(&c->d_dpart, 2 * (size_t)3 * km * ((d + DIR_CHUNK - 1) / DIR_CHUNK)));
    if (c->sparse()) {
      ok = ok && chk(c->alloc(&c->d_tcl, (size_t)((km + 3) & ~3) * d));
      ok = ok && chk(c->alloc(&c->d_tsub, 2 * (size_t)km * d));
      ok = ok && chk(c->alloc(&c->d_cw, 3 * (size_t)km));
    }
  }
  // every failure below releases what was allocated through dpmm_destroy
  if (!ok) {
    dpmm_destroy(ctx.release());
    return bad(DPMM_E_OOM, "device allocation failed");
  }
  if (cfg->learned > 0 && learned_alloc(c) != DPMM_OK) {
    g_create_error = c->err;
    dpmm_destroy(ctx.release());
    return DPMM_E_OOM;
  }
  hipError_t e = hipSuccess;
  if (c->gaussian()) {
    e = hipMemcpy(c->d_m, c->m.data(), d * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_psi, c->psi.data(), (size_t)d * d * sizeof(double), hipMemcpyHostToDevice);
  } else if (c->poisson()) {
    e = hipMemcpy(c->d_gshape, c->gshape.data(), d * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_grate, c->grate.data(), d * sizeof(double), hipMemcpyHostToDevice);
  } else {
    e = hipMemcpy(c->d_beta, c->beta.data(), d * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(c->d_lgamma_beta, c->lgamma_beta.data(), d * sizeof(double), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemset(c->d_err, 0, sizeof(int));
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_cnt, 2 * (size_t)km * sizeof(long long), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_flag, sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess && ensure_items(c, (size_t)std::max(3 * km, 256)) != DPMM_OK) e = hipErrorOutOfMemory;
  if (e == hipSuccess) e = hipMemset(c->d_packed, 0, 3 * (size_t)km * c->stride * sizeof(float));
  for (int i = 0; i < 9 && e == hipSuccess; ++i) e = hipEventCreate(&c->ev[i]);
  if (e != hipSuccess) {
    g_create_error = std::string("device setup failed: ") + hipGetErrorString(e);
    dpmm_destroy(ctx.release());
    return DPMM_E_DEVICE;
  }
  *out = ctx.release();
  return DPMM_OK;
}

void dpmm_destroy(dpmm_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) hipStreamSynchronize(ctx->stream);
  else hipDeviceSynchronize();
  for (auto& b : ctx->bufs) hipFree(b.p);
  if (ctx->d_perm) hipFree(ctx->d_perm);
  if (ctx->d_zsort) hipFree(ctx->d_zsort);
  if (ctx->d_part) hipFree(ctx->d_part);
  if (ctx->d_cand) hipFree(ctx->d_cand);
  if (ctx->d_sflag) hipFree(ctx->d_sflag);
  if (ctx->d_perm_c) hipFree(ctx->d_perm_c);
  if (ctx->d_zrow_c) hipFree(ctx->d_zrow_c);
  if (ctx->d_sel) hipFree(ctx->d_sel);
  if (ctx->d_side) hipFree(ctx->d_side);
  if (ctx->h_frame) hipHostFree(ctx->h_frame);
  if (ctx->h_back) hipHostFree(ctx->h_back);
  hipFree(ctx->d_items);
  hipFree(ctx->d_logml);
  hipFree(ctx->d_mflag);
  hipFree(ctx->d_plist);
  hipHostFree(ctx->h_items);
  hipHostFree(ctx->h_lml);
  hipHostFree(ctx->h_mflag);
  hipFree(ctx->d_rb);
  hipHostFree(ctx->h_rb);
  hipHostFree(ctx->h_cnt);
  hipHostFree(ctx->h_flag);
  for (auto& e : ctx->ev)
    if (e) hipEventDestroy(e);
  delete ctx;
}

dpmm_status dpmm_init_labels(dpmm_ctx* ctx, int64_t n, int32_t* z, uint8_t* zsub) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(check_n(ctx, z, n));
  if (n > 0 && !zsub) return ctx->fail(DPMM_E_ARG, "zsub is NULL");
  DPMM_HIP(ctx, launch_init_labels(n, ctx->cfg.seed, z, zsub, ctx->stream), "init kernel");
  ctx->K = 1;
  ctx->age.assign(1, 0);
  ctx->have_stats = false;
  ctx->have_params = false;
  return DPMM_OK;
}

dpmm_status dpmm_set_state(dpmm_ctx* ctx, int32_t K, const int32_t* age) {
  if (!ctx) return DPMM_E_ARG;
  if (K < 1 || K > ctx->cfg.k_max) return ctx->fail(DPMM_E_CAPACITY, "K must lie in [1, k_max]");
  ctx->K = K;
  ctx->age.assign(K, 0);
  if (age)
    for (int k = 0; k < K; ++k) ctx->age[k] = age[k];
  ctx->have_params = false;
  ctx->have_stats = false;
  return DPMM_OK;
}

dpmm_status dpmm_get_state(dpmm_ctx* ctx, int32_t* K, int32_t* age) {
  if (!ctx || !K) return DPMM_E_ARG;
  *K = ctx->K;
  if (age)
    for (int k = 0; k < ctx->K; ++k) age[k] = ctx->age[k];
  return DPMM_OK;
}

dpmm_status dpmm_set_params(dpmm_ctx* ctx, int32_t K, const double* log_pi, const double* log_pisub,
                            const double* comp) {
  if (!ctx) return DPMM_E_ARG;
  if (!log_pi || !log_pisub || !comp) return ctx->fail(DPMM_E_ARG, "parameter array is NULL");
  if (K < 1 || K > ctx->cfg.k_max) return ctx->fail(DPMM_E_CAPACITY, "K must lie in [1, k_max]");
  const int d = ctx->d;
  const size_t P = ctx->gaussian() ? (size_t)d + (size_t)d * d : (size_t)d;
  for (int k = 0; k < K; ++k)
    if (std::isnan(log_pi[k]) || std::isnan(log_pisub[2 * k]) || std::isnan(log_pisub[2 * k + 1]))
      return ctx->fail(DPMM_E_NUMERIC, "weights must not be NaN");
  for (size_t i = 0; i < (size_t)K * 3 * P; ++i)
    if (!std::isfinite(comp[i])) return ctx->fail(DPMM_E_NUMERIC, "component parameters must be finite");
  if (ctx->K != K) ctx->age.assign(K, 0);
  ctx->K = K;
  DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_log_pi, log_pi, K * sizeof(double), hipMemcpyHostToDevice, ctx->stream), "copy");
  DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_log_pisub, log_pisub, 2 * K * sizeof(double), hipMemcpyHostToDevice, ctx->stream),
           "copy");
  if (ctx->gaussian()) {
    std::vector<double> mu((size_t)3 * K * d), sig((size_t)3 * K * d * d);
    for (int e = 0; e < 3 * K; ++e) {
      std::memcpy(&mu[(size_t)e * d], comp + e * P, d * sizeof(double));
      std::memcpy(&sig[(size_t)e * d * d], comp + e * P + d, (size_t)d * d * sizeof(double));
    }
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_mu, mu.data(), mu.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream),
             "copy");
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_sigma, sig.data(), sig.size() * sizeof(double), hipMemcpyHostToDevice,
                                 ctx->stream), "copy");
    DPMM_TRY(pack_params(ctx));
    DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    DPMM_TRY(check_device_error(ctx));
  } else {
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_log_theta, comp, (size_t)3 * K * d * sizeof(double), hipMemcpyHostToDevice,
                                 ctx->stream), "copy");
    DPMM_TRY(pack_params(ctx));
    DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  }
  return DPMM_OK;
}

dpmm_status dpmm_get_params(dpmm_ctx* ctx, double* log_pi, double* log_pisub, double* comp) {
  if (!ctx) return DPMM_E_ARG;
  if (!log_pi || !log_pisub || !comp) return ctx->fail(DPMM_E_ARG, "parameter array is NULL");
  if (!ctx->have_params) return ctx->fail(DPMM_E_STATE, "no parameters yet");
  const int K = ctx->K, d = ctx->d;
  DPMM_HIP(ctx, hipMemcpyAsync(log_pi, ctx->d_log_pi, K * sizeof(double), hipMemcpyDeviceToHost, ctx->stream), "copy");
  DPMM_HIP(ctx, hipMemcpyAsync(log_pisub, ctx->d_log_pisub, 2 * K * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
           "copy");
  if (ctx->gaussian()) {
    const size_t P = (size_t)d + (size_t)d * d;
    std::vector<double> mu((size_t)3 * K * d), sig((size_t)3 * K * d * d);
    DPMM_HIP(ctx, hipMemcpyAsync(mu.data(), ctx->d_mu, mu.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
             "copy");
    DPMM_HIP(ctx, hipMemcpyAsync(sig.data(), ctx->d_sigma, sig.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 ctx->stream), "copy");
    DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    for (int e = 0; e < 3 * K; ++e) {
      std::memcpy(comp + e * P, &mu[(size_t)e * d], d * sizeof(double));
      std::memcpy(comp + e * P + d, &sig[(size_t)e * d * d], (size_t)d * d * sizeof(double));
    }
  } else {
    DPMM_HIP(ctx, hipMemcpyAsync(comp, ctx->d_log_theta, (size_t)3 * K * d * sizeof(double), hipMemcpyDeviceToHost,
                                 ctx->stream), "copy");
    DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  }
  if (ctx->sparse()) DPMM_TRY(check_device_error(ctx));  // range checks of the sparse rows
  return DPMM_OK;
}

dpmm_status dpmm_set_stats(dpmm_ctx* ctx, int32_t K, const void* stats) {
  if (!ctx) return DPMM_E_ARG;
  if (!stats) return ctx->fail(DPMM_E_ARG, "stats is NULL");
  if (K < 1 || K > ctx->cfg.k_max) return ctx->fail(DPMM_E_CAPACITY, "K must lie in [1, k_max]");
  const int d = ctx->d;
  std::vector<long long> cnt(2 * (size_t)K);
  if (ctx->gaussian()) {
    const double* s = (const double*)stats;
    const size_t R = 1 + (size_t)d + (size_t)d * d;
    std::vector<double> mom(2 * (size_t)K * ctx->E);
    for (int g = 0; g < 2 * K; ++g) {
      const double* r = s + g * R;
      if (!(r[0] >= 0.0) || r[0] != std::floor(r[0])) return ctx->fail(DPMM_E_ARG, "counts must be whole numbers >= 0");
      cnt[g] = (long long)r[0];
      double* o = &mom[(size_t)g * ctx->E];
      for (int i = 0; i < d; ++i) o[i] = r[1 + i];
      for (int a = 0; a < d; ++a)
        for (int b = a; b < d; ++b) o[d + tri_index(a, b, d)] = r[1 + d + a * d + b];
    }
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_moments, mom.data(), mom.size() * sizeof(double), hipMemcpyHostToDevice,
                                 ctx->stream), "copy");
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_counts, cnt.data(), cnt.size() * sizeof(long long), hipMemcpyHostToDevice,
                                 ctx->stream), "copy");
  } else {
    const long long* s = (const long long*)stats;
    const size_t R = 1 + (size_t)d;
    std::vector<long long> sums(2 * (size_t)K * d);
    for (int g = 0; g < 2 * K; ++g) {
      if (s[g * R] < 0) return ctx->fail(DPMM_E_ARG, "counts must be >= 0");
      cnt[g] = s[g * R];
      for (int v = 0; v < d; ++v) sums[(size_t)g * d + v] = s[g * R + 1 + v];
    }
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_sums, sums.data(), sums.size() * sizeof(long long), hipMemcpyHostToDevice,
                                 ctx->stream), "copy");
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_counts, cnt.data(), cnt.size() * sizeof(long long), hipMemcpyHostToDevice,
                                 ctx->stream), "copy");
  }
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  if (ctx->K != K) ctx->age.assign(K, 0);
  ctx->K = K;
  ctx->have_stats = true;
  return DPMM_OK;
}

dpmm_status dpmm_get_stats(dpmm_ctx* ctx, void* stats) {
  if (!ctx) return DPMM_E_ARG;
  if (!stats) return ctx->fail(DPMM_E_ARG, "stats is NULL");
  if (!ctx->have_stats) return ctx->fail(DPMM_E_STATE, "no statistics yet");
  const int K = ctx->K, d = ctx->d;
  std::vector<long long> cnt(2 * (size_t)K);
  DPMM_HIP(ctx, hipMemcpyAsync(cnt.data(), ctx->d_counts, cnt.size() * sizeof(long long), hipMemcpyDeviceToHost,
                               ctx->stream), "copy");
  if (ctx->gaussian()) {
    std::vector<double> mom(2 * (size_t)K * ctx->E);
    DPMM_HIP(ctx, hipMemcpyAsync(mom.data(), ctx->d_moments, mom.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 ctx->stream), "copy");
    DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    double* s = (double*)stats;
    const size_t R = 1 + (size_t)d + (size_t)d * d;
    for (int g = 0; g < 2 * K; ++g) {
      double* r = s + g * R;
      const double* o = &mom[(size_t)g * ctx->E];
      r[0] = (double)cnt[g];
      for (int i = 0; i < d; ++i) r[1 + i] = o[i];
      for (int a = 0; a < d; ++a)
        for (int b = a; b < d; ++b) r[1 + d + a * d + b] = r[1 + d + b * d + a] = o[d + tri_index(a, b, d)];
    }
  } else {
    std::vector<long long> sums(2 * (size_t)K * d);
    DPMM_HIP(ctx, hipMemcpyAsync(sums.data(), ctx->d_sums, sums.size() * sizeof(long long), hipMemcpyDeviceToHost,
                                 ctx->stream), "copy");
    DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    long long* s = (long long*)stats;
    const size_t R = 1 + (size_t)d;
    for (int g = 0; g < 2 * K; ++g) {
      s[g * R] = cnt[g];
      for (int v = 0; v < d; ++v) s[g * R + 1 + v] = sums[(size_t)g * d + v];
    }
  }
  if (ctx->sparse()) DPMM_TRY(check_device_error(ctx));  // range checks of the sparse rows
  return DPMM_OK;
}

dpmm_status dpmm_loglik(dpmm_ctx* ctx, const void* x, int64_t n, float* out) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(check_n(ctx, x, n));
  if (!out && n > 0) return ctx->fail(DPMM_E_ARG, "out is NULL");
  if (!ctx->have_params) return ctx->fail(DPMM_E_STATE, "no parameters yet");
  hipError_t e =
      ctx->gaussian()
          ? launch_loglik_gauss(ctx->d, (const float*)x, n, ctx->d_packed, ctx->K, ctx->cfg.k_max, out, ctx->stream)
      : ctx->sparse()
          ? launch_loglik_csr(sparse_rows(x), n, ctx->d, ctx->d_tcl, ctx->d_tsub, ctx->d_cw, ctx->K, out, ctx->d_err,
                              ctx->stream)
          : launch_loglik_mult(ctx->d, (const int*)x, n, ctx->d_packed, ctx->K, ctx->cfg.k_max, out, ctx->stream);
  DPMM_HIP(ctx, e, "log-likelihood kernel");
  return DPMM_OK;
}

}  // extern "C"

namespace {

// First half of the label step: the cluster draw (sorted path, d >= 5) or the
// fused cluster + sub-label kernel (small d, multinomial).
dpmm_status label_phase(dpmm_ctx* ctx, const void* x, int64_t n, uint32_t t, int32_t* z, uint8_t* zsub, int* G,
                        long long* per) {
  ctx->labels_gave_stats = false;
  if (ctx->sorted_path()) {
    sorted_plan(n, ctx->K, ctx->hist_cap, G, per);
    DPMM_TRY(ensure_perm(ctx, n));
    if (ctx->d_whi) {
      DPMM_HIP(ctx, launch_label_gauss_mfma(ctx->d, ctx->cfg.precision == DPMM_BF16X3, (const float*)x, n, *G, *per,
                                            ctx->d_packed, ctx->d_whi, ctx->d_wlo, ctx->d_wbias, ctx->K,
                                            ctx->cfg.k_max, t, ctx->cfg.seed, z,
                                            ctx->d_hist, ctx->d_tot, ctx->d_perm, ctx->d_cand, ctx->d_nflag,
                                            ctx->stream, ctx->label_timing ? ctx->ev[7] : nullptr,
                                            ctx->label_timing ? ctx->ev[8] : nullptr, ctx->d_cst),
               "matrix-core label kernel");
      ctx->label_kernel_timed = ctx->label_timing && n > 0;
      return DPMM_OK;
    }
    DPMM_HIP(ctx, launch_label_gauss_z(ctx->d, (const float*)x, n, *G, *per, ctx->d_packed, ctx->K, t, ctx->cfg.seed, z,
                                       ctx->d_hist, ctx->d_tot, ctx->stream), "label kernel");
    return DPMM_OK;
  }
  hipError_t e =
      ctx->gaussian() ? launch_label_gauss(ctx->d, (const float*)x, n, ctx->d_packed, ctx->K, ctx->cfg.k_max, t,
                                           ctx->cfg.seed, z, zsub, ctx->stream)
      : ctx->sparse() ? launch_label_csr(sparse_rows(x), n, ctx->d, ctx->d_tcl, ctx->d_tsub, ctx->d_cw, ctx->K, t,
                                         ctx->cfg.seed, z, zsub, ctx->d_err, ctx->stream)
                      : launch_label_mult(ctx->d, (const int*)x, n, ctx->d_packed, ctx->K, ctx->cfg.k_max, t,
                                          ctx->cfg.seed, z, zsub, ctx->stream);
  DPMM_HIP(ctx, e, "label kernel");
  return DPMM_OK;
}

// Second half on the sorted path: sort by cluster, sub-labels, statistics.
dpmm_status sub_phase(dpmm_ctx* ctx, const void* x, int64_t n, uint32_t t, int32_t* z, uint8_t* zsub, int G,
                      long long per) {
  if (!ctx->sorted_path()) return DPMM_OK;
  DPMM_TRY(sorted_pass(ctx, x, n, true, true, t, z, zsub, G, per));
  ctx->labels_gave_stats = true;
  return DPMM_OK;
}

}  // namespace

extern "C" {

dpmm_status dpmm_sample_labels(dpmm_ctx* ctx, const void* x, int64_t n, uint32_t t, int32_t* z, uint8_t* zsub) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(check_n(ctx, x, n));
  if (n > 0 && (!z || !zsub)) return ctx->fail(DPMM_E_ARG, "z / zsub is NULL");
  if (!ctx->have_params) return ctx->fail(DPMM_E_STATE, "no parameters yet");
  int G = 0;
  long long per = 0;
  DPMM_TRY(label_phase(ctx, x, n, t, z, zsub, &G, &per));
  return sub_phase(ctx, x, n, t, z, zsub, G, per);
}

dpmm_status dpmm_suffstats(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, const uint8_t* zsub) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(check_n(ctx, x, n));
  if (n > 0 && (!z || !zsub)) return ctx->fail(DPMM_E_ARG, "z / zsub is NULL");
  if (ctx->K < 1) return ctx->fail(DPMM_E_STATE, "no clusters yet (call dpmm_init_labels or dpmm_set_state)");
  return launch_stats(ctx, x, n, z, zsub);
}

dpmm_status dpmm_sample_params(dpmm_ctx* ctx, uint32_t t) {
  if (!ctx) return DPMM_E_ARG;
  if (!ctx->have_stats) return ctx->fail(DPMM_E_STATE, "no statistics yet");
  const int K = ctx->K;
  hipLaunchKernelGGL(k_weights, dim3(1), dim3(256), 0, ctx->stream, K, ctx->cfg.alpha, ctx->d_counts, ctx->cfg.seed, t,
                     ctx->d_log_pi, ctx->d_log_pisub, ctx->d_tmp);
  DPMM_HIP(ctx, hipGetLastError(), "weights kernel");
  if (ctx->gaussian()) {
    DPMM_HIP(ctx, launch_niw_draw(K, ctx->d, ctx->cfg.k_max, prior_dev(ctx), ctx->d_counts, ctx->d_moments,
                                  ctx->d_log_pi, ctx->d_log_pisub, ctx->cfg.seed, t, ctx->d_mu, ctx->d_sigma,
                                  ctx->d_scratch, ctx->d_packed, ctx->d_logdet, ctx->d_err, ctx->stream),
             "posterior draw kernel");
    if (ctx->d_whi)
      DPMM_HIP(ctx, launch_pack_wfrag(K, ctx->d, ctx->cfg.k_max, ctx->d_packed, ctx->d_whi, ctx->d_wlo, ctx->d_wbias,
                                    ctx->d_shi, ctx->d_slo, ctx->stream),
               "fragment pack kernel");
    ctx->have_params = true;
    return DPMM_OK;
  }
  const int nch = (ctx->d + DIR_CHUNK - 1) / DIR_CHUNK;
  if (ctx->poisson()) {
    hipLaunchKernelGGL(k_pois_draw, dim3(std::min(nch * 8, 256), 3 * K), dim3(256), 0, ctx->stream, K, ctx->d,
                       ctx->d_gshape, ctx->d_grate, ctx->d_counts, ctx->d_sums, ctx->cfg.seed, t, ctx->d_log_theta);
  } else if (nch > 1) {
    hipLaunchKernelGGL(k_dir_draw_chunk, dim3(nch, 3 * K), dim3(256), 0, ctx->stream, K, ctx->d, ctx->d_beta,
                       ctx->d_sums, ctx->cfg.seed, t, ctx->d_log_theta, ctx->d_dpart);
    hipLaunchKernelGGL(k_dir_norm, dim3(nch, 3 * K), dim3(256), 0, ctx->stream, K, ctx->d, ctx->d_dpart,
                       ctx->d_log_theta);
  } else {
    hipLaunchKernelGGL(k_dir_draw, dim3(3 * K), dim3(256), 0, ctx->stream, K, ctx->d, ctx->d_beta, ctx->d_sums,
                       ctx->cfg.seed, t, ctx->d_log_theta);
  }
  DPMM_HIP(ctx, hipGetLastError(), "posterior draw kernel");
  return pack_params(ctx);
}

dpmm_status dpmm_split_merge(dpmm_ctx* ctx, const void* x, int64_t n, uint32_t t, int32_t* z, uint8_t* zsub,
                             dpmm_iter_info* info) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(check_n(ctx, x, n));
  if (n > 0 && (!z || !zsub)) return ctx->fail(DPMM_E_ARG, "z / zsub is NULL");
  if (!ctx->have_stats) return ctx->fail(DPMM_E_STATE, "no statistics yet");
  const double alpha = ctx->cfg.alpha;
  const uint64_t seed = ctx->cfg.seed;
  const int burn = ctx->cfg.burn_out;
  dpmm_iter_info local{};
  std::vector<long long> cnt;
  std::vector<double> lml;
  std::vector<std::pair<int, int>> pairs;
  std::vector<unsigned char> merge_ok;
  // Marginal likelihoods of every cluster, sub-cluster and eligible pair are
  // computed in one launch and read back with the counts and the error flag:
  // one synchronisation per iteration unless a cluster became empty.
  for (int round = 0;; ++round) {
    const int K = ctx->K;
    std::vector<LogmlItem> items(3 * K);
    for (int k = 0; k < K; ++k) {
      items[3 * k] = LogmlItem{{2 * k, 2 * k + 1, -1, -1}};
      items[3 * k + 1] = LogmlItem{{2 * k, -1, -1, -1}};
      items[3 * k + 2] = LogmlItem{{2 * k + 1, -1, -1, -1}};
    }
    pairs.clear();
    for (int k1 = 0; k1 < K; ++k1) {
      if (ctx->age[k1] < burn) continue;
      for (int k2 = k1 + 1; k2 < K; ++k2)
        if (ctx->age[k2] >= burn) {
          pairs.emplace_back(k1, k2);
          items.push_back(LogmlItem{{2 * k1, 2 * k1 + 1, 2 * k2, 2 * k2 + 1}});
        }
    }
    const int P = (int)pairs.size();
    const bool paper_form = ctx->cfg.merge_form == DPMM_MERGE_PAPER;
    // the merge tests on the device, one read-back: counts, the 3K cluster /
    // sub-cluster marginals, the pair decisions and the error flag
    if (ctx->gaussian() && P > 0 && ctx->d <= MERGE_BOUND_MAX_D) {
      // Gaussian, small d: the bound items log|Psi / 2 + C_k| after the pairs;
      // the merge bound rejects most pairs, and only the others get the union's
      // Cholesky.  (Above MERGE_BOUND_MAX_D the bound is too loose to pay for
      // its K extra factorisations on ill-conditioned covariances.)
      for (int k = 0; k < K; ++k) items.push_back(LogmlItem{{2 * k, 2 * k + 1, -1, LOGML_BOUND}});
      DPMM_TRY(logml_upload(ctx, items.data(), items.size()));
      DPMM_TRY(logml_range(ctx, 0, 3 * (size_t)K));
      DPMM_TRY(logml_range(ctx, 3 * (size_t)K + P, (size_t)K));
      DPMM_HIP(ctx, launch_merge_prune(P, ctx->d_items + 3 * K, ctx->d, prior_dev(ctx), ctx->logdet_psi, ctx->lam_psi,
                                       ctx->d_counts, ctx->d_moments, ctx->d_logml, ctx->d_logml + 3 * K + P, alpha,
                                       paper_form, seed, t, ctx->d_mflag, ctx->d_plist, ctx->d_pcount, ctx->stream),
               "merge bound kernel");
      DPMM_HIP(ctx, launch_logml_gauss(P, ctx->d_items, ctx->d, prior_dev(ctx), ctx->logdet_psi, ctx->d_counts,
                                       ctx->d_moments, ctx->d_scratch, ctx->d_logml, ctx->d_err, ctx->stream,
                                       ctx->d_plist, ctx->d_pcount, 3 * K),
               "log marginal likelihood kernel");
      DPMM_HIP(ctx, launch_merge_decide(P, ctx->d_items + 3 * K, ctx->d_counts, ctx->d_logml, ctx->d_logml + 3 * K,
                                        alpha, paper_form, seed, t, ctx->d_mflag, ctx->stream, ctx->d_plist,
                                        ctx->d_pcount), "merge test kernel");
    } else {
      DPMM_TRY(logml_launch(ctx, items.data(), items.size()));
      DPMM_HIP(ctx, launch_merge_decide(P, ctx->d_items + 3 * K, ctx->d_counts, ctx->d_logml, ctx->d_logml + 3 * K,
                                        alpha, paper_form, seed, t, ctx->d_mflag, ctx->stream), "merge test kernel");
    }
    DPMM_HIP(ctx, launch_pack_readback(K, P, ctx->d_counts, ctx->d_logml, ctx->d_mflag, ctx->d_err, ctx->d_rb,
                                       ctx->stream), "read-back kernel");
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->h_rb, ctx->d_rb, readback_bytes(K, P), hipMemcpyDeviceToHost, ctx->stream),
             "copy read-back");
    DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
    const long long* rb_cnt = reinterpret_cast<const long long*>(ctx->h_rb + 8);
    const double* rb_lml = reinterpret_cast<const double*>(ctx->h_rb + 8 + 16 * (size_t)K);
    const unsigned char* rb_m = ctx->h_rb + 8 + 40 * (size_t)K;
    cnt.assign(rb_cnt, rb_cnt + 2 * (size_t)K);
    lml.assign(rb_lml, rb_lml + 3 * (size_t)K);
    merge_ok.assign(rb_m, rb_m + P);
    const int flag = (int)*reinterpret_cast<const long long*>(ctx->h_rb);
    if (flag) return flag_fail(ctx, flag);
    // delete empty clusters (stable), then start over with the new K
    int kept = 0;
    std::vector<int> newidx(K, -1);
    for (int k = 0; k < K; ++k)
      if (cnt[2 * k] + cnt[2 * k + 1] > 0) newidx[k] = kept++;
    if (kept == 0) return ctx->fail(DPMM_E_STATE, "every cluster is empty");
    if (kept == K) break;
    if (round > 0) return ctx->fail(DPMM_E_STATE, "empty clusters remain after compaction");
    std::vector<RelabelEntry> tab(2 * K);
    std::vector<int> age;
    for (int k = 0; k < K; ++k) {
      tab[2 * k] = RelabelEntry{newidx[k] < 0 ? 0 : newidx[k], 0};
      tab[2 * k + 1] = tab[2 * k];
      if (newidx[k] >= 0) age.push_back(ctx->age[k]);
    }
    DPMM_TRY(apply_relabel(ctx, tab, n, t, z, zsub));
    ctx->K = kept;
    ctx->age = age;
    local.removed = K - kept;
    DPMM_TRY(launch_stats(ctx, x, n, z, zsub));
  }
  const int K = ctx->K;
  std::vector<double> lml_cluster(K);
  for (int k = 0; k < K; ++k) lml_cluster[k] = lml[3 * k];
  // splits (Sec. 2.3 eq. HastingsRatioSplit)
  std::vector<char> touched(K, 0);
  std::vector<int> split_slot(K, -1);
  int new_slot = K;
  for (int k = 0; k < K; ++k) {
    if (ctx->age[k] < burn) continue;
    const long long nl = cnt[2 * k], nr = cnt[2 * k + 1];
    if (nl == 0 || nr == 0) continue;
    const double lh = std::log(alpha) + std::lgamma((double)nl) + lml[3 * k + 1] + std::lgamma((double)nr) +
                      lml[3 * k + 2] - std::lgamma((double)(nl + nr)) - lml[3 * k];
    const double u = uniform_d(rng_block(seed, t, (uint32_t)k, TAG_SPLIT, 0).x);
    if (std::log(u) < lh) {
      if (new_slot >= ctx->cfg.k_max) continue;  // capacity: the split is not taken
      split_slot[k] = new_slot++;
      touched[k] = 1;
    }
  }
  local.splits = new_slot - K;
  // merges among clusters not split (Sec. 4.1 eq. sample_merges), lexicographic
  std::vector<int> merged_into(K, -1);  // k2 -> k1
  std::vector<char> is_merge_target(K, 0);
  for (size_t p = 0; p < pairs.size(); ++p) {
    const int k1 = pairs[p].first, k2 = pairs[p].second;
    if (touched[k1] || touched[k2]) continue;
    if (merge_ok[p]) {  // the test of k_merge_decide
      touched[k1] = touched[k2] = 1;
      merged_into[k2] = k1;
      is_merge_target[k1] = 1;
      ++local.merges;
    }
  }
  // relabel and compact
  if (local.splits > 0 || local.merges > 0) {
    const int K2 = new_slot;
    std::vector<int> final_idx(K2, -1);
    int kept = 0;
    for (int s = 0; s < K2; ++s)
      if (!(s < K && merged_into[s] >= 0)) final_idx[s] = kept++;
    std::vector<RelabelEntry> tab(2 * K);
    std::vector<int> age(kept, 0);
    for (int k = 0; k < K; ++k) {
      if (split_slot[k] >= 0) {
        tab[2 * k] = RelabelEntry{final_idx[k], 3};
        tab[2 * k + 1] = RelabelEntry{final_idx[split_slot[k]], 3};
      } else if (merged_into[k] >= 0) {
        tab[2 * k] = tab[2 * k + 1] = RelabelEntry{final_idx[merged_into[k]], 2};
      } else if (is_merge_target[k]) {
        tab[2 * k] = tab[2 * k + 1] = RelabelEntry{final_idx[k], 1};
      } else {
        tab[2 * k] = RelabelEntry{final_idx[k], 0};
        tab[2 * k + 1] = RelabelEntry{final_idx[k], 0};
        age[final_idx[k]] = ctx->age[k];
      }
    }
    DPMM_TRY(apply_relabel(ctx, tab, n, t, z, zsub));
    ctx->K = kept;
    ctx->age = age;
    DPMM_TRY(launch_stats(ctx, x, n, z, zsub));
    std::vector<LogmlItem> fitems(kept);
    for (int k = 0; k < kept; ++k) fitems[k] = LogmlItem{{2 * k, 2 * k + 1, -1, -1}};
    cnt.assign(2 * (size_t)kept, 0);
    DPMM_HIP(ctx, hipMemcpyAsync(cnt.data(), ctx->d_counts, cnt.size() * sizeof(long long), hipMemcpyDeviceToHost,
                                 ctx->stream), "copy counts");
    int flag = 0;
    DPMM_TRY(logml(ctx, fitems, lml_cluster, &flag));
    if (flag) return flag_fail(ctx, flag);
  }
  local.K = ctx->K;
  local.logpost = log_posterior(ctx, cnt, lml_cluster);
  ctx->have_params = false;  // parameters refer to the clusters before the moves
  if (info) {
    info->K = local.K;
    info->splits = local.splits;
    info->merges = local.merges;
    info->removed = local.removed;
    info->logpost = local.logpost;
  }
  return DPMM_OK;
}

dpmm_status dpmm_step(dpmm_ctx* ctx, const void* x, int64_t n, uint32_t t, int32_t* z, uint8_t* zsub,
                      dpmm_iter_info* info) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(check_n(ctx, x, n));
  if (n > 0 && (!z || !zsub)) return ctx->fail(DPMM_E_ARG, "z / zsub is NULL");
  if (ctx->K < 1) return ctx->fail(DPMM_E_STATE, "no clusters yet (call dpmm_init_labels)");
  if (!ctx->have_stats) DPMM_TRY(launch_stats(ctx, x, n, z, zsub));
  DPMM_HIP(ctx, hipEventRecord(ctx->ev[0], ctx->stream), "event");
  DPMM_TRY(dpmm_sample_params(ctx, t));
  DPMM_HIP(ctx, hipEventRecord(ctx->ev[1], ctx->stream), "event");
  int G = 0;
  long long per = 0;
  ctx->label_timing = true;
  ctx->label_kernel_timed = false;
  const dpmm_status lp = label_phase(ctx, x, n, t, z, zsub, &G, &per);
  ctx->label_timing = false;
  DPMM_TRY(lp);
  DPMM_HIP(ctx, hipEventRecord(ctx->ev[2], ctx->stream), "event");
  // the sorted path records ev[3] between its sort and its statistics kernel
  ctx->timing = ctx->sorted_path();
  const dpmm_status sp = sub_phase(ctx, x, n, t, z, zsub, G, per);
  ctx->timing = false;
  DPMM_TRY(sp);
  if (!ctx->sorted_path()) DPMM_HIP(ctx, hipEventRecord(ctx->ev[3], ctx->stream), "event");
  if (!ctx->labels_gave_stats) DPMM_TRY(launch_stats(ctx, x, n, z, zsub));
  DPMM_HIP(ctx, hipEventRecord(ctx->ev[4], ctx->stream), "event");
  dpmm_iter_info local{};
  DPMM_TRY(dpmm_split_merge(ctx, x, n, t, z, zsub, &local));
  DPMM_HIP(ctx, hipEventRecord(ctx->ev[5], ctx->stream), "event");
  dpmm_learned_info li{};
  if (ctx->lm > 0) {
    DPMM_TRY(learned_move(ctx, x, n, t, z, zsub, nullptr, &li));
    local.K = ctx->K;
  }
  DPMM_HIP(ctx, hipEventRecord(ctx->ev[6], ctx->stream), "event");
  for (auto& a : ctx->age) ++a;
  if (info) {
    *info = local;
    info->learned_kind = li.kind;
    info->learned_accepted = li.accepted;
    DPMM_HIP(ctx, hipEventSynchronize(ctx->ev[6]), "event sync");
    hipEventElapsedTime(&info->ms_learned, ctx->ev[5], ctx->ev[6]);
    hipEventElapsedTime(&info->ms_params, ctx->ev[0], ctx->ev[1]);
    hipEventElapsedTime(&info->ms_labels, ctx->ev[1], ctx->ev[2]);
    hipEventElapsedTime(&info->ms_sort, ctx->ev[2], ctx->ev[3]);
    hipEventElapsedTime(&info->ms_stats, ctx->ev[3], ctx->ev[4]);
    hipEventElapsedTime(&info->ms_splitmerge, ctx->ev[4], ctx->ev[5]);
    info->ms_label_kernel = info->ms_labels;
    if (ctx->label_kernel_timed) hipEventElapsedTime(&info->ms_label_kernel, ctx->ev[7], ctx->ev[8]);
  }
  return DPMM_OK;
}

}  // extern "C"
