// User-level run of the sampler (the paper's fit interface, Sec. 3.4): a run
// of iterations with a per-iteration trace, the final weights and
// parameters, the normalised mutual information against ground-truth labels
// when they are given, and checkpoint files from which a run resumes bit for
// bit.  Host code over the C ABI of api.cpp; every O(N) step runs in its
// kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "ctx.hpp"

using namespace dpmm;
using namespace dpmm::host;

namespace {

// dense ids 0..m-1 of the distinct values of v (in order of first appearance)
int dense_ids(const int32_t* v, int64_t n, std::vector<int>& id) {
  std::unordered_map<int32_t, int> m;
  m.reserve(1024);
  id.resize((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    auto it = m.find(v[i]);
    if (it == m.end()) it = m.emplace(v[i], (int)m.size()).first;
    id[(size_t)i] = it->second;
  }
  return (int)m.size();
}

}  // namespace

extern "C" {

// NMI with the arithmetic-mean normalisation I(a; b) / ((H(a) + H(b)) / 2),
// from the contingency table of the two labelings (1 when both are constant).
dpmm_status dpmm_nmi(const int32_t* a, const int32_t* b, int64_t n, double* out) {
  if (!out || n < 0 || (n > 0 && (!a || !b))) return DPMM_E_ARG;
  if (n == 0) {
    *out = 1.0;
    return DPMM_OK;
  }
  std::vector<int> ia, ib;
  const int ka = dense_ids(a, n, ia), kb = dense_ids(b, n, ib);
  std::vector<double> pa(ka, 0.0), pb(kb, 0.0);
  std::unordered_map<long long, long long> joint;
  joint.reserve((size_t)std::min<long long>((long long)ka * kb, 1 << 20));
  for (int64_t i = 0; i < n; ++i) {
    pa[ia[(size_t)i]] += 1.0;
    pb[ib[(size_t)i]] += 1.0;
    ++joint[(long long)ia[(size_t)i] * kb + ib[(size_t)i]];
  }
  const double N = (double)n;
  double ha = 0.0, hb = 0.0, mi = 0.0;
  for (double c : pa) ha -= (c / N) * std::log(c / N);
  for (double c : pb) hb -= (c / N) * std::log(c / N);
  for (const auto& kv : joint) {
    const double p = (double)kv.second / N;
    const double qa = pa[(size_t)(kv.first / kb)] / N, qb = pb[(size_t)(kv.first % kb)] / N;
    mi += p * (std::log(p) - std::log(qa * qb));
  }
  *out = ha + hb == 0.0 ? 1.0 : mi / (0.5 * (ha + hb));
  return DPMM_OK;
}

}  // extern "C"

namespace {

// ---- checkpoint file: a fixed header, then the arrays it announces, all
// little-endian as in memory
constexpr char CKPT_MAGIC[8] = {'D', 'P', 'M', 'M', 'C', 'K', 'P', 'T'};
constexpr uint32_t CKPT_VERSION = 1;

struct CkptHeader {
  char magic[8];
  uint32_t version;
  int32_t family, d, k_max, burn_out, precision, merge_form, learned;
  uint64_t seed;
  double alpha, kappa, nu;
  int64_t n;
  uint32_t t;          // the last iteration the state has completed
  int32_t K;
  int64_t n_mlp;       // network parameters that follow (0 without the learned proposal)
  int32_t adam_t;
  uint32_t train_counter;
  double prior_sum;    // sum of the prior arrays (m, psi or beta): a check that the prior matches
};

double prior_sum(const dpmm_ctx* ctx) {
  double s = 0.0;
  for (double v : ctx->m) s += v;
  for (double v : ctx->psi) s += v;
  for (double v : ctx->beta) s += v;
  for (double v : ctx->gshape) s += v;
  for (double v : ctx->grate) s += 2.0 * v;
  return s;
}

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) fclose(f);
  }
};

}  // namespace

extern "C" {

dpmm_status dpmm_save_checkpoint(dpmm_ctx* ctx, const char* path, int64_t n, uint32_t t, const int32_t* z,
                                 const uint8_t* zsub) {
  if (!ctx) return DPMM_E_ARG;
  if (!path) return ctx->fail(DPMM_E_ARG, "path is NULL");
  DPMM_TRY(check_n(ctx, z, n));
  if (n > 0 && !zsub) return ctx->fail(DPMM_E_ARG, "zsub is NULL");
  if (ctx->K < 1) return ctx->fail(DPMM_E_STATE, "no clusters yet");
  CkptHeader h{};
  std::memcpy(h.magic, CKPT_MAGIC, 8);
  h.version = CKPT_VERSION;
  h.family = ctx->cfg.family;
  h.d = ctx->d;
  h.k_max = ctx->cfg.k_max;
  h.burn_out = ctx->cfg.burn_out;
  h.precision = ctx->cfg.precision;
  h.merge_form = ctx->cfg.merge_form;
  h.learned = ctx->cfg.learned;
  h.seed = ctx->cfg.seed;
  h.alpha = ctx->cfg.alpha;
  h.kappa = ctx->cfg.kappa;
  h.nu = ctx->cfg.nu;
  h.n = n;
  h.t = t;
  h.K = ctx->K;
  h.n_mlp = ctx->lm > 0 ? ctx->n_mlp : 0;
  h.adam_t = ctx->adam_t;
  h.train_counter = ctx->train_counter;
  h.prior_sum = prior_sum(ctx);
  std::vector<int32_t> zh((size_t)n);
  std::vector<uint8_t> sh((size_t)n);
  std::vector<float> mlp((size_t)h.n_mlp * 3);
  if (n > 0) {
    DPMM_HIP(ctx, hipMemcpyAsync(zh.data(), z, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream),
             "copy labels");
    DPMM_HIP(ctx, hipMemcpyAsync(sh.data(), zsub, (size_t)n, hipMemcpyDeviceToHost, ctx->stream), "copy sub-labels");
  }
  if (h.n_mlp > 0) {
    const size_t np = (size_t)h.n_mlp;
    DPMM_HIP(ctx, hipMemcpyAsync(mlp.data(), ctx->d_p, np * sizeof(float), hipMemcpyDeviceToHost, ctx->stream), "copy");
    DPMM_HIP(ctx, hipMemcpyAsync(mlp.data() + np, ctx->d_am, np * sizeof(float), hipMemcpyDeviceToHost, ctx->stream),
             "copy");
    DPMM_HIP(ctx, hipMemcpyAsync(mlp.data() + 2 * np, ctx->d_av, np * sizeof(float), hipMemcpyDeviceToHost,
                                 ctx->stream), "copy");
  }
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  const std::string tmp = std::string(path) + ".tmp";
  {
    File f;
    f.f = fopen(tmp.c_str(), "wb");
    if (!f.f) return ctx->fail(DPMM_E_ARG, "cannot open " + tmp + " for writing");
    bool ok = fwrite(&h, sizeof h, 1, f.f) == 1;
    ok = ok && fwrite(ctx->age.data(), sizeof(int32_t), ctx->age.size(), f.f) == ctx->age.size();
    ok = ok && (n == 0 || fwrite(zh.data(), sizeof(int32_t), zh.size(), f.f) == zh.size());
    ok = ok && (n == 0 || fwrite(sh.data(), 1, sh.size(), f.f) == sh.size());
    ok = ok && (mlp.empty() || fwrite(mlp.data(), sizeof(float), mlp.size(), f.f) == mlp.size());
    ok = ok && fflush(f.f) == 0;
    if (!ok) return ctx->fail(DPMM_E_ARG, "writing " + tmp + " failed");
  }
  if (rename(tmp.c_str(), path) != 0) return ctx->fail(DPMM_E_ARG, std::string("cannot rename to ") + path);
  return DPMM_OK;
}

dpmm_status dpmm_load_checkpoint(dpmm_ctx* ctx, const char* path, int64_t n, uint32_t* t, int32_t* z,
                                 uint8_t* zsub) {
  if (!ctx) return DPMM_E_ARG;
  if (!path || !t) return ctx->fail(DPMM_E_ARG, "path / t is NULL");
  DPMM_TRY(check_n(ctx, z, n));
  if (n > 0 && !zsub) return ctx->fail(DPMM_E_ARG, "zsub is NULL");
  File f;
  f.f = fopen(path, "rb");
  if (!f.f) return ctx->fail(DPMM_E_ARG, std::string("cannot open ") + path);
  CkptHeader h{};
  if (fread(&h, sizeof h, 1, f.f) != 1 || std::memcmp(h.magic, CKPT_MAGIC, 8) != 0 || h.version != CKPT_VERSION)
    return ctx->fail(DPMM_E_ARG, std::string(path) + " is not a checkpoint of this version");
  if (h.family != ctx->cfg.family || h.d != ctx->d || h.seed != ctx->cfg.seed || h.alpha != ctx->cfg.alpha ||
      h.burn_out != ctx->cfg.burn_out || h.precision != ctx->cfg.precision || h.merge_form != ctx->cfg.merge_form ||
      h.learned != ctx->cfg.learned || h.kappa != ctx->cfg.kappa || h.nu != ctx->cfg.nu ||
      h.prior_sum != prior_sum(ctx))
    return ctx->fail(DPMM_E_ARG, "the checkpoint was written under another configuration");
  if (h.n != n) return ctx->fail(DPMM_E_SHAPE, "the checkpoint holds " + std::to_string(h.n) + " points");
  if (h.K < 1 || h.K > ctx->cfg.k_max) return ctx->fail(DPMM_E_CAPACITY, "the checkpoint's K exceeds k_max");
  if (h.n_mlp != (ctx->lm > 0 ? ctx->n_mlp : 0)) return ctx->fail(DPMM_E_ARG, "network size mismatch");
  std::vector<int32_t> age((size_t)h.K);
  std::vector<int32_t> zh((size_t)n);
  std::vector<uint8_t> sh((size_t)n);
  std::vector<float> mlp((size_t)h.n_mlp * 3);
  bool ok = fread(age.data(), sizeof(int32_t), age.size(), f.f) == age.size();
  ok = ok && (n == 0 || fread(zh.data(), sizeof(int32_t), zh.size(), f.f) == zh.size());
  ok = ok && (n == 0 || fread(sh.data(), 1, sh.size(), f.f) == sh.size());
  ok = ok && (mlp.empty() || fread(mlp.data(), sizeof(float), mlp.size(), f.f) == mlp.size());
  if (!ok) return ctx->fail(DPMM_E_ARG, std::string(path) + " is truncated");
  for (int32_t v : zh)
    if (v < 0 || v >= h.K) return ctx->fail(DPMM_E_ARG, "a label in the checkpoint lies outside [0, K)");
  for (uint8_t v : sh)
    if (v > 1) return ctx->fail(DPMM_E_ARG, "a sub-label in the checkpoint is not 0 or 1");
  if (n > 0) {
    DPMM_HIP(ctx, hipMemcpyAsync(z, zh.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream),
             "copy labels");
    DPMM_HIP(ctx, hipMemcpyAsync(zsub, sh.data(), (size_t)n, hipMemcpyHostToDevice, ctx->stream), "copy sub-labels");
  }
  if (h.n_mlp > 0) {
    const size_t np = (size_t)h.n_mlp;
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_p, mlp.data(), np * sizeof(float), hipMemcpyHostToDevice, ctx->stream), "copy");
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_am, mlp.data() + np, np * sizeof(float), hipMemcpyHostToDevice, ctx->stream),
             "copy");
    DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_av, mlp.data() + 2 * np, np * sizeof(float), hipMemcpyHostToDevice,
                                 ctx->stream), "copy");
    ctx->adam_t = h.adam_t;
    ctx->train_counter = h.train_counter;
    ctx->weights_fresh = false;
  }
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  DPMM_TRY(dpmm_set_state(ctx, h.K, age.data()));
  *t = h.t;
  return DPMM_OK;
}

dpmm_status dpmm_fit(dpmm_ctx* ctx, const void* x, int64_t n, const dpmm_fit_options* opt, int32_t* z, uint8_t* zsub,
                     dpmm_iter_info* trace, double* seconds) {
  if (!ctx) return DPMM_E_ARG;
  if (!opt) return ctx->fail(DPMM_E_ARG, "opt is NULL");
  DPMM_TRY(check_n(ctx, x, n));
  if (n > 0 && (!z || !zsub)) return ctx->fail(DPMM_E_ARG, "z / zsub is NULL");
  if (opt->t0 < 1 || opt->iters < 0) return ctx->fail(DPMM_E_ARG, "t0 must be >= 1 and iters >= 0");
  if (opt->train_every < 0) return ctx->fail(DPMM_E_ARG, "train_every must be >= 0");
  if (opt->train_every > 0 && ctx->lm == 0) return ctx->fail(DPMM_E_STATE, "training needs the learned proposal");
  for (int32_t j = 0; j < opt->iters; ++j) {
    const uint32_t t = opt->t0 + (uint32_t)j;
    const auto a = std::chrono::steady_clock::now();
    dpmm_iter_info info{};
    DPMM_TRY(dpmm_step(ctx, x, n, t, z, zsub, &info));
    if (opt->train_every > 0 && t % (uint32_t)opt->train_every == 0 && t <= (uint32_t)opt->train_until)
      DPMM_TRY(dpmm_mlp_train(ctx, x, n, z, zsub, opt->train_steps, opt->train_batch, opt->train_lr, nullptr));
    if (trace) trace[j] = info;
    if (seconds) seconds[j] = std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
  }
  return DPMM_OK;
}

}  // extern "C"
