// Host runtime of the learned split proposal (an added form; the paper has no
// learned component): network weights and training, set features, and the
// learned Metropolis-Hastings move of include/dpmm.h.
//
// Device work: selection of a set's points, features, the MLP forward and
// backward passes (matrix cores), the per-point Bernoulli sides and their
// log-probability sums, the float64 statistics of the proposed sides, the
// marginal likelihoods and the relabelling.  Host work per move: one
// symmetric eigendecomposition of the set's d x d covariance (Householder
// tridiagonalisation and implicit QR, float64) and the O(1) accept / reject
// arithmetic on values read back; two synchronisations per move.
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "ctx.hpp"
#include "eigen.hpp"

using namespace dpmm;
using namespace dpmm::host;

namespace {

constexpr int H = MLP_HIDDEN;

struct Offsets {
  int W1, b1, W2, b2, w3, b3, n;
};

Offsets offsets(int F) {
  Offsets o;
  o.W1 = 0;
  o.b1 = F * H;
  o.W2 = o.b1 + H;
  o.b2 = o.W2 + H * H;
  o.w3 = o.b2 + H;
  o.b3 = o.w3 + H;
  o.n = o.b3 + 1;
  return o;
}

int frame_size(const dpmm_ctx* ctx) { return ctx->d + ctx->lm * ctx->d + ctx->lm; }

// Frame of a set with statistics (n, s, upper triangle U of sum x x^T):
// out = [mu (d), P (m x d), ratios (m)] as float32, with mu the mean, Sigma
// the covariance plus 1e-9 (1 + tr Sigma / d) I, eigenpairs by decreasing
// eigenvalue with each eigenvector's largest-magnitude entry positive,
// P_j = v_j / sqrt(lambda_j) and ratios_j = lambda_j / sum lambda.  Also
// returns P_0 in float64 (for the training targets' orientation).  False if
// the eigen-iteration did not converge.
bool set_frame(double n, const double* s, const double* U, int d, int m, float* out, std::vector<double>* p0) {
  std::vector<double> mu(d), A((size_t)d * d);
  for (int i = 0; i < d; ++i) mu[i] = s[i] / n;
  for (int a = 0; a < d; ++a)
    for (int b = a; b < d; ++b) {
      const double v = U[tri_index(a, b, d)] / n - mu[a] * mu[b];
      A[(size_t)a * d + b] = A[(size_t)b * d + a] = v;
    }
  double tr = 0.0;
  for (int i = 0; i < d; ++i) tr += A[(size_t)i * d + i];
  const double reg = 1e-9 * (1.0 + tr / d);
  for (int i = 0; i < d; ++i) A[(size_t)i * d + i] += reg;
  std::vector<double> w, V;
  if (!eig::sym_eigen(A, d, w, V)) return false;
  std::vector<int> order(d);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
  double total = 0.0;
  std::vector<double> lam(d);
  for (int j = 0; j < d; ++j) {
    lam[j] = std::max(w[order[j]], 1e-300);
    total += lam[j];
  }
  for (int i = 0; i < d; ++i) out[i] = (float)mu[i];
  for (int j = 0; j < m; ++j) {
    const double* vec = &V[(size_t)order[j] * d];
    int amax = 0;
    for (int i = 1; i < d; ++i)
      if (std::fabs(vec[i]) > std::fabs(vec[amax])) amax = i;
    const double scale = (vec[amax] < 0.0 ? -1.0 : 1.0) / std::sqrt(lam[j]);
    for (int i = 0; i < d; ++i) out[d + j * d + i] = (float)(vec[i] * scale);
    if (j == 0 && p0) {
      p0->resize(d);
      for (int i = 0; i < d; ++i) (*p0)[i] = vec[i] * scale;
    }
    out[d + m * d + j] = (float)(lam[j] / total);
  }
  return true;
}

dpmm_status need_learned(dpmm_ctx* ctx) {
  if (ctx->lm <= 0) return ctx->fail(DPMM_E_STATE, "the learned proposal is off (cfg.learned = 0)");
  return DPMM_OK;
}

dpmm_status ensure_sel(dpmm_ctx* ctx, int64_t n) {
  if (n > 0x7FFFFFFFLL) return ctx->fail(DPMM_E_SHAPE, "the learned proposal takes n < 2^31 points");
  if (n <= ctx->sel_cap) return DPMM_OK;
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  if (ctx->d_sel) hipFree(ctx->d_sel);
  if (ctx->d_side) hipFree(ctx->d_side);
  ctx->d_sel = nullptr;
  ctx->d_side = nullptr;
  ctx->sel_cap = 0;
  DPMM_HIP(ctx, hipMalloc(&ctx->d_sel, (size_t)n * sizeof(int)), "allocate selection");
  DPMM_HIP(ctx, hipMalloc(&ctx->d_side, (size_t)n), "allocate sides");
  ctx->sel_cap = n;
  return DPMM_OK;
}

dpmm_status ensure_weights(dpmm_ctx* ctx) {
  if (ctx->weights_fresh) return DPMM_OK;
  DPMM_HIP(ctx, launch_refresh_weights(ctx->d_p, ctx->F, ctx->Fp, ctx->d_w1t, ctx->d_w2t, ctx->d_w2, ctx->stream),
           "weight refresh kernel");
  ctx->weights_fresh = true;
  return DPMM_OK;
}

// logits of c rows whose BF16 features are in d_x16; keep_t also writes H1^T
dpmm_status forward_chunk(dpmm_ctx* ctx, int c, bool keep_t, float* logits) {
  const Offsets of = offsets(ctx->F);
  hipStream_t s = ctx->stream;
  DPMM_HIP(ctx, launch_gemm_nt(ctx->d_x16, ctx->Fp, ctx->d_w1t, ctx->Fp, c, H, ctx->Fp, ctx->d_p + of.b1, true,
                               nullptr, 0, nullptr, 0, false, ctx->d_h1, H, keep_t ? ctx->d_h1t : nullptr, MLP_CHUNK,
                               s), "layer 1 kernel");
  DPMM_HIP(ctx, launch_gemm_nt(ctx->d_h1, H, ctx->d_w2t, H, c, H, H, ctx->d_p + of.b2, true, nullptr, 0, ctx->d_h2, H,
                               false, nullptr, 0, nullptr, 0, s), "layer 2 kernel");
  DPMM_HIP(ctx, launch_out_layer(ctx->d_h2, c, ctx->d_p + of.w3, ctx->d_p + of.b3, logits, s), "output layer kernel");
  return DPMM_OK;
}

// gradient contributions of c rows (after forward_chunk with keep_t, the
// transposed features in d_x16t and targets y); accumulates into d_g and the
// loss into d_lsums[4]
dpmm_status backward_chunk(dpmm_ctx* ctx, int c, const float* y) {
  const Offsets of = offsets(ctx->F);
  hipStream_t s = ctx->stream;
  float* g = ctx->d_g;
  DPMM_HIP(ctx, launch_out_backward(ctx->d_o, y, ctx->d_h2, c, MLP_CHUNK, ctx->d_p + of.w3, ctx->d_d2, ctx->d_d2t,
                                    g + of.w3, g + of.b3, ctx->d_lsums + 4, ctx->d_red, s), "output backward kernel");
  DPMM_HIP(ctx, launch_gemm_nt(ctx->d_d2, H, ctx->d_w2, H, c, H, H, nullptr, false, ctx->d_h1, H, nullptr, 0, false,
                               ctx->d_d1, H, ctx->d_d1t, MLP_CHUNK, s), "layer 2 backward kernel");
  DPMM_HIP(ctx, launch_colsum(ctx->d_d2, H, c, H, g + of.b2, ctx->d_red, s), "bias gradient kernel");
  DPMM_HIP(ctx, launch_colsum(ctx->d_d1, H, c, H, g + of.b1, ctx->d_red, s), "bias gradient kernel");
  DPMM_HIP(ctx, launch_gemm_nt(ctx->d_h1t, MLP_CHUNK, ctx->d_d2t, MLP_CHUNK, H, H, c, nullptr, false, nullptr, 0,
                               g + of.W2, H, true, nullptr, 0, nullptr, 0, s), "W2 gradient kernel");
  DPMM_HIP(ctx, launch_gemm_nt(ctx->d_x16t, MLP_CHUNK, ctx->d_d1t, MLP_CHUNK, ctx->F, H, c, nullptr, false, nullptr,
                               0, g + of.W1, H, true, nullptr, 0, nullptr, 0, s), "W1 gradient kernel");
  return DPMM_OK;
}

dpmm_status zero_grad(dpmm_ctx* ctx) {
  DPMM_HIP(ctx, launch_zero64(ctx->d_g, (size_t)(ctx->n_mlp + 1) / 2, ctx->stream), "zero kernel");
  DPMM_HIP(ctx, launch_zero64(ctx->d_lsums, 8, ctx->stream), "zero kernel");
  return DPMM_OK;
}

// gradient of the summed loss over n FP32 feature rows (device)
dpmm_status grad_rows(dpmm_ctx* ctx, const float* X, const float* y, int64_t n) {
  DPMM_TRY(ensure_weights(ctx));
  DPMM_TRY(zero_grad(ctx));
  for (int64_t off = 0; off < n; off += MLP_CHUNK) {
    const int c = (int)std::min<int64_t>(MLP_CHUNK, n - off);
    DPMM_HIP(ctx, launch_convert(X + off * ctx->F, c, ctx->F, ctx->Fp, ctx->d_x16, ctx->d_x16t, MLP_CHUNK,
                                 ctx->stream), "convert kernel");
    DPMM_TRY(forward_chunk(ctx, c, true, ctx->d_o));
    DPMM_TRY(backward_chunk(ctx, c, y + off));
  }
  return DPMM_OK;
}

dpmm_status adam_update(dpmm_ctx* ctx, float lr) {
  ++ctx->adam_t;
  DPMM_HIP(ctx, launch_adam(ctx->d_p, ctx->d_g, ctx->d_am, ctx->d_av, ctx->n_mlp, lr, 0.9f, 0.999f, 1e-8f,
                            ctx->adam_t, ctx->stream), "Adam kernel");
  ctx->weights_fresh = false;
  return ensure_weights(ctx);
}

// read back the counts of every cluster and the moments of the given slots
// (one copy per run of consecutive slots)
dpmm_status read_set_stats(dpmm_ctx* ctx, const std::vector<int>& slots, std::vector<long long>& cnt,
                           std::vector<double>& mom) {
  const int K = ctx->K, E = ctx->E;
  cnt.assign(2 * (size_t)K, 0);
  mom.assign(slots.size() * (size_t)E, 0.0);
  DPMM_HIP(ctx, hipMemcpyAsync(cnt.data(), ctx->d_counts, cnt.size() * sizeof(long long), hipMemcpyDeviceToHost,
                               ctx->stream), "copy counts");
  for (size_t j = 0; j < slots.size();) {
    size_t r = j + 1;
    while (r < slots.size() && slots[r] == slots[r - 1] + 1) ++r;
    DPMM_HIP(ctx, hipMemcpyAsync(mom.data() + j * E, ctx->d_moments + (size_t)slots[j] * E, (r - j) * E * sizeof(double),
                                 hipMemcpyDeviceToHost, ctx->stream), "copy moments");
    j = r;
  }
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  return DPMM_OK;
}

// frame of the union of the given slots' statistics, staged in the pinned
// buffer h_frame and copied to frame row 0 (asynchronously: the caller
// synchronises before h_frame is written again)
dpmm_status upload_set_frame(dpmm_ctx* ctx, const std::vector<int>& slots, const std::vector<long long>& cnt,
                             const std::vector<double>& mom, long long* n_set) {
  const int d = ctx->d, E = ctx->E;
  std::vector<double> sum(E, 0.0);
  long long nn = 0;
  for (size_t j = 0; j < slots.size(); ++j) {
    nn += cnt[slots[j]];
    for (int e = 0; e < E; ++e) sum[e] += mom[j * E + e];
  }
  *n_set = nn;
  if (nn == 0) return ctx->fail(DPMM_E_STATE, "the set is empty");
  if (!set_frame((double)nn, sum.data(), sum.data() + d, d, ctx->lm, ctx->h_frame, nullptr))
    return ctx->fail(DPMM_E_NUMERIC, "the eigen-iteration of the set covariance did not converge");
  DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_frames, ctx->h_frame, frame_size(ctx) * sizeof(float), hipMemcpyHostToDevice,
                               ctx->stream), "copy frame");
  return DPMM_OK;
}

// stable list of the points of clusters k1 (and k2 >= 0) in d_sel; the
// number found lands in the pinned h_back->sel_count after the next
// synchronisation (check_selected compares it with the statistics)

dpmm_status select_set(dpmm_ctx* ctx, const int32_t* z, int64_t n, int k1, int k2) {
  DPMM_TRY(ensure_sel(ctx, n));
  DPMM_HIP(ctx, launch_select(z, n, k1, k2, nullptr, ctx->K, ctx->d_selcnt, ctx->d_sel, ctx->stream),
           "selection kernels");
  DPMM_HIP(ctx, hipMemcpyAsync(&ctx->h_back->sel_count, ctx->d_selcnt + SELECT_BLOCKS, sizeof(int),
                               hipMemcpyDeviceToHost, ctx->stream), "copy count");
  return DPMM_OK;
}

dpmm_status check_selected(dpmm_ctx* ctx, long long n_expect) {
  const int got = ctx->h_back->sel_count;
  if (got != n_expect)
    return ctx->fail(DPMM_E_STATE, "the statistics do not match z (" + std::to_string(got) + " labelled points, " +
                                       std::to_string(n_expect) + " counted); recompute them with dpmm_suffstats");
  return DPMM_OK;
}

void pair_of(long long p, int K, int* k1, int* k2) {
  int a = 0;
  while (p >= K - 1 - a) {
    p -= K - 1 - a;
    ++a;
  }
  *k1 = a;
  *k2 = a + 1 + (int)p;
}

double logaddexp(double a, double b) {
  const double m = std::max(a, b);
  if (m == -INFINITY) return m;
  return m + std::log(std::exp(a - m) + std::exp(b - m));
}

}  // namespace

namespace dpmm::host {

dpmm_status learned_alloc(dpmm_ctx* ctx) {
  const int m = ctx->cfg.learned;
  ctx->lm = m;
  ctx->F = 2 * m;
  ctx->Fp = (ctx->F + 15) / 16 * 16;
  const Offsets of = offsets(ctx->F);
  ctx->n_mlp = of.n;
  const size_t np = (size_t)(of.n + 1) / 2 * 2, CH = MLP_CHUNK, km = ctx->cfg.k_max;
  dpmm_ctx* c = ctx;
  hipError_t e = hipSuccess;
  auto A = [&](auto** p, size_t count) {
    if (e == hipSuccess) e = c->alloc(p, count);
  };
  A(&c->d_p, np);
  A(&c->d_g, np);
  A(&c->d_am, np);
  A(&c->d_av, np);
  A(&c->d_w1t, (size_t)H * c->Fp);
  A(&c->d_w2t, (size_t)H * H);
  A(&c->d_w2, (size_t)H * H);
  A(&c->d_x16, CH * c->Fp);
  A(&c->d_x16t, CH * c->Fp);
  A(&c->d_h1, CH * H);
  A(&c->d_h1t, CH * H);
  A(&c->d_d2, CH * H);
  A(&c->d_d2t, CH * H);
  A(&c->d_d1, CH * H);
  A(&c->d_d1t, CH * H);
  A(&c->d_h2, CH * H);
  A(&c->d_o, CH);
  A(&c->d_y, CH);
  A(&c->d_bidx, CH);
  A(&c->d_bcl, CH);
  A(&c->d_frames, (km + 1) * (size_t)frame_size(c));
  A(&c->d_flip, km);
  A(&c->d_elig, km);
  A(&c->d_lsums, 8);
  A(&c->d_red, MLP_RED_DOUBLES);
  A(&c->d_setpart, (size_t)SET_STATS_BLOCKS * 2 * (1 + c->E));
  A(&c->d_selcnt, SELECT_BLOCKS + 1);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_frame, frame_size(c) * sizeof(float), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_back, sizeof(LearnedBack), hipHostMallocDefault);
  if (e != hipSuccess) return c->hip(e, "allocate learned-proposal buffers");
  // He-uniform initial weights from Philox (tag TAG_MLPINIT), biases zero
  std::vector<float> p(np, 0.0f);
  auto fill = [&](int off, int count, int fan_in) {
    const double scale = std::sqrt(6.0 / fan_in);
    for (int q = off; q < off + count; ++q) {
      const double u = uniform_d(rng_block(c->cfg.seed, 0, (uint32_t)q, TAG_MLPINIT, 0).x);
      p[q] = (float)((2.0 * u - 1.0) * scale);
    }
  };
  fill(of.W1, c->F * H, c->F);
  fill(of.W2, H * H, H);
  fill(of.w3, H, H);
  e = hipMemcpy(c->d_p, p.data(), np * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->d_am, 0, np * sizeof(float));
  if (e == hipSuccess) e = hipMemset(c->d_av, 0, np * sizeof(float));
  if (e != hipSuccess) return c->hip(e, "initialise weights");
  c->weights_fresh = false;
  return DPMM_OK;
}

dpmm_status learned_move(dpmm_ctx* ctx, const void* x, int64_t n, uint32_t t, int32_t* z, uint8_t* zsub,
                         uint8_t* side_out, dpmm_learned_info* info) {
  DPMM_TRY(need_learned(ctx));
  DPMM_TRY(check_n(ctx, x, n));
  if (n > 0 && (!z || !zsub)) return ctx->fail(DPMM_E_ARG, "z / zsub is NULL");
  if (!ctx->have_stats) return ctx->fail(DPMM_E_STATE, "no statistics yet");
  const int K = ctx->K;
  const uint64_t seed = ctx->cfg.seed;
  const u32x4 w = rng_block(seed, t, 0, TAG_MOVE, 0);
  const double u_type = uniform_d(w.x), u_pick = uniform_d(w.y), u_acc = uniform_d(w.z);
  const bool split = K == 1 || u_type < 0.5;
  dpmm_learned_info li{};
  li.k2 = -1;
  int k1, k2 = -1;
  const long long npairs = (long long)K * (K - 1) / 2;
  if (split) {
    k1 = std::min((int)(u_pick * K), K - 1);
    li.kind = 1;
  } else {
    const long long p = std::min((long long)(u_pick * (double)npairs), npairs - 1);
    pair_of(p, K, &k1, &k2);
    li.kind = 2;
    li.k2 = k2;
  }
  li.k1 = k1;
  auto finish = [&]() {
    if (info) *info = li;
    return DPMM_OK;
  };
  if (split && K + 1 > ctx->cfg.k_max) {
    li.skipped = 2;
    return finish();
  }
  std::vector<int> slots = {2 * k1, 2 * k1 + 1};
  if (!split) {
    slots.push_back(2 * k2);
    slots.push_back(2 * k2 + 1);
  }
  std::vector<long long> cnt;
  std::vector<double> mom;
  DPMM_TRY(read_set_stats(ctx, slots, cnt, mom));
  for (int k = 0; k < K; ++k)
    if (cnt[2 * k] + cnt[2 * k + 1] == 0)
      return ctx->fail(DPMM_E_STATE, "cluster " + std::to_string(k) + " is empty (run dpmm_split_merge first)");
  long long nC = 0;
  DPMM_TRY(upload_set_frame(ctx, slots, cnt, mom, &nC));
  DPMM_TRY(select_set(ctx, z, n, k1, k2));
  unsigned char* side = side_out ? side_out : ctx->d_side;
  DPMM_TRY(ensure_weights(ctx));
  hipStream_t s = ctx->stream;
  LearnedBack* back = ctx->h_back;
  DPMM_HIP(ctx, launch_zero64(ctx->d_lsums, 8, s), "zero kernel");
  for (long long off = 0; off < nC; off += MLP_CHUNK) {
    const int c = (int)std::min<long long>(MLP_CHUNK, nC - off);
    DPMM_HIP(ctx, launch_features((const float*)x, ctx->d, n, ctx->d_sel + off, nullptr, c, ctx->d_frames, ctx->lm,
                                  ctx->F, ctx->Fp, ctx->d_x16, nullptr, 0, nullptr, s), "features kernel");
    DPMM_TRY(forward_chunk(ctx, c, false, ctx->d_o));
    DPMM_HIP(ctx, launch_proposal(ctx->d_o, n, ctx->d_sel + off, c, split ? -1 : k1, z, seed, t, side, ctx->d_lsums,
                                  ctx->d_red, s), "proposal kernel");
  }
  std::vector<LogmlItem> items;
  int a_off = 0;  // segment of side A (side == 1) within slot, slot + 1
  if (split) {
    const int slot = 2 * K;
    // the sorted-order kernels keep side h in segment slot + h; the generic one puts side A first
    a_off = partition_stats_supported(ctx->d) ? 1 : 0;
    if (partition_stats_supported(ctx->d)) {
      DPMM_TRY(ensure_part(ctx, nC));
      DPMM_HIP(ctx, launch_set_pair(ctx->d_cspan, 0, (int)nC, s), "span kernel");
      DPMM_HIP(ctx, launch_partition_stats(ctx->d, (const float*)x, n, ctx->d_sel, nC, z, k1, K, side, slot,
                                           ctx->d_counts, ctx->d_moments, ctx->d_cspan, ctx->d_part, s),
               "partition statistics kernels");
    } else
      DPMM_HIP(ctx, launch_set_stats((const float*)x, ctx->d, n, ctx->d_sel, (int)nC, side, ctx->d_setpart, slot,
                                     ctx->d_counts, ctx->d_moments, s), "partition statistics kernels");
    DPMM_HIP(ctx, hipMemcpyAsync(back->side_cnt, ctx->d_counts + slot, 2 * sizeof(long long), hipMemcpyDeviceToHost,
                                 s), "copy counts");
    items = {LogmlItem{{slot + a_off, -1, -1, -1}}, LogmlItem{{slot + 1 - a_off, -1, -1, -1}},
             LogmlItem{{2 * k1, 2 * k1 + 1, -1, -1}}};
  } else {
    items = {LogmlItem{{2 * k1, 2 * k1 + 1, -1, -1}}, LogmlItem{{2 * k2, 2 * k2 + 1, -1, -1}},
             LogmlItem{{2 * k1, 2 * k1 + 1, 2 * k2, 2 * k2 + 1}}};
  }
  DPMM_HIP(ctx, hipMemcpyAsync(back->sums, ctx->d_lsums, 4 * sizeof(double), hipMemcpyDeviceToHost, s), "copy sums");
  std::vector<double> lml;
  int flag = 0;
  DPMM_TRY(logml(ctx, items, lml, &flag));  // synchronises
  if (flag) return flag_fail(ctx, flag);
  DPMM_TRY(check_selected(ctx, nC));
  const long long nA = split ? back->side_cnt[a_off] : cnt[2 * k1] + cnt[2 * k1 + 1];
  const long long nB = split ? back->side_cnt[1 - a_off] : cnt[2 * k2] + cnt[2 * k2 + 1];
  li.n_a = nA;
  li.n_b = nB;
  // q(s): side-A points take log b, side-B points log(1 - b); q(not s) swaps them
  const double* sums = back->sums;
  li.log_q_part = logaddexp(sums[0] + sums[3], sums[1] + sums[2]);
  if (nA == 0 || nB == 0) {
    li.skipped = 1;
    return finish();
  }
  const double alpha = ctx->cfg.alpha;
  li.log_target = std::log(alpha) + std::lgamma((double)nA) + lml[0] + std::lgamma((double)nB) + lml[1] -
                  std::lgamma((double)(nA + nB)) - lml[2];
  if (split) {
    const double lq_fwd = std::log(K == 1 ? 1.0 : 0.5) - std::log((double)K) + li.log_q_part;
    const double lq_rev = std::log(0.5) - std::log((double)(K + 1) * K / 2.0);
    li.log_h = li.log_target + lq_rev - lq_fwd;
  } else {
    const double lq_fwd = std::log(0.5) - std::log((double)npairs);
    const double lq_rev = std::log(K - 1 == 1 ? 1.0 : 0.5) - std::log((double)(K - 1)) + li.log_q_part;
    li.log_h = -li.log_target + lq_rev - lq_fwd;
  }
  if (!(std::log(u_acc) < li.log_h)) return finish();
  li.accepted = 1;
  if (split) {
    DPMM_HIP(ctx, launch_apply_split(n, ctx->d_sel, (int)nC, side, K, seed, t, z, zsub, s), "apply kernel");
    ctx->age[k1] = 0;
    ctx->age.push_back(0);
    ctx->K = K + 1;
  } else {
    std::vector<RelabelEntry> tab(2 * (size_t)K);
    std::vector<int> age;
    for (int k = 0; k < K; ++k) {
      const int nk = k < k2 ? k : k - 1;
      if (k == k1) {
        tab[2 * k] = tab[2 * k + 1] = RelabelEntry{nk, 1};
      } else if (k == k2) {
        tab[2 * k] = tab[2 * k + 1] = RelabelEntry{k1, 2};
      } else {
        tab[2 * k] = tab[2 * k + 1] = RelabelEntry{nk, 0};
      }
      if (k != k2) age.push_back(k == k1 ? 0 : ctx->age[k]);
    }
    DPMM_TRY(apply_relabel(ctx, tab, n, t, z, zsub));
    ctx->K = K - 1;
    ctx->age = age;
  }
  ctx->have_params = false;
  DPMM_TRY(launch_stats(ctx, x, n, z, zsub));
  return finish();
}

}  // namespace dpmm::host

extern "C" {

int64_t dpmm_mlp_n_params(const dpmm_ctx* ctx) { return ctx && ctx->lm > 0 ? ctx->n_mlp : 0; }

dpmm_status dpmm_mlp_set_weights(dpmm_ctx* ctx, const double* params) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(need_learned(ctx));
  if (!params) return ctx->fail(DPMM_E_ARG, "params is NULL");
  std::vector<float> p((size_t)(ctx->n_mlp + 1) / 2 * 2, 0.0f);
  for (int q = 0; q < ctx->n_mlp; ++q) {
    if (!std::isfinite(params[q])) return ctx->fail(DPMM_E_NUMERIC, "weights must be finite");
    p[q] = (float)params[q];
  }
  DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_p, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice, ctx->stream),
           "copy weights");
  DPMM_HIP(ctx, launch_zero64(ctx->d_am, p.size() / 2, ctx->stream), "zero kernel");
  DPMM_HIP(ctx, launch_zero64(ctx->d_av, p.size() / 2, ctx->stream), "zero kernel");
  ctx->adam_t = 0;
  ctx->weights_fresh = false;
  DPMM_TRY(ensure_weights(ctx));
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  return DPMM_OK;
}

dpmm_status dpmm_mlp_get_weights(dpmm_ctx* ctx, double* params) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(need_learned(ctx));
  if (!params) return ctx->fail(DPMM_E_ARG, "params is NULL");
  std::vector<float> p(ctx->n_mlp);
  DPMM_HIP(ctx, hipMemcpyAsync(p.data(), ctx->d_p, p.size() * sizeof(float), hipMemcpyDeviceToHost, ctx->stream),
           "copy weights");
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  for (int q = 0; q < ctx->n_mlp; ++q) params[q] = p[q];
  return DPMM_OK;
}

dpmm_status dpmm_mlp_forward(dpmm_ctx* ctx, const float* X, int64_t n, float* logits) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(need_learned(ctx));
  if (n < 0 || n > 0x7FFFFFFFLL) return ctx->fail(DPMM_E_SHAPE, "n must lie in [0, 2^31)");
  if (n > 0 && (!X || !logits)) return ctx->fail(DPMM_E_ARG, "X / logits is NULL");
  DPMM_TRY(ensure_weights(ctx));
  for (int64_t off = 0; off < n; off += MLP_CHUNK) {
    const int c = (int)std::min<int64_t>(MLP_CHUNK, n - off);
    DPMM_HIP(ctx, launch_convert(X + off * ctx->F, c, ctx->F, ctx->Fp, ctx->d_x16, nullptr, 0, ctx->stream),
             "convert kernel");
    DPMM_TRY(forward_chunk(ctx, c, false, logits + off));
  }
  return DPMM_OK;
}

dpmm_status dpmm_mlp_grad(dpmm_ctx* ctx, const float* X, const float* y, int64_t n, double* grad, double* loss) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(need_learned(ctx));
  if (n < 0 || n > 0x7FFFFFFFLL) return ctx->fail(DPMM_E_SHAPE, "n must lie in [0, 2^31)");
  if (n > 0 && (!X || !y)) return ctx->fail(DPMM_E_ARG, "X / y is NULL");
  DPMM_TRY(grad_rows(ctx, X, y, n));
  std::vector<float> g(ctx->n_mlp);
  double l = 0.0;
  DPMM_HIP(ctx, hipMemcpyAsync(g.data(), ctx->d_g, g.size() * sizeof(float), hipMemcpyDeviceToHost, ctx->stream),
           "copy gradient");
  DPMM_HIP(ctx, hipMemcpyAsync(&l, ctx->d_lsums + 4, sizeof(double), hipMemcpyDeviceToHost, ctx->stream), "copy loss");
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  if (grad)
    for (int q = 0; q < ctx->n_mlp; ++q) grad[q] = g[q];
  if (loss) *loss = l;
  return DPMM_OK;
}

dpmm_status dpmm_mlp_adam_step(dpmm_ctx* ctx, const float* X, const float* y, int64_t n, float lr, double* loss) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(need_learned(ctx));
  if (n < 0 || n > 0x7FFFFFFFLL) return ctx->fail(DPMM_E_SHAPE, "n must lie in [0, 2^31)");
  if (n > 0 && (!X || !y)) return ctx->fail(DPMM_E_ARG, "X / y is NULL");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return ctx->fail(DPMM_E_ARG, "lr must be > 0");
  DPMM_TRY(grad_rows(ctx, X, y, n));
  DPMM_TRY(adam_update(ctx, lr));
  double l = 0.0;
  DPMM_HIP(ctx, hipMemcpyAsync(&l, ctx->d_lsums + 4, sizeof(double), hipMemcpyDeviceToHost, ctx->stream), "copy loss");
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");
  if (loss) *loss = l;
  return DPMM_OK;
}

dpmm_status dpmm_set_features(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, int32_t k1, int32_t k2,
                              float* feats, int32_t* idx, int64_t capacity, int64_t* n_set) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(need_learned(ctx));
  DPMM_TRY(check_n(ctx, x, n));
  if (n > 0 && !z) return ctx->fail(DPMM_E_ARG, "z is NULL");
  if (!n_set) return ctx->fail(DPMM_E_ARG, "n_set is NULL");
  if (!ctx->have_stats) return ctx->fail(DPMM_E_STATE, "no statistics yet");
  if (k1 < 0 || k1 >= ctx->K || k2 >= ctx->K || k2 == k1) return ctx->fail(DPMM_E_ARG, "cluster index out of range");
  std::vector<int> slots = {2 * k1, 2 * k1 + 1};
  if (k2 >= 0) {
    slots.push_back(2 * k2);
    slots.push_back(2 * k2 + 1);
  }
  std::vector<long long> cnt;
  std::vector<double> mom;
  DPMM_TRY(read_set_stats(ctx, slots, cnt, mom));
  long long nC = 0;
  DPMM_TRY(upload_set_frame(ctx, slots, cnt, mom, &nC));
  *n_set = nC;
  if (feats || idx) {
    if (capacity < nC) return ctx->fail(DPMM_E_SHAPE, "capacity is below the set size");
    DPMM_TRY(select_set(ctx, z, n, k1, k2));
    if (feats)
      DPMM_HIP(ctx, launch_features((const float*)x, ctx->d, n, ctx->d_sel, nullptr, (int)nC, ctx->d_frames, ctx->lm,
                                    ctx->F, ctx->Fp, nullptr, nullptr, 0, feats, ctx->stream), "features kernel");
    if (idx)
      DPMM_HIP(ctx, hipMemcpyAsync(idx, ctx->d_sel, (size_t)nC * sizeof(int), hipMemcpyDeviceToDevice, ctx->stream),
               "copy indices");
  }
  DPMM_HIP(ctx, hipStreamSynchronize(ctx->stream), "synchronise");  // h_frame / h_back are reused
  if (feats || idx) DPMM_TRY(check_selected(ctx, nC));
  return DPMM_OK;
}

dpmm_status dpmm_learned_move(dpmm_ctx* ctx, const void* x, int64_t n, uint32_t t, int32_t* z, uint8_t* zsub,
                              uint8_t* side_out, dpmm_learned_info* info) {
  if (!ctx) return DPMM_E_ARG;
  return learned_move(ctx, x, n, t, z, zsub, side_out, info);
}

}  // extern "C"

namespace {

// The training rows of the sampler's own sub-labels: frames and target flips
// of every cluster with age >= burn_out and two non-empty sub-clusters go to
// d_frames / d_flip, and the stable list of their points to d_sel; *n_sel is
// their number (0: nothing qualifies).
dpmm_status training_rows(dpmm_ctx* ctx, int64_t n, const int32_t* z, int* n_sel) {
  *n_sel = 0;
  const int K = ctx->K, d = ctx->d, E = ctx->E, fs = frame_size(ctx);
  std::vector<int> slots(2 * (size_t)K);
  std::iota(slots.begin(), slots.end(), 0);
  std::vector<long long> cnt;
  std::vector<double> mom;
  DPMM_TRY(read_set_stats(ctx, slots, cnt, mom));
  std::vector<float> frames((size_t)K * fs, 0.0f);
  std::vector<int> elig(K, 0), flip(K, 0);
  std::vector<int> todo;
  for (int k = 0; k < K; ++k)
    if (ctx->age[k] >= ctx->cfg.burn_out && cnt[2 * k] > 0 && cnt[2 * k + 1] > 0) todo.push_back(k);
  // frames of the eligible clusters, spread over host threads
  std::vector<char> ok(todo.size(), 1);
  auto work = [&](size_t j0, size_t step) {
    std::vector<double> sum(E), p0;
    for (size_t j = j0; j < todo.size(); j += step) {
      const int k = todo[j];
      const long long nl = cnt[2 * k], nr = cnt[2 * k + 1];
      for (int e = 0; e < E; ++e) sum[e] = mom[(size_t)(2 * k) * E + e] + mom[(size_t)(2 * k + 1) * E + e];
      if (!set_frame((double)(nl + nr), sum.data(), sum.data() + d, d, ctx->lm, frames.data() + (size_t)k * fs,
                     &p0)) {
        ok[j] = 0;
        continue;
      }
      // orientation: side l must have the larger mean first principal coordinate
      double pl = 0.0, pr = 0.0;
      for (int i = 0; i < d; ++i) {
        pl += p0[i] * mom[(size_t)(2 * k) * E + i] / (double)nl;
        pr += p0[i] * mom[(size_t)(2 * k + 1) * E + i] / (double)nr;
      }
      flip[k] = pl < pr ? 1 : 0;
      elig[k] = 1;
    }
  };
  const size_t nthreads = std::min<size_t>(todo.size(), std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  if (nthreads <= 1 || (size_t)d * d * todo.size() < 200000) {
    work(0, 1);
  } else {
    std::vector<std::thread> pool;
    for (size_t i = 0; i < nthreads; ++i) pool.emplace_back(work, i, nthreads);
    for (auto& th : pool) th.join();
  }
  for (char o : ok)
    if (!o) return ctx->fail(DPMM_E_NUMERIC, "the eigen-iteration of a cluster covariance did not converge");
  if (todo.empty()) return DPMM_OK;
  hipStream_t s = ctx->stream;
  DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_frames, frames.data(), frames.size() * sizeof(float), hipMemcpyHostToDevice, s),
           "copy frames");
  DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_elig, elig.data(), K * sizeof(int), hipMemcpyHostToDevice, s), "copy");
  DPMM_HIP(ctx, hipMemcpyAsync(ctx->d_flip, flip.data(), K * sizeof(int), hipMemcpyHostToDevice, s), "copy");
  DPMM_TRY(ensure_sel(ctx, n));
  DPMM_HIP(ctx, launch_select(z, n, -1, -1, ctx->d_elig, K, ctx->d_selcnt, ctx->d_sel, s), "selection kernels");
  DPMM_HIP(ctx, hipMemcpyAsync(&ctx->h_back->sel_count, ctx->d_selcnt + SELECT_BLOCKS, sizeof(int),
                               hipMemcpyDeviceToHost, s), "copy count");
  DPMM_HIP(ctx, hipStreamSynchronize(s), "synchronise");  // also keeps the host tables alive until copied
  *n_sel = ctx->h_back->sel_count;
  return DPMM_OK;
}

dpmm_status training_args(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, const uint8_t* zsub) {
  DPMM_TRY(need_learned(ctx));
  DPMM_TRY(check_n(ctx, x, n));
  if (n > 0 && (!z || !zsub)) return ctx->fail(DPMM_E_ARG, "z / zsub is NULL");
  if (!ctx->have_stats) return ctx->fail(DPMM_E_STATE, "no statistics yet");
  return DPMM_OK;
}

}  // namespace

extern "C" {

dpmm_status dpmm_mlp_training_set(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, const uint8_t* zsub,
                                  float* feats, float* y, int32_t* idx, int64_t capacity, int64_t* n_rows) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(training_args(ctx, x, n, z, zsub));
  if (!n_rows) return ctx->fail(DPMM_E_ARG, "n_rows is NULL");
  int n_sel = 0;
  DPMM_TRY(training_rows(ctx, n, z, &n_sel));
  *n_rows = n_sel;
  if (n_sel == 0 || (!feats && !y && !idx)) return DPMM_OK;
  if (capacity < n_sel) return ctx->fail(DPMM_E_SHAPE, "capacity is below the number of training rows");
  hipStream_t s = ctx->stream;
  if (feats)
    DPMM_HIP(ctx, launch_features((const float*)x, ctx->d, n, ctx->d_sel, z, n_sel, ctx->d_frames, ctx->lm, ctx->F,
                                  ctx->Fp, nullptr, nullptr, 0, feats, s, true), "features kernel");
  if (y) DPMM_HIP(ctx, launch_targets(ctx->d_sel, z, n_sel, zsub, ctx->d_flip, y, s, true), "targets kernel");
  if (idx)
    DPMM_HIP(ctx, hipMemcpyAsync(idx, ctx->d_sel, (size_t)n_sel * sizeof(int), hipMemcpyDeviceToDevice, s),
             "copy indices");
  DPMM_HIP(ctx, hipStreamSynchronize(s), "synchronise");
  return DPMM_OK;
}

dpmm_status dpmm_mlp_train(dpmm_ctx* ctx, const void* x, int64_t n, const int32_t* z, const uint8_t* zsub,
                           int32_t steps, int32_t batch, float lr, double* loss) {
  if (!ctx) return DPMM_E_ARG;
  DPMM_TRY(training_args(ctx, x, n, z, zsub));
  if (steps < 0) return ctx->fail(DPMM_E_ARG, "steps must be >= 0");
  if (batch < 1 || batch > MLP_CHUNK) return ctx->fail(DPMM_E_ARG, "batch must lie in [1, 65536]");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return ctx->fail(DPMM_E_ARG, "lr must be > 0");
  if (loss) *loss = NAN;
  if (steps == 0) return DPMM_OK;
  int n_sel = 0;
  DPMM_TRY(training_rows(ctx, n, z, &n_sel));
  if (n_sel == 0) return DPMM_OK;
  hipStream_t s = ctx->stream;
  const int d = ctx->d;
  DPMM_TRY(ensure_weights(ctx));
  for (int st = 0; st < steps; ++st) {
    DPMM_HIP(ctx, launch_batch_pick(ctx->d_sel, n_sel, batch, ctx->cfg.seed, ctx->train_counter++, z, ctx->d_bidx,
                                    ctx->d_bcl, s), "batch kernel");
    DPMM_HIP(ctx, launch_features((const float*)x, d, n, ctx->d_bidx, ctx->d_bcl, batch, ctx->d_frames, ctx->lm, ctx->F,
                                  ctx->Fp, ctx->d_x16, ctx->d_x16t, MLP_CHUNK, nullptr, s), "features kernel");
    DPMM_HIP(ctx, launch_targets(ctx->d_bidx, ctx->d_bcl, batch, zsub, ctx->d_flip, ctx->d_y, s), "targets kernel");
    DPMM_TRY(zero_grad(ctx));
    DPMM_TRY(forward_chunk(ctx, batch, true, ctx->d_o));
    DPMM_TRY(backward_chunk(ctx, batch, ctx->d_y));
    DPMM_TRY(adam_update(ctx, lr));
  }
  double l = 0.0;
  DPMM_HIP(ctx, hipMemcpyAsync(&l, ctx->d_lsums + 4, sizeof(double), hipMemcpyDeviceToHost, s), "copy loss");
  DPMM_HIP(ctx, hipStreamSynchronize(s), "synchronise");
  if (loss) *loss = l / batch;
  return DPMM_OK;
}

}  // extern "C"
