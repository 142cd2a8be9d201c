// Parameter kernels (float64 on the device): Sec. 4.1 steps (a)-(d).
//
//   k_weights        (a) and (b): Dirichlet cluster and sub-cluster weights
//                    as normalised Gamma draws.
//   k_niw_draw       (c) and (d), Gaussian: NIW posterior from the
//                    sufficient statistics and Bartlett's construction of the
//                    covariance draw, one workgroup per component, followed by
//                    the component's float32 scoring record.
//   k_dir_draw       (c) and (d), multinomial: Dirichlet posterior draw.
//   k_pack_gauss     float32 scoring record per component: Cholesky of Sigma,
//                    whitener W = L^-1, constant log w - 1/2 log|Sigma| - d/2 log 2pi.
//   k_pack_mult      float32 record: log w and log theta.
//
// Work here is O(K d^3) per iteration; one workgroup per component keeps every
// matrix of a component on one CU, in LDS for d <= 64 (the dependent
// accesses of Cholesky columns and triangular solves then cost LDS latency,
// not HBM latency), with the triangular solves and Cholesky columns parallel
// over rows.
#include "kernels.hpp"
#include "linalg.hpp"
#include "wave64.hpp"

namespace dpmm {

using namespace wave64;

namespace {

__device__ double block_reduce_max(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ double block_reduce_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int tri_index(int a, int b, int d) {
  // packed upper triangle (a <= b), row-major: row a starts at a*d - a(a-1)/2
  return a * d - (a * (a - 1)) / 2 + (b - a);
}

}  // namespace

// Every log-gamma draw of the step on a thread of its own (the K + 1 of the
// cluster weights, then the 2K of the sub-cluster weights, into tmp), then the
// normalisations; tmp holds at least 3K + 1 doubles.
__global__ void k_weights(int K, double alpha, const long long* __restrict__ counts, uint64_t seed,
                          uint32_t t, double* __restrict__ log_pi, double* __restrict__ log_pisub,
                          double* __restrict__ tmp) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double mx = -INFINITY;
  for (int q = tid; q <= 3 * K; q += blockDim.x) {
    double lg;
    if (q <= K) {
      const double shape = q < K ? (double)(counts[2 * q] + counts[2 * q + 1]) : alpha;
      lg = log_gamma_draw(seed, t, (uint32_t)q, TAG_WEIGHTS, 0, shape);
      mx = fmax(mx, lg);
    } else {
      const int r = q - (K + 1), k = r >> 1, h = r & 1;
      lg = log_gamma_draw(seed, t, (uint32_t)k, TAG_SUBWEIGHTS, (uint32_t)h, (double)counts[2 * k + h] + 0.5 * alpha);
    }
    tmp[q] = lg;
  }
  // the draws are read by other threads below: release them to the device
  // scope before the reduction's barriers and acquire after
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  mx = block_reduce_max(mx, red);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double s = 0.0;
  for (int j = tid; j <= K; j += blockDim.x) s += exp(tmp[j] - mx);
  s = block_reduce_sum(s, red);
  const double lse = mx + log(s);
  for (int j = tid; j < K; j += blockDim.x) log_pi[j] = tmp[j] - lse;
  for (int k = tid; k < K; k += blockDim.x) {
    const double l0 = tmp[K + 1 + 2 * k], l1 = tmp[K + 2 + 2 * k];
    const double m = fmax(l0, l1);
    const double l = m + log(exp(l0 - m) + exp(l1 - m));
    log_pisub[2 * k] = l0 - l;
    log_pisub[2 * k + 1] = l1 - l;
  }
}

// Per-component float64 workspace: three d x d matrices and a d-vector, in
// LDS when they fit (d <= NIW_LDS_MAX_D), else in the component's slot of the
// global scratch buffer.
struct Work {
  double *M0, *M1, *M2, *v;
};

__device__ __forceinline__ Work workspace(double* lds, double* scratch, int e, int d) {
  double* base = d <= NIW_LDS_MAX_D ? lds : scratch + (size_t)e * NIW_SCRATCH(d);
  Work w;
  w.M0 = base;
  w.M1 = base + d * d;
  w.M2 = base + 2 * d * d;
  w.v = base + 3 * d * d;
  return w;
}

// Factor Sigma (in G) = G G^T in place, W = G^-1 (lower) into Wm, and write the
// float32 scoring record of a component with log weight lw.
__device__ void pack_record(double* G, double* Wm, int d, double lw, const double* mu, float* rec,
                            double* logdet_out, int* err, int* flag, double* red) {
  const int tid = threadIdx.x;
  if (!wg_cholesky(G, d, flag)) {
    if (tid == 0) atomicOr(err, 2);
  }
  wg_lower_inverse(G, Wm, d);
  double ld = 0.0;
  for (int i = tid; i < d; i += blockDim.x) ld += log(G[i * d + i]);
  ld = 2.0 * block_reduce_sum(ld, red);
  __syncthreads();
  const int stride = gauss_rec_stride(d);
  if (tid == 0) {
    rec[0] = (float)(lw - 0.5 * ld - 0.5 * d * 1.8378770664093453);
    rec[1] = rec[2] = rec[3] = 0.0f;
    *logdet_out = ld;
  }
  for (int i = tid; i < d; i += blockDim.x) rec[4 + i] = (float)mu[i];
  for (int r = 0; r < d; ++r) {
    const int row0 = r * (r + 1) / 2;
    for (int col = tid; col <= r; col += blockDim.x) rec[4 + d + row0 + col] = (float)Wm[r * d + col];
  }
  for (int idx = 4 + d + d * (d + 1) / 2 + tid; idx < stride; idx += blockDim.x) rec[idx] = 0.0f;
}

__device__ __forceinline__ int record_slot(int k, int c, int k_max) { return c == 0 ? k : k_max + 2 * k + (c - 1); }

// One workgroup per component e = 3k + c: NIW posterior from the statistics,
// Bartlett draw of (mu, Sigma), then the float32 scoring record.  Writes
// mu[e][d], sigma[e][d][d] (float64), the record and log|Sigma|.
__global__ void k_niw_draw(int K, int d, int k_max, NiwPriorDev prior, const long long* __restrict__ counts,
                           const double* __restrict__ moments, const double* __restrict__ log_pi,
                           const double* __restrict__ log_pisub, uint64_t seed, uint32_t t,
                           double* __restrict__ mu_out, double* __restrict__ sigma_out,
                           double* __restrict__ scratch, float* __restrict__ packed,
                           double* __restrict__ logdet_out, int* __restrict__ err) {
  extern __shared__ double lds_w[];
  __shared__ double red[256];
  __shared__ int flag;
  __shared__ double sh_n;
  const int e = blockIdx.x;
  if (e >= 3 * K) return;
  const int k = e / 3, c = e % 3;
  const int tid = threadIdx.x;
  const int E = d + d * (d + 1) / 2;
  Work w = workspace(lds_w, scratch, e, d);
  double* L = w.M0;
  double* A = w.M1;
  double* F = w.M2;
  double* eps = w.v;
  double* mn = mu_out + (size_t)e * d;  // m_n staged in the output row
  const int s0 = c == 0 ? 2 * k : 2 * k + (c - 1);
  const int s1 = c == 0 ? 2 * k + 1 : -1;
  const double* M0 = moments + (size_t)s0 * E;
  const double* M1 = s1 >= 0 ? moments + (size_t)s1 * E : nullptr;
  if (tid == 0) sh_n = (double)counts[s0] + (s1 >= 0 ? (double)counts[s1] : 0.0);
  __syncthreads();
  const double n = sh_n, kn = prior.kappa + n, nun = prior.nu + n;
  // m_n = (kappa m + s) / kappa_n
  for (int i = tid; i < d; i += blockDim.x) {
    const double s = M0[i] + (M1 ? M1[i] : 0.0);
    mn[i] = (prior.kappa * prior.m[i] + s) / kn;
  }
  // Psi_n = Psi + C + (kappa n / kappa_n)(xbar - m)(xbar - m)^T, C = S - n xbar xbar^T
  for (int idx = tid; idx < d * d; idx += blockDim.x) {
    const int i = idx / d, j = idx % d;
    double v = prior.psi[idx];
    if (n > 0.0) {
      const int a = i < j ? i : j, b = i < j ? j : i;
      const double S = M0[d + tri_index(a, b, d)] + (M1 ? M1[d + tri_index(a, b, d)] : 0.0);
      const double si = M0[i] + (M1 ? M1[i] : 0.0);
      const double sj = M0[j] + (M1 ? M1[j] : 0.0);
      const double xi = si / n, xj = sj / n;
      v += (S - n * xi * xj) + (prior.kappa * n / kn) * (xi - prior.m[i]) * (xj - prior.m[j]);
    }
    L[idx] = v;
  }
  __syncthreads();
  if (!wg_cholesky(L, d, &flag)) {
    if (tid == 0) atomicOr(err, 1);
  }
  // Bartlett factor A (lower): A[i][j] ~ N(0,1) for i > j, A[i][i] = sqrt(chi2(nu_n - i))
  const int nq_off = d * (d - 1) / 2;
  for (int idx = tid; idx < d * d; idx += blockDim.x) {
    const int i = idx / d, j = idx % d;
    double v = 0.0;
    if (j < i) {
      v = normal_draw(seed, t, (uint32_t)e, TAG_NIW, (uint32_t)(i * (i - 1) / 2 + j));
    } else if (j == i) {
      const double lg = log_gamma_draw(seed, t, (uint32_t)e, TAG_NIW, (uint32_t)(nq_off + i), 0.5 * (nun - i));
      v = exp(0.5 * (0.69314718055994531 + lg));
    }
    A[idx] = v;
  }
  for (int q = tid; q < d; q += blockDim.x)
    eps[q] = normal_draw(seed, t, (uint32_t)e, TAG_NIW, (uint32_t)(nq_off + d + q));
  __syncthreads();
  // F = L A^-T
  for (int idx = tid; idx < d * d; idx += blockDim.x) F[idx] = L[idx];
  __syncthreads();
  wg_right_solve_lower_t(F, A, d);
  // mu = m_n + F eps / sqrt(kappa_n)
  const double rs = 1.0 / sqrt(kn);
  for (int r = tid; r < d; r += blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < d; ++q) s += F[r * d + q] * eps[q];
    mn[r] += s * rs;
  }
  // Sigma = F F^T (into L's storage and the output)
  double* sig = sigma_out + (size_t)e * d * d;
  for (int idx = tid; idx < d * d; idx += blockDim.x) {
    const int i = idx / d, j = idx % d;
    if (j < i) continue;
    double s = 0.0;
    for (int q = 0; q < d; ++q) s += F[i * d + q] * F[j * d + q];
    sig[i * d + j] = s;
    sig[j * d + i] = s;
    L[i * d + j] = s;
    L[j * d + i] = s;
  }
  __syncthreads();
  const double lw = c == 0 ? log_pi[k] : log_pisub[2 * k + (c - 1)];
  pack_record(L, A, d, lw, mn, packed + (size_t)record_slot(k, c, k_max) * gauss_rec_stride(d),
              logdet_out + e, err, &flag, red);
}

constexpr int NIW_BIG_THREADS = 512;

// k_niw_draw for 64 < d <= NIW_BIG_MAX_D: one workgroup of 512 threads per
// component with one d x d float64 matrix resident in LDS (row stride d + 1),
// reused in place by every stage: Psi_n -> L = chol(Psi_n) -> F = L A^-T (the
// Bartlett factor A from the component's global scratch, eight columns at a
// time) -> Sigma = F F^T (4 x 4 register tiles) -> G = chol(Sigma) -> W = G^-1,
// the factorisations, the solve and the inverse in eight-column panels (two
// barriers per panel).  Same random draws and outputs as k_niw_draw.
__global__ __launch_bounds__(NIW_BIG_THREADS) void k_niw_draw_lds(
    int K, int d, int k_max, NiwPriorDev prior, const long long* __restrict__ counts,
    const double* __restrict__ moments, const double* __restrict__ log_pi, const double* __restrict__ log_pisub,
    uint64_t seed, uint32_t t, double* __restrict__ mu_out, double* __restrict__ sigma_out,
    double* __restrict__ scratch, float* __restrict__ packed, double* __restrict__ logdet_out, int* __restrict__ err) {
  extern __shared__ double M[];  // [d][d + 1]
  __shared__ double colbuf[2][NIW_BIG_MAX_D], eps[NIW_BIG_MAX_D], red[NIW_BIG_THREADS];
  __shared__ double apan[PNL * NIW_BIG_MAX_D];  // a panel of A's columns, then the inverse's products
  __shared__ int flag;
  __shared__ double sh_n;
  const int e = blockIdx.x;
  if (e >= 3 * K) return;
  const int k = e / 3, c = e % 3;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int tx = tid & 31, ty = tid >> 5, nty = nt >> 5;
  const int ld = d + 1;
  const int E = d + d * (d + 1) / 2;
  double* At = scratch + (size_t)e * NIW_SCRATCH(d);  // A^T: row j holds column j of A
  double* mn = mu_out + (size_t)e * d;                // m_n staged in the output row
  const int s0 = c == 0 ? 2 * k : 2 * k + (c - 1);
  const int s1 = c == 0 ? 2 * k + 1 : -1;
  const double* M0 = moments + (size_t)s0 * E;
  const double* M1 = s1 >= 0 ? moments + (size_t)s1 * E : nullptr;
  if (tid == 0) sh_n = (double)counts[s0] + (s1 >= 0 ? (double)counts[s1] : 0.0);
  __syncthreads();
  const double n = sh_n, kn = prior.kappa + n, nun = prior.nu + n;
  // m_n = (kappa m + s) / kappa_n
  for (int i = tid; i < d; i += nt) {
    const double sv = M0[i] + (M1 ? M1[i] : 0.0);
    mn[i] = (prior.kappa * prior.m[i] + sv) / kn;
  }
  // Psi_n = Psi + C + (kappa n / kappa_n)(xbar - m)(xbar - m)^T, C = S - n xbar xbar^T
  for (int idx = tid; idx < d * d; idx += nt) {
    const int i = idx / d, j = idx % d;
    double v = prior.psi[idx];
    if (n > 0.0) {
      const int a = i < j ? i : j, b = i < j ? j : i;
      const double S = M0[d + tri_index(a, b, d)] + (M1 ? M1[d + tri_index(a, b, d)] : 0.0);
      const double si = M0[i] + (M1 ? M1[i] : 0.0);
      const double sj = M0[j] + (M1 ? M1[j] : 0.0);
      const double xi = si / n, xj = sj / n;
      v += (S - n * xi * xj) + (prior.kappa * n / kn) * (xi - prior.m[i]) * (xj - prior.m[j]);
    }
    M[i * ld + j] = v;
  }
  // Bartlett factor (A[i][j] ~ N(0,1) for i > j, A[i][i] = sqrt(chi2(nu_n - i))), stored transposed
  const int nq_off = d * (d - 1) / 2;
  for (int idx = tid; idx < d * d; idx += nt) {
    const int j = idx / d, i = idx % d;  // At[j][i] = A[i][j]
    double v = 0.0;
    if (j < i) {
      v = normal_draw(seed, t, (uint32_t)e, TAG_NIW, (uint32_t)(i * (i - 1) / 2 + j));
    } else if (j == i) {
      const double lg = log_gamma_draw(seed, t, (uint32_t)e, TAG_NIW, (uint32_t)(nq_off + i), 0.5 * (nun - i));
      v = exp(0.5 * (0.69314718055994531 + lg));
    }
    At[idx] = v;
  }
  for (int q = tid; q < d; q += nt) eps[q] = normal_draw(seed, t, (uint32_t)e, TAG_NIW, (uint32_t)(nq_off + d + q));
  __threadfence_block();
  __syncthreads();
  if (!wg_cholesky_panel(M, d, ld, &flag)) {
    if (tid == 0) atomicOr(err, 1);
  }
  // F = L A^-T in place (panels of eight columns of A staged in LDS)
  wg_right_solve_lt_panel(M, d, ld, At, apan, colbuf[0]);
  // mu = m_n + F eps / sqrt(kappa_n)
  const double rs = 1.0 / sqrt(kn);
  for (int r = tid; r < d; r += nt) {
    double sv = 0.0;
    for (int q = 0; q < d; ++q) sv += M[r * ld + q] * eps[q];
    mn[r] += sv * rs;
  }
  // Sigma = F F^T: thread u owns the 4 x 4 tiles u and u + nt of the upper block triangle
  const int nb = (d + 3) / 4, ntile = nb * (nb + 1) / 2;
  double acc[2][4][4];
  int tI[2], tJ[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int u = tid + h * nt, a = 0;
    tI[h] = tJ[h] = -1;
    if (u < ntile) {
      while (u >= nb - a) {
        u -= nb - a;
        ++a;
      }
      tI[h] = a;
      tJ[h] = a + u;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[h][i][j] = 0.0;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (tI[h] < 0) continue;
    int ra[4], rb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ra[i] = min(4 * tI[h] + i, d - 1) * ld;
      rb[i] = min(4 * tJ[h] + i, d - 1) * ld;
    }
    for (int q = 0; q < d; ++q) {
      double fa[4], fb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        fa[i] = M[ra[i] + q];
        fb[i] = M[rb[i] + q];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[h][i][j] = fma(fa[i], fb[j], acc[h][i][j]);
    }
  }
  __syncthreads();  // every read of F is done
  double* sig = sigma_out + (size_t)e * d * d;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (tI[h] < 0) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int a = 4 * tI[h] + i, b = 4 * tJ[h] + j;
        if (a < d && b < d && (tI[h] < tJ[h] || i <= j)) {
          const double v = acc[h][i][j];
          sig[a * d + b] = v;
          sig[b * d + a] = v;
          M[a * ld + b] = v;
          M[b * ld + a] = v;
        }
      }
  }
  __syncthreads();
  // G = chol(Sigma), log|Sigma|, W = G^-1, the float32 record
  if (!wg_cholesky_panel(M, d, ld, &flag)) {
    if (tid == 0) atomicOr(err, 2);
  }
  double lds = 0.0;
  for (int i = tid; i < d; i += nt) lds += log(M[i * ld + i]);
  lds = 2.0 * block_reduce_sum(lds, red);
  wg_lower_inverse_panel(M, d, ld, apan);
  const double lw = c == 0 ? log_pi[k] : log_pisub[2 * k + (c - 1)];
  float* rec = packed + (size_t)record_slot(k, c, k_max) * gauss_rec_stride(d);
  const int stride = gauss_rec_stride(d);
  if (tid == 0) {
    rec[0] = (float)(lw - 0.5 * lds - 0.5 * d * 1.8378770664093453);
    rec[1] = rec[2] = rec[3] = 0.0f;
    logdet_out[e] = lds;
  }
  for (int i = tid; i < d; i += nt) rec[4 + i] = (float)mn[i];
  for (int r = ty; r < d; r += nty) {
    const int row0 = r * (r + 1) / 2;
    for (int cc = tx; cc <= r; cc += 32) rec[4 + d + row0 + cc] = (float)M[r * ld + cc];
  }
  for (int idx = 4 + d + d * (d + 1) / 2 + tid; idx < stride; idx += nt) rec[idx] = 0.0f;
}

// k_niw_draw for d <= D (D in {16, 32, 64}) with two waves per component and
// a single workgroup barrier.  Wave 0 owns the matrices: lane i holds row i of
// each d x d matrix of the draw, padded to D rows with an identity block
// (pivots 1, no coupling to the d x d block), in registers; pivots travel by
// v_readlane and broadcast columns and rows through LDS.  Wave 1 meanwhile
// draws the Bartlett factor, its diagonal reciprocals and the mean's normals
// into LDS.  The random draws are those of k_niw_draw; the float64 arithmetic
// follows it except for the pivots (refined reciprocal square roots), the
// reciprocals taken ahead of the triangular solves and the order of the sums
// in Sigma = F F^T and log|Sigma|.
template <int D>
__global__ __launch_bounds__(128) void k_niw_draw_wave(int K, int d, int k_max, NiwPriorDev prior,
                                                       const long long* __restrict__ counts,
                                                       const double* __restrict__ moments,
                                                       const double* __restrict__ log_pi,
                                                       const double* __restrict__ log_pisub, uint64_t seed,
                                                       uint32_t t, double* __restrict__ mu_out,
                                                       double* __restrict__ sigma_out, float* __restrict__ packed,
                                                       double* __restrict__ logdet_out, int* __restrict__ err) {
  constexpr int LD = D + 1;
  constexpr int ED = D + D * (D + 1) / 2;
  __shared__ double sm[D * LD];  // Bartlett factor A, then F, then G
  __shared__ double sst[ED];     // the component's summed statistics (wave 0)
  static_assert(D % 4 == 0, "Sigma is formed four columns at a time");
  __shared__ double rdiag[D];    // 1 / A[j][j], then 1 / G[j][j]
  __shared__ double seps[D];     // the mean's normals
  const int e = blockIdx.x;
  if (e >= 3 * K) return;
  const int k = e / 3, c = e % 3;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool live = lane < d;
  const int E = d + d * (d + 1) / 2;
  const int s0 = c == 0 ? 2 * k : 2 * k + (c - 1);
  const int s1 = c == 0 ? 2 * k + 1 : -1;
  const double n = (double)counts[s0] + (s1 >= 0 ? (double)counts[s1] : 0.0);
  const double kn = prior.kappa + n, nun = prior.nu + n;
  const int nq_off = d * (d - 1) / 2;
  if (wave == 1) {
    // Bartlett factor A (lower): A[i][j] ~ N(0,1) for i > j,
    // A[i][i] = sqrt(chi2(nu_n - i)); identity in the padding
    if (lane < D)
      for (int row = 0; row < D; ++row) sm[row * LD + lane] = row == lane ? 1.0 : 0.0;
    wave_sync();
    for (int q = lane; q < nq_off; q += 64) {
      int i = (int)((1.0 + sqrt(1.0 + 8.0 * (double)q)) * 0.5);  // q = i (i - 1) / 2 + j, 0 <= j < i
      while (i * (i - 1) / 2 > q) --i;
      while ((i + 1) * i / 2 <= q) ++i;
      const int j = q - i * (i - 1) / 2;
      sm[i * LD + j] = normal_draw(seed, t, (uint32_t)e, TAG_NIW, (uint32_t)q);
    }
    double a = 1.0;
    if (live) {
      const double lg =
          log_gamma_draw(seed, t, (uint32_t)e, TAG_NIW, (uint32_t)(nq_off + lane), 0.5 * (nun - lane));
      a = exp(0.5 * (0.69314718055994531 + lg));
      sm[lane * LD + lane] = a;
    }
    if (lane < D) {
      rdiag[lane] = 1.0 / a;
      seps[lane] = live ? normal_draw(seed, t, (uint32_t)e, TAG_NIW, (uint32_t)(nq_off + d + lane)) : 0.0;
    }
  }
  double r[D];
  double diag = 1.0, mu_i = 0.0;
  if (wave == 0) {
    const double* M0 = moments + (size_t)s0 * E;
    const double* M1 = s1 >= 0 ? moments + (size_t)s1 * E : M0;
    // one round of loads: the summed statistics into LDS, the prior's row into r
#pragma unroll
    for (int i = 0; i < (ED + 63) / 64; ++i) {
      // unconditional loads (M1 is M0 when there is no second segment), then selected
      const int q = lane + 64 * i, qc = q < E ? q : 0;
      const double a0 = M0[qc], a1 = M1[qc];
      if (q < E) sst[q] = a0 + (s1 >= 0 ? a1 : 0.0);
    }
#pragma unroll
    for (int j = 0; j < D; ++j) r[j] = (live && j < d) ? prior.psi[lane * d + j] : 0.0;
    const double mi = live ? prior.m[lane] : 0.0;
    wave_sync();
    const double si = live ? sst[lane] : 0.0;
    const double mni = (prior.kappa * mi + si) / kn;
    const double xi = n > 0.0 ? si / n : 0.0;
    const double cm = prior.kappa * n / kn;
    // row of Psi_n = Psi + C + (kappa n / kappa_n)(xbar - m)(xbar - m)^T
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double xj = readlane_d(xi, j), mj = readlane_d(mi, j);
      const bool in = live && j < d;
      const int a = lane < j ? lane : j, b = lane < j ? j : lane;
      const int ti = in ? d + tri_index(a, b, d) : 0;
      const double ps = r[j];
      const double v = n > 0.0 ? ps + ((sst[ti] - n * xi * xj) + cm * (xi - mi) * (xj - mj)) : ps;
      r[j] = in ? v : (j == lane ? 1.0 : 0.0);
    }
    if (!wave_cholesky<D>(r, lane, diag) && lane == 0) atomicOr(err, 1);
    __syncthreads();
    // F = L A^-T, row by row: F[i][j] *= 1 / A[j][j], then F[i][q] -= F[i][j] A[q][j] (q > j)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      issue_fence();
      r[j] *= rdiag[j];
#pragma unroll
      for (int q = j + 1; q < D; ++q) r[q] = fma(-r[j], sm[q * LD + j], r[q]);
    }
    // mu = m_n + F eps / sqrt(kappa_n)
    {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < D; ++q) acc = fma(r[q], seps[q], acc);
      mu_i = mni + acc * (1.0 / sqrt(kn));
      if (live) mu_out[(size_t)e * d + lane] = mu_i;
    }
    // Sigma = F F^T: row `lane` against every row of F (in LDS), four rows at a time
    wave_sync();
    if (lane < D) {
#pragma unroll
      for (int q = 0; q < D; ++q) sm[lane * LD + q] = r[q];
    }
    wave_sync();
    // (the row of Sigma stays in registers for its Cholesky factorisation)
    double* sig = sigma_out + (size_t)e * d * d;
    double sg[D];
#pragma unroll
    for (int j = 0; j < D; j += 4) {
      issue_fence();
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      if (j < d) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
          a0 = fma(r[q], sm[j * LD + q], a0);
          a1 = fma(r[q], sm[(j + 1) * LD + q], a1);
          a2 = fma(r[q], sm[(j + 2) * LD + q], a2);
          a3 = fma(r[q], sm[(j + 3) * LD + q], a3);
        }
        if (live) {
          sig[lane * d + j] = a0;
          if (j + 1 < d) sig[lane * d + j + 1] = a1;
          if (j + 2 < d) sig[lane * d + j + 2] = a2;
          if (j + 3 < d) sig[lane * d + j + 3] = a3;
        }
      }
      sg[j] = a0;
      sg[j + 1] = a1;
      sg[j + 2] = a2;
      sg[j + 3] = a3;
    }
    // the scoring record: Sigma = G G^T, W = G^-1, log|Sigma|
#pragma unroll
    for (int j = 0; j < D; ++j) r[j] = (live && j < d) ? sg[j] : (j == lane ? 1.0 : 0.0);
    if (!wave_cholesky<D>(r, lane, diag) && lane == 0) atomicOr(err, 2);
    wave_sync();
    if (lane < D) {
#pragma unroll
      for (int q = 0; q < D; ++q) sm[lane * LD + q] = r[q];
      rdiag[lane] = 1.0 / diag;
    }
    wave_sync();
    // W = G^-1 by columns: lane c owns column c and runs the forward
    // substitution w[r] = (delta_rc - sum_{k<r} G[r][k] w[k]) / G[r][r] with the
    // rows of G read as LDS broadcasts (w[k] = 0 for k < c adds nothing)
#pragma unroll
    for (int rr = 0; rr < D; ++rr) {
      issue_fence();
      double acc = rr == lane ? 1.0 : 0.0;
#pragma unroll
      for (int kk = 0; kk < rr; ++kk) acc = fma(-sm[rr * LD + kk], r[kk], acc);
      r[rr] = acc * rdiag[rr];
    }
  } else {
    __syncthreads();
  }
  if (wave != 0) return;
  const double ld = 2.0 * wave_sum(live ? log(diag) : 0.0);
  const double lw = c == 0 ? log_pi[k] : log_pisub[2 * k + (c - 1)];
  const int stride = gauss_rec_stride(d);
  float* rec = packed + (size_t)record_slot(k, c, k_max) * stride;
  if (lane == 0) {
    rec[0] = (float)(lw - 0.5 * ld - 0.5 * d * 1.8378770664093453);
    rec[1] = rec[2] = rec[3] = 0.0f;
    logdet_out[e] = ld;
  }
  if (live) {
    rec[4 + lane] = (float)mu_i;
    // column `lane` of W: W[i][lane] for lane <= i < d
    float* wc = rec + 4 + d + lane;
#pragma unroll
    for (int i = 0; i < D; ++i)
      if (i >= lane && i < d) wc[i * (i + 1) / 2] = (float)r[i];
  }
  for (int idx = 4 + d + d * (d + 1) / 2 + lane; idx < stride; idx += 64) rec[idx] = 0.0f;
}

// One workgroup per component: log theta ~ log Dir(beta + c).
__global__ void k_dir_draw(int K, int V, const double* __restrict__ beta,
                           const long long* __restrict__ sums, uint64_t seed, uint32_t t,
                           double* __restrict__ log_theta) {
  __shared__ double red[256];
  const int e = blockIdx.x;
  if (e >= 3 * K) return;
  const int k = e / 3, c = e % 3;
  const int s0 = c == 0 ? 2 * k : 2 * k + (c - 1);
  const int s1 = c == 0 ? 2 * k + 1 : -1;
  double* out = log_theta + (size_t)e * V;
  double mx = -INFINITY;
  for (int v = threadIdx.x; v < V; v += blockDim.x) {
    const double cnt = (double)sums[(size_t)s0 * V + v] + (s1 >= 0 ? (double)sums[(size_t)s1 * V + v] : 0.0);
    const double lg = log_gamma_draw(seed, t, (uint32_t)e, TAG_DIRTHETA, (uint32_t)v, beta[v] + cnt);
    out[v] = lg;
    mx = fmax(mx, lg);
  }
  mx = block_reduce_max(mx, red);
  double s = 0.0;
  for (int v = threadIdx.x; v < V; v += blockDim.x) s += exp(out[v] - mx);
  s = block_reduce_sum(s, red);
  const double lse = mx + log(s);
  __syncthreads();
  for (int v = threadIdx.x; v < V; v += blockDim.x) out[v] -= lse;
}

// The Dirichlet draw of a large vocabulary over a grid of (word chunk,
// component): the chunk's log-Gamma variates, and the chunk's maximum and
// sum of exp(variate - maximum) into part[e][chunk]; k_dir_norm then
// subtracts each component's log-sum-exp, taken over the chunks in order.
__global__ void k_dir_draw_chunk(int K, int V, const double* __restrict__ beta, const long long* __restrict__ sums,
                                 uint64_t seed, uint32_t t, double* __restrict__ log_theta, double* __restrict__ part) {
  __shared__ double red[256];
  const int e = blockIdx.y, ch = blockIdx.x, nch = gridDim.x;
  if (e >= 3 * K) return;
  const int k = e / 3, c = e % 3;
  const int s0 = c == 0 ? 2 * k : 2 * k + (c - 1);
  const int s1 = c == 0 ? 2 * k + 1 : -1;
  double* out = log_theta + (size_t)e * V;
  const int v0 = ch * DIR_CHUNK, v1 = min(V, v0 + DIR_CHUNK);
  double mx = -INFINITY;
  for (int v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
    const double cnt = (double)sums[(size_t)s0 * V + v] + (s1 >= 0 ? (double)sums[(size_t)s1 * V + v] : 0.0);
    const double lg = log_gamma_draw(seed, t, (uint32_t)e, TAG_DIRTHETA, (uint32_t)v, beta[v] + cnt);
    out[v] = lg;
    mx = fmax(mx, lg);
  }
  mx = block_reduce_max(mx, red);
  double sm = 0.0;
  for (int v = v0 + threadIdx.x; v < v1; v += blockDim.x) sm += exp(out[v] - mx);
  sm = block_reduce_sum(sm, red);
  if (threadIdx.x == 0) {
    part[((size_t)e * nch + ch) * 2] = mx;
    part[((size_t)e * nch + ch) * 2 + 1] = sm;
  }
}

__global__ void k_dir_norm(int K, int V, const double* __restrict__ part, double* __restrict__ log_theta) {
  const int e = blockIdx.y, ch = blockIdx.x, nch = gridDim.x;
  if (e >= 3 * K) return;
  const double* p = part + (size_t)e * nch * 2;
  double mx = -INFINITY;
  for (int j = 0; j < nch; ++j) mx = fmax(mx, p[2 * j]);
  double sm = 0.0;
  for (int j = 0; j < nch; ++j) sm += p[2 * j + 1] * exp(p[2 * j] - mx);
  const double lse = mx + log(sm);
  double* out = log_theta + (size_t)e * V;
  const int v1 = min(V, (ch + 1) * DIR_CHUNK);
  for (int v = ch * DIR_CHUNK + threadIdx.x; v < v1; v += blockDim.x) out[v] -= lse;
}

// Poisson family, a grid of (word chunk, component): log lambda_v for
// lambda_v ~ Gamma(a_v + c_v, b_v + n) (shape, rate), the Gamma(a_v + c_v, 1)
// variate of draw v of (3k + c, TAG_DIRTHETA) divided by the rate.
__global__ void k_pois_draw(int K, int V, const double* __restrict__ shape, const double* __restrict__ rate,
                            const long long* __restrict__ counts, const long long* __restrict__ sums, uint64_t seed,
                            uint32_t t, double* __restrict__ log_lambda) {
  const int e = blockIdx.y;
  if (e >= 3 * K) return;
  const int k = e / 3, c = e % 3;
  const int s0 = c == 0 ? 2 * k : 2 * k + (c - 1);
  const int s1 = c == 0 ? 2 * k + 1 : -1;
  const double n = (double)counts[s0] + (s1 >= 0 ? (double)counts[s1] : 0.0);
  double* out = log_lambda + (size_t)e * V;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) {
    const double cnt = (double)sums[(size_t)s0 * V + v] + (s1 >= 0 ? (double)sums[(size_t)s1 * V + v] : 0.0);
    out[v] = log_gamma_draw(seed, t, (uint32_t)e, TAG_DIRTHETA, (uint32_t)v, shape[v] + cnt) - log(rate[v] + n);
  }
}

// Pack component e = 3k + c from its float64 (mu, Sigma): record slot k
// (cluster) or k_max + 2k + h (sub-cluster).
__global__ void k_pack_gauss(int K, int d, int k_max, const double* __restrict__ log_pi,
                             const double* __restrict__ log_pisub, const double* __restrict__ mu,
                             const double* __restrict__ sigma, double* __restrict__ scratch,
                             float* __restrict__ packed, double* __restrict__ logdet_out,
                             int* __restrict__ err) {
  extern __shared__ double lds_w[];
  __shared__ int flag;
  __shared__ double red[256];
  const int e = blockIdx.x;
  if (e >= 3 * K) return;
  const int k = e / 3, c = e % 3;
  Work w = workspace(lds_w, scratch, e, d);
  const double* sig = sigma + (size_t)e * d * d;
  for (int idx = threadIdx.x; idx < d * d; idx += blockDim.x) w.M0[idx] = sig[idx];
  __syncthreads();
  const double lw = c == 0 ? log_pi[k] : log_pisub[2 * k + (c - 1)];
  pack_record(w.M0, w.M1, d, lw, mu + (size_t)e * d, packed + (size_t)record_slot(k, c, k_max) * gauss_rec_stride(d),
              logdet_out + e, err, &flag, red);
}

// Count families: record = (log w, log theta) (multinomial) or (log w - sum
// lambda, log lambda) (Poisson, poisson != 0): the score c + sum_v x_v rec_v
// is the component's log-likelihood without its per-point factor.
__global__ void k_pack_mult(int K, int V, int k_max, const double* __restrict__ log_pi,
                            const double* __restrict__ log_pisub, const double* __restrict__ log_theta,
                            float* __restrict__ packed, int poisson) {
  __shared__ double red[256];
  const int e = blockIdx.x;
  if (e >= 3 * K) return;
  const int k = e / 3, c = e % 3;
  const int stride = mult_rec_stride(V);
  const int slot = c == 0 ? k : k_max + 2 * k + (c - 1);
  float* rec = packed + (size_t)slot * stride;
  double lw = c == 0 ? log_pi[k] : log_pisub[2 * k + (c - 1)];
  if (poisson) {
    double s = 0.0;
    for (int v = threadIdx.x; v < V; v += blockDim.x) s += exp(log_theta[(size_t)e * V + v]);
    lw -= block_reduce_sum(s, red);
  }
  if (threadIdx.x == 0) {
    rec[0] = (float)lw;
    rec[1] = rec[2] = rec[3] = 0.0f;
  }
  for (int v = threadIdx.x; v < V; v += blockDim.x) rec[4 + v] = (float)log_theta[(size_t)e * V + v];
  for (int idx = 4 + V + threadIdx.x; idx < stride; idx += blockDim.x) rec[idx] = 0.0f;
}

hipError_t launch_niw_draw(int K, int d, int k_max, NiwPriorDev prior, const long long* counts,
                           const double* moments, const double* log_pi, const double* log_pisub, uint64_t seed,
                           uint32_t t, double* mu_out, double* sigma_out, double* scratch, float* packed,
                           double* logdet_out, int* err, hipStream_t s) {
  if (K <= 0) return hipSuccess;
#define DPMM_NIW_WAVE(DD)                                                                                    \
  hipLaunchKernelGGL(k_niw_draw_wave<DD>, dim3(3 * K), dim3(128), 0, s, K, d, k_max, prior, counts, moments,  \
                     log_pi, log_pisub, seed, t, mu_out, sigma_out, packed, logdet_out, err)
  if (d <= 16)
    DPMM_NIW_WAVE(16);
  else if (d <= 32)
    DPMM_NIW_WAVE(32);
  else if (d <= 64)
    DPMM_NIW_WAVE(64);
  else if (d <= NIW_BIG_MAX_D) {
    // one d x (d + 1) float64 matrix in LDS: above 64 KB, raise the limit once
    static bool attr_set = false;
    const size_t lds = (size_t)d * (d + 1) * sizeof(double);
    if (!attr_set) {
      const hipError_t e = hipFuncSetAttribute((const void*)k_niw_draw_lds,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)((size_t)NIW_BIG_MAX_D * (NIW_BIG_MAX_D + 1) * sizeof(double)));
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    hipLaunchKernelGGL(k_niw_draw_lds, dim3(3 * K), dim3(NIW_BIG_THREADS), lds, s, K, d, k_max, prior, counts,
                       moments, log_pi, log_pisub, seed, t, mu_out, sigma_out, scratch, packed, logdet_out, err);
  } else
    hipLaunchKernelGGL(k_niw_draw, dim3(3 * K), dim3(256), niw_lds_bytes(d), s, K, d, k_max, prior, counts, moments,
                       log_pi, log_pisub, seed, t, mu_out, sigma_out, scratch, packed, logdet_out, err);
#undef DPMM_NIW_WAVE
  return hipGetLastError();
}

}  // namespace dpmm
