// Split/merge support kernels: Sec. 2.3 (split Hastings ratio, merge) and
// Sec. 4.1 (eqs. sample_splits, sample_merges), plus label bookkeeping.
//
//   k_logml_gauss  log marginal likelihood of the union of up to four
//                  sub-cluster segments under the NIW prior, one workgroup
//                  per item (float64 Cholesky of Psi_n in LDS for log|Psi_n|);
//   k_logml_gauss_wave  the same for d <= 64, one wave per item with the
//                  matrix in registers (lane i holds row i);
//   k_logml_mult   the Dirichlet-multinomial log marginal likelihood;
//   k_relabel      applies a split/merge/compaction move table to (z, zsub)
//                  in one O(N) pass;
//   k_init_labels  the one-cluster initial state.
// The O(K^2) accept/reject bookkeeping runs on the host from these values.
#include "kernels.hpp"
#include "wave64.hpp"
#include "linalg.hpp"

namespace dpmm {

using namespace wave64;

namespace {

// log Gamma as one shared (not inlined) copy: the kernels below call it several
// times each, and their code is fetched once per wave
__device__ __attribute__((noinline)) double lgamma_d(double v) { return lgamma(v); }


constexpr int BLOCK = 256;

__device__ __forceinline__ int tri_index(int a, int b, int d) {
  return a * d - (a * (a - 1)) / 2 + (b - a);
}

__device__ double reduce_sum(double v, double* red) {
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

__global__ void k_zero64(unsigned long long* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void k_set_pair(int* p, int a, int b) {
  if (threadIdx.x == 0) {
    p[0] = a;
    p[1] = b;
  }
}

__global__ void k_logml_gauss(int n_items, const LogmlItem* __restrict__ items, int d, NiwPriorDev prior,
                              double logdet_psi, const long long* __restrict__ counts,
                              const double* __restrict__ moments, double* __restrict__ scratch,
                              double* __restrict__ out, int* __restrict__ err) {
  extern __shared__ double lds_p[];
  __shared__ double red[BLOCK];
  __shared__ int flag;
  const int it = blockIdx.x;
  if (it >= n_items) return;
  const int tid = threadIdx.x;
  const int E = d + d * (d + 1) / 2;
  const LogmlItem item = items[it];
  double n = 0.0;
  for (int q = 0; q < 4; ++q)
    if (item.seg[q] >= 0) n += (double)counts[item.seg[q]];
  if (n == 0.0) {
    if (tid == 0) out[it] = 0.0;
    return;
  }
  double* P = d <= LOGML_LDS_MAX_D ? lds_p : scratch + (size_t)it * d * d;
  const double kn = prior.kappa + n, nun = prior.nu + n;
  for (int idx = tid; idx < d * d; idx += BLOCK) {
    const int i = idx / d, j = idx % d;
    const int a = i < j ? i : j, b = i < j ? j : i;
    double S = 0.0, si = 0.0, sj = 0.0;
    for (int q = 0; q < 4; ++q) {
      const int sg = item.seg[q];
      if (sg < 0) continue;
      const double* M = moments + (size_t)sg * E;
      S += M[d + tri_index(a, b, d)];
      si += M[i];
      sj += M[j];
    }
    const double xi = si / n, xj = sj / n;
    P[idx] = prior.psi[idx] + (S - n * xi * xj) + (prior.kappa * n / kn) * (xi - prior.m[i]) * (xj - prior.m[j]);
  }
  __syncthreads();
  const bool ok = wg_cholesky(P, d, &flag);
  double ld = 0.0, lg = 0.0;
  for (int i = tid; i < d; i += BLOCK) {
    ld += log(P[i * d + i]);
    // log Gamma_d(nu_n / 2) - log Gamma_d(nu / 2), term j = i + 1
    lg += lgamma_d(0.5 * nun - 0.5 * i) - lgamma_d(0.5 * prior.nu - 0.5 * i);
  }
  ld = 2.0 * reduce_sum(ld, red);
  lg = reduce_sum(lg, red);
  if (tid == 0) {
    if (!ok) atomicOr(err, 4);
    out[it] = -0.5 * n * d * 1.1447298858494002 + lg + 0.5 * prior.nu * logdet_psi - 0.5 * nun * ld +
              0.5 * d * (log(prior.kappa) - log(kn));
  }
}

// One wave per item, D >= d rows padded with an identity block (whose
// pivots are 1 and add nothing to log|Psi_n|).  Lane i builds row i of Psi_n
// (entries k <= i) from the item's statistics, staged in the wave's LDS
// buffer in one round of loads, and factors it with the wave Cholesky (pivots
// and column entries by v_readlane): no workgroup barrier.
template <int D>
__global__ __launch_bounds__(BLOCK) void k_logml_gauss_wave(int n_items, const LogmlItem* __restrict__ items, int d,
                                                            NiwPriorDev prior, double logdet_psi,
                                                            const long long* __restrict__ counts,
                                                            const double* __restrict__ moments,
                                                            double* __restrict__ out, int* __restrict__ err) {
  constexpr int ED = D + D * (D + 1) / 2;
  __shared__ double ssum[BLOCK / 64][ED];  // per wave: the item's summed statistics
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int it = blockIdx.x * (BLOCK / 64) + wave;
  if (it >= n_items) return;
  const int E = d + d * (d + 1) / 2;
  const LogmlItem item = items[it];
  const bool live = lane < d;
  // every load of the item in one round: its counts, the sum of its segments'
  // statistics (summed in segment order into the wave's LDS buffer) and the
  // prior's row of Psi (entries k <= lane)
  // (absent segments read segment 0 and add +0.0: unconditional loads, no
  // branches, so that they are all in flight together)
  const double* Mq[4];
  bool hq[4];
  double nq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    hq[q] = item.seg[q] >= 0;
    Mq[q] = moments + (size_t)(hq[q] ? item.seg[q] : 0) * E;
    const long long c = counts[hq[q] ? item.seg[q] : 0];
    nq[q] = hq[q] ? (double)c : 0.0;
  }
  double* sm = ssum[wave];
#pragma unroll
  for (int i = 0; i < (ED + 63) / 64; ++i) {
    const int e = lane + 64 * i, ec = e < E ? e : 0;
    double m[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) m[q] = Mq[q][ec];
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) v += hq[q] ? m[q] : 0.0;
    if (e < E) sm[e] = v;
  }
  double r[D];
#pragma unroll
  for (int k = 0; k < D; ++k) r[k] = (k < d && live && k <= lane) ? prior.psi[lane * d + k] : 0.0;
  double n = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) n += nq[q];
  if (n == 0.0) {
    if (lane == 0) out[it] = 0.0;
    return;
  }
  const double kn = prior.kappa + n, nun = prior.nu + n, cm = prior.kappa * n / kn;
  wave_sync();
  const double si = live ? sm[lane] : 0.0;
  const double xi = si / n;
  const double dmi = live ? xi - prior.m[lane] : 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double xk = readlane_d(xi, k), dmk = readlane_d(dmi, k);
    const bool in = k < d && live && k <= lane;
    const int tk = in ? d + k * d - (k * (k - 1)) / 2 + (lane - k) : 0;  // packed (k, lane), k <= lane
    const double v = r[k] + (sm[tk] - n * xi * xk) + cm * dmi * dmk;
    r[k] = in ? v : (k == lane ? 1.0 : 0.0);
  }
  double mydiag;
  const bool ok = wave_cholesky<D>(r, lane, mydiag);
  // log|Psi_n| = 2 sum log L_ii; log Gamma_d(nu_n / 2) - log Gamma_d(nu / 2)
  const double ld = 2.0 * wave_sum(live ? log(mydiag) : 0.0);
  const double lg = wave_sum(live ? lgamma_d(0.5 * nun - 0.5 * lane) - lgamma_d(0.5 * prior.nu - 0.5 * lane) : 0.0);
  if (lane == 0) {
    if (!ok) atomicOr(err, 4);
    out[it] = -0.5 * n * d * 1.1447298858494002 + lg + 0.5 * prior.nu * logdet_psi - 0.5 * nun * ld +
              0.5 * d * (log(prior.kappa) - log(kn));
  }
}

// Read-back of one split/merge round in a single buffer (one copy to the
// host instead of four): [int error flag, padded to 8 bytes][counts, 2K
// int64][log marginals of the 3K cluster / sub-cluster items, float64][P merge
// decisions, bytes].
__global__ void k_pack_readback(int K, int P, const long long* __restrict__ counts, const double* __restrict__ lml,
                                const unsigned char* __restrict__ mflag, const int* __restrict__ err,
                                unsigned char* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *reinterpret_cast<long long*>(out) = (long long)*err;
  long long* oc = reinterpret_cast<long long*>(out + 8);
  double* ol = reinterpret_cast<double*>(out + 8 + 16 * (size_t)K);
  unsigned char* om = out + 8 + 40 * (size_t)K;
  if (i < 2 * K)
    oc[i] = counts[i];
  else if (i < 5 * K)
    ol[i - 2 * K] = lml[i - 2 * K];
  else if (i < 5 * K + P)
    om[i - 5 * K] = mflag[i - 5 * K];
}

// Merge test of every listed pair (Sec. 4.1 eq. sample_merges; with
// paper_form = 0 the reciprocal of the split ratio of Sec. 2.3): pair p is the
// item pairs[p] = (2 k1, 2 k1 + 1, 2 k2, 2 k2 + 1) with union marginal
// lml_pair[p]; lml_cluster[3 k] is cluster k's marginal.  accept[p] = 1 when
// log u < log H_merge with u the merge uniform of (k1, k2).
__global__ void k_merge_decide(int n_pairs, const LogmlItem* __restrict__ pairs, const long long* __restrict__ counts,
                               const double* __restrict__ lml_cluster, const double* __restrict__ lml_pair,
                               double alpha, int paper_form, uint64_t seed, uint32_t t,
                               unsigned char* __restrict__ accept) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const LogmlItem it = pairs[p];
  const int k1 = it.seg[0] >> 1, k2 = it.seg[2] >> 1;
  const double n1 = (double)(counts[2 * k1] + counts[2 * k1 + 1]);
  const double n2 = (double)(counts[2 * k2] + counts[2 * k2 + 1]);
  double lh = lgamma_d(n1 + n2) - log(alpha) - lgamma_d(n1) - lgamma_d(n2) + lml_pair[p] - lml_cluster[3 * k1] -
              lml_cluster[3 * k2];
  if (paper_form)
    lh += lgamma_d(alpha) - lgamma_d(alpha + n1 + n2) + lgamma_d(0.5 * alpha + n1) + lgamma_d(0.5 * alpha + n2) -
          2.0 * lgamma_d(0.5 * alpha);
  const double u = uniform_d(rng_block(seed, t, merge_entity(k1, k2), TAG_MERGE, 0).x);
  accept[p] = log(u) < lh ? 1 : 0;
}

__global__ void k_logml_mult(int n_items, const LogmlItem* __restrict__ items, int V,
                             const double* __restrict__ beta, double beta_sum, double lgamma_beta_sum,
                             const double* __restrict__ lgamma_beta, const long long* __restrict__ counts,
                             const long long* __restrict__ sums, double* __restrict__ out) {
  __shared__ double red[BLOCK];
  const int it = blockIdx.x;
  if (it >= n_items) return;
  const LogmlItem item = items[it];
  long long npts = 0;
  for (int q = 0; q < 4; ++q)
    if (item.seg[q] >= 0) npts += counts[item.seg[q]];
  if (npts == 0) {
    if (threadIdx.x == 0) out[it] = 0.0;
    return;
  }
  double acc = 0.0, tot = 0.0;
  for (int v = threadIdx.x; v < V; v += BLOCK) {
    long long c = 0;
    for (int q = 0; q < 4; ++q)
      if (item.seg[q] >= 0) c += sums[(size_t)item.seg[q] * V + v];
    acc += lgamma_d(beta[v] + (double)c) - lgamma_beta[v];
    tot += (double)c;
  }
  acc = reduce_sum(acc, red);
  tot = reduce_sum(tot, red);
  if (threadIdx.x == 0) out[it] = lgamma_beta_sum - lgamma_d(beta_sum + tot) + acc;
}

__global__ void k_relabel(long long n, const RelabelEntry* __restrict__ table, int n_entries, uint32_t t,
                          uint64_t seed, int* __restrict__ z, unsigned char* __restrict__ zsub) {
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * BLOCK) {
    const int zi = z[i], zs = zsub[i];
    const int s = 2 * zi + zs;
    if (zi < 0 || zs > 1 || s >= n_entries) continue;  // labels outside the table stay as they are
    const RelabelEntry e = table[s];
    z[i] = e.new_z;
    if (e.mode == 1) {
      zsub[i] = 0;
    } else if (e.mode == 2) {
      zsub[i] = 1;
    } else if (e.mode == 3) {
      zsub[i] = (unsigned char)(rng_block(seed, t, (uint32_t)i, TAG_SUBINIT, 0).x & 1u);
    }
  }
}

__global__ void k_init_labels(long long n, uint64_t seed, int* __restrict__ z, unsigned char* __restrict__ zsub) {
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * BLOCK) {
    z[i] = 0;
    zsub[i] = (unsigned char)(rng_block(seed, 0, (uint32_t)i, TAG_SUBINIT, 0).x & 1u);
  }
}

int grid_for(long long n) {
  long long g = (n + BLOCK - 1) / BLOCK;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_set_pair(int* p, int a, int b, hipStream_t s) {
  hipLaunchKernelGGL(k_set_pair, dim3(1), dim3(64), 0, s, p, a, b);
  return hipGetLastError();
}

hipError_t launch_zero64(void* p, size_t n_words, hipStream_t s) {
  if (n_words == 0) return hipSuccess;
  size_t g = (n_words + BLOCK - 1) / BLOCK;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_zero64, dim3((unsigned)g), dim3(BLOCK), 0, s, (unsigned long long*)p, n_words);
  return hipGetLastError();
}

hipError_t launch_logml_gauss(int n_items, const LogmlItem* items, int d, NiwPriorDev prior, double logdet_psi,
                              const long long* counts, const double* moments, double* scratch, double* out,
                              int* err, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  const dim3 wg((n_items + BLOCK / 64 - 1) / (BLOCK / 64));
  if (d <= 16) {
    hipLaunchKernelGGL(k_logml_gauss_wave<16>, wg, dim3(BLOCK), 0, s, n_items, items, d, prior, logdet_psi, counts,
                       moments, out, err);
    return hipGetLastError();
  }
  if (d <= 32) {
    hipLaunchKernelGGL(k_logml_gauss_wave<32>, wg, dim3(BLOCK), 0, s, n_items, items, d, prior, logdet_psi, counts,
                       moments, out, err);
    return hipGetLastError();
  }
  if (d <= 64) {
    hipLaunchKernelGGL(k_logml_gauss_wave<64>, wg, dim3(BLOCK), 0, s, n_items, items, d, prior, logdet_psi, counts,
                       moments, out, err);
    return hipGetLastError();
  }
  const size_t lds = d <= LOGML_LDS_MAX_D ? (size_t)d * d * sizeof(double) : 0;
  hipLaunchKernelGGL(k_logml_gauss, dim3(n_items), dim3(BLOCK), lds, s, n_items, items, d, prior, logdet_psi,
                     counts, moments, scratch, out, err);
  return hipGetLastError();
}

hipError_t launch_logml_mult(int n_items, const LogmlItem* items, int V, const double* beta, double beta_sum,
                             double lgamma_beta_sum, const double* lgamma_beta, const long long* counts,
                             const long long* sums, double* out, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_logml_mult, dim3(n_items), dim3(BLOCK), 0, s, n_items, items, V, beta, beta_sum,
                     lgamma_beta_sum, lgamma_beta, counts, sums, out);
  return hipGetLastError();
}

hipError_t launch_merge_decide(int n_pairs, const LogmlItem* pairs, const long long* counts, const double* lml_cluster,
                               const double* lml_pair, double alpha, bool paper_form, uint64_t seed, uint32_t t,
                               unsigned char* accept, hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge_decide, dim3((n_pairs + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, n_pairs, pairs, counts,
                     lml_cluster, lml_pair, alpha, paper_form ? 1 : 0, seed, t, accept);
  return hipGetLastError();
}

size_t readback_bytes(int K, int P) { return 8 + 40 * (size_t)K + (size_t)P; }

hipError_t launch_pack_readback(int K, int P, const long long* counts, const double* lml, const unsigned char* mflag,
                                const int* err, unsigned char* out, hipStream_t s) {
  const int n = 5 * K + P;
  hipLaunchKernelGGL(k_pack_readback, dim3((n + 255) / 256), dim3(256), 0, s, K, P, counts, lml, mflag, err, out);
  return hipGetLastError();
}

hipError_t launch_relabel(long long n, const RelabelEntry* table, int n_entries, uint32_t t, uint64_t seed, int* z,
                          unsigned char* zsub, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_relabel, dim3(grid_for(n)), dim3(BLOCK), 0, s, n, table, n_entries, t, seed, z, zsub);
  return hipGetLastError();
}

hipError_t launch_init_labels(long long n, uint64_t seed, int* z, unsigned char* zsub, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_labels, dim3(grid_for(n)), dim3(BLOCK), 0, s, n, seed, z, zsub);
  return hipGetLastError();
}

}  // namespace dpmm
