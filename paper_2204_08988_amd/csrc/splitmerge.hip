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

// Item it of a launch: it itself, or in list mode (list != nullptr) the
// base + list[q]-th item for q < *list_count (the survivors of the merge bound).
__device__ __forceinline__ int logml_item(int q, int n_items, const int* list, const int* list_count, int base) {
  if (!list) return q < n_items ? q : -1;
  return q < *list_count ? base + list[q] : -1;
}

__global__ void k_logml_gauss(int n_items, const LogmlItem* __restrict__ items, int d, NiwPriorDev prior,
                              double logdet_psi, const long long* __restrict__ counts,
                              const double* __restrict__ moments, double* __restrict__ scratch,
                              double* __restrict__ out, int* __restrict__ err, const int* __restrict__ list,
                              const int* __restrict__ list_count, int list_base) {
  extern __shared__ double lds_p[];
  __shared__ double red[BLOCK];
  __shared__ int flag;
  const int it = logml_item(blockIdx.x, n_items, list, list_count, list_base);
  if (it < 0) return;
  const int tid = threadIdx.x;
  const int E = d + d * (d + 1) / 2;
  const LogmlItem item = items[it];
  // bound item: log|Psi / 2 + C| of the union's scatter C (for the merge bound)
  const bool bound = item.seg[3] == LOGML_BOUND;
  double n = 0.0;
  for (int q = 0; q < 4; ++q)
    if (item.seg[q] >= 0) n += (double)counts[item.seg[q]];
  if (n == 0.0) {
    if (tid == 0) out[it] = 0.0;
    return;
  }
  double* P = d <= LOGML_LDS_MAX_D ? lds_p : scratch + (size_t)blockIdx.x * d * d;
  const double kn = prior.kappa + n, nun = prior.nu + n;
  const double wpsi = bound ? 0.5 : 1.0, wmean = bound ? 0.0 : prior.kappa * n / kn;
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
    P[idx] = wpsi * prior.psi[idx] + (S - n * xi * xj) + wmean * (xi - prior.m[i]) * (xj - prior.m[j]);
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
    out[it] = bound ? ld
                    : -0.5 * n * d * 1.1447298858494002 + lg + 0.5 * prior.nu * logdet_psi - 0.5 * nun * ld +
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
                                                            double* __restrict__ out, int* __restrict__ err,
                                                            const int* __restrict__ list,
                                                            const int* __restrict__ list_count, int list_base) {
  constexpr int ED = D + D * (D + 1) / 2;
  __shared__ double ssum[BLOCK / 64][ED];  // per wave: the item's summed statistics
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int it = logml_item(blockIdx.x * (BLOCK / 64) + wave, n_items, list, list_count, list_base);
  if (it < 0) return;
  const int E = d + d * (d + 1) / 2;
  const LogmlItem item = items[it];
  const bool bound = item.seg[3] == LOGML_BOUND;  // log|Psi / 2 + C| (merge bound)
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
  const double wpsi = bound ? 0.5 : 1.0;
#pragma unroll
  for (int k = 0; k < D; ++k) r[k] = (k < d && live && k <= lane) ? wpsi * prior.psi[lane * d + k] : 0.0;
  double n = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) n += nq[q];
  if (n == 0.0) {
    if (lane == 0) out[it] = 0.0;
    return;
  }
  const double kn = prior.kappa + n, nun = prior.nu + n, cm = bound ? 0.0 : prior.kappa * n / kn;
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
    out[it] = bound ? ld
                    : -0.5 * n * d * 1.1447298858494002 + lg + 0.5 * prior.nu * logdet_psi - 0.5 * nun * ld +
                          0.5 * d * (log(prior.kappa) - log(kn));
  }
}
// 64 < d <= 128: one workgroup per item, Psi_n held in registers as the
// 136 lower 8 x 8 tiles of a 128 x 128 matrix (d padded with an identity
// block, whose pivots are 1), one tile per thread of the first 136.  Blocked
// right-looking Cholesky, one 8-column panel per step: the diagonal tile's
// owner factors it in registers and publishes L_jj (its own 8 x 8 buffer), the
// owners of the tiles below solve against it and publish the panel, and every
// trailing tile takes the rank-8 update from the published panel -- two
// barriers per 8 columns, an 8 KB panel buffer in LDS read as contiguous 8-row
// pieces.  A buffer is rewritten only after the barrier that follows its last
// reads (L_jj: read before the panel barrier; the panel: read before the next
// step's first barrier).  log|Psi_n| is
// summed as one log per panel (the product of its 8 pivots).
constexpr int TILE_T = 136;  // 16 * 17 / 2 lower tiles of 8 x 8
constexpr int CHOL_T = 192;  // three waves cover the 136 tile owners

__global__ __launch_bounds__(CHOL_T) void k_logml_gauss_tile(int n_items, const LogmlItem* __restrict__ items, int d,
                                                             NiwPriorDev prior, double logdet_psi,
                                                             const long long* __restrict__ counts,
                                                             const double* __restrict__ moments,
                                                             double* __restrict__ out, int* __restrict__ err,
                                                             const int* __restrict__ list,
                                                             const int* __restrict__ list_count, int list_base,
                                                             const double* __restrict__ cmom, int K) {
  constexpr int DP = 128, T = 8, NTL = DP / T;
  __shared__ double xbar[DP];
  __shared__ __align__(16) double pan[T][DP];  // pan[c][row] = L[row][8 jt + c] below the diagonal tile
  __shared__ double dg[T][T];                 // dg[c][r] = L[8 jt + r][8 jt + c] of the diagonal tile
  __shared__ double red[CHOL_T / 64];
  __shared__ int bad;
  const int it = logml_item(blockIdx.x, n_items, list, list_count, list_base);
  if (it < 0) return;
  const int tid = threadIdx.x;
  const int E = d + d * (d + 1) / 2;
  const LogmlItem item = items[it];
  const bool bound = item.seg[3] == LOGML_BOUND;  // log|Psi / 2 + C| (merge bound)
  double n = 0.0;
  for (int q = 0; q < 4; ++q)
    if (item.seg[q] >= 0) n += (double)counts[item.seg[q]];
  if (n == 0.0) {
    if (tid == 0) out[it] = 0.0;
    return;
  }
  const double kn = prior.kappa + n, nun = prior.nu + n;
  const double wpsi = bound ? 0.5 : 1.0, wmean = bound ? 0.0 : prior.kappa * n / kn;
  if (tid < DP) {
    double si = 0.0;
    if (tid < d)
      for (int q = 0; q < 4; ++q)
        if (item.seg[q] >= 0) si += moments[(size_t)item.seg[q] * E + tid];
    xbar[tid] = si / n;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  // this thread's tile (TR, TC), TR >= TC
  int TR = 0, TC = 0;
  {
    int u = tid < TILE_T ? tid : 0;
    while (u > TR) {
      u -= TR + 1;
      ++TR;
    }
    TC = u;
  }
  const bool owner = tid < TILE_T;
  // whole clusters among the item's segments (2 k, 2 k + 1): their summed scatter
  // with Psi / 2 comes precomputed in cmom[k], this thread's tile contiguous
  auto whole = [&](int q) {
    const int a0 = item.seg[q], a1 = item.seg[q + 1];
    return (cmom && a0 >= 0 && (a0 & 1) == 0 && a1 == a0 + 1 && a0 / 2 < K) ? a0 / 2 : -1;
  };
  const int ca = whole(0), cb = item.seg[2] >= 0 ? whole(2) : -1;
  // pair of whole clusters: Psi + S = cmom[ca] + cmom[cb]; one whole cluster: cmom[ca]
  // plus Psi / 2 (slot K); a bound item wants Psi / 2 + S: cmom[ca] alone
  const bool use_c = ca >= 0 && (item.seg[2] < 0 || cb >= 0);
  const double* tca = use_c ? cmom + ((size_t)ca * TILE_T + (owner ? tid : 0)) * 64 : nullptr;
  const double* tcb = use_c ? cmom + ((size_t)(cb >= 0 ? cb : K) * TILE_T + (owner ? tid : 0)) * 64 : nullptr;
  const double wrest = (cb >= 0 || !bound) ? 1.0 : 0.0;
  double a[T][T];
#pragma unroll
  for (int r = 0; r < T; ++r)
#pragma unroll
    for (int c = 0; c < T; ++c) {
      const int i = T * TR + r, k = T * TC + c;
      double v = 0.0;
      if (owner && k <= i) {
        if (i < d) {
          const int lo = k, hi = i;  // k <= i: packed upper-triangle entry (k, i)
          const double xi = xbar[i], xk = xbar[k];
          if (use_c) {
            const double pc = tca[T * r + c] + wrest * tcb[T * r + c];
            v = (pc - n * xi * xk) + wmean * (xi - prior.m[i]) * (xk - prior.m[k]);
          } else {
            double S = 0.0;
            for (int q = 0; q < 4; ++q)
              if (item.seg[q] >= 0) S += moments[(size_t)item.seg[q] * E + d + tri_index(lo, hi, d)];
            v = wpsi * prior.psi[i * d + k] + (S - n * xi * xk) + wmean * (xi - prior.m[i]) * (xk - prior.m[k]);
          }
        } else {
          v = i == k ? 1.0 : 0.0;  // the identity padding
        }
      }
      a[r][c] = v;
    }
  double ld = 0.0;  // sum of log L_jj over this thread's diagonal tiles
  for (int jt = 0; jt < NTL; ++jt) {
    // the diagonal tile, factored in registers (lower triangle; the upper part is never read)
    if (owner && TR == jt && TC == jt) {
      double prod = 1.0;
      bool ok = true;
#pragma unroll
      for (int c = 0; c < T; ++c) {
        double s = a[c][c];
        if (!(s > 0.0) || !isfinite(s)) {
          ok = false;
          s = 1.0;
        }
        const double l = sqrt(s), inv = 1.0 / l;
        prod *= l;
        a[c][c] = l;
#pragma unroll
        for (int r = c + 1; r < T; ++r) a[r][c] *= inv;
#pragma unroll
        for (int c2 = c + 1; c2 < T; ++c2)
#pragma unroll
          for (int r = c2; r < T; ++r) a[r][c2] = fma(-a[r][c], a[c2][c], a[r][c2]);
      }
      if (!ok) bad = 1;
      ld += log(prod);
#pragma unroll
      for (int c = 0; c < T; ++c)
#pragma unroll
        for (int r = 0; r < T; ++r) dg[c][r] = r >= c ? a[r][c] : 0.0;
    }
    __syncthreads();
    // the tiles below it: A_ij L_jj^-T, row by row forward substitution
    if (owner && TC == jt && TR > jt) {
      // column by column: row c of L_jj (at most 8 values) is all a column needs
#pragma unroll
      for (int c = 0; c < T; ++c) {
        double lr[T];
#pragma unroll
        for (int c2 = 0; c2 < c; ++c2) lr[c2] = dg[c2][c];
        const double ic = 1.0 / dg[c][c];
#pragma unroll
        for (int r = 0; r < T; ++r) {
          double v = a[r][c];
#pragma unroll
          for (int c2 = 0; c2 < c; ++c2) v = fma(-a[r][c2], lr[c2], v);
          a[r][c] = v * ic;
        }
      }
#pragma unroll
      for (int c = 0; c < T; ++c)
#pragma unroll
        for (int r = 0; r < T; ++r) pan[c][T * TR + r] = a[r][c];
    }
    __syncthreads();
    // the trailing tiles: A_ik -= L_i L_k^T over the panel's 8 columns
    if (owner && TC > jt) {
#pragma unroll
      for (int c2 = 0; c2 < T; ++c2) {
        double pr[T], pc[T];
#pragma unroll
        for (int r = 0; r < T; ++r) pr[r] = pan[c2][T * TR + r];
#pragma unroll
        for (int c = 0; c < T; ++c) pc[c] = pan[c2][T * TC + c];
#pragma unroll
        for (int r = 0; r < T; ++r)
#pragma unroll
          for (int c = 0; c < T; ++c) a[r][c] = fma(-pr[r], pc[c], a[r][c]);
      }
    }
  }
  // log|Psi_n| = 2 sum log L_jj; log Gamma_d(nu_n / 2) - log Gamma_d(nu / 2)
  double lg = 0.0;
  for (int i = tid; i < d; i += CHOL_T) lg += lgamma_d(0.5 * nun - 0.5 * i) - lgamma_d(0.5 * prior.nu - 0.5 * i);
  auto block_sum = [&](double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < CHOL_T / 64; ++w) t += red[w];
    return t;
  };
  const double ldet = 2.0 * block_sum(ld);
  lg = block_sum(lg);
  if (tid == 0) {
    if (bad) atomicOr(err, 4);
    out[it] = bound ? ldet
                    : -0.5 * n * d * 1.1447298858494002 + lg + 0.5 * prior.nu * logdet_psi - 0.5 * nun * ldet +
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
// log Gamma_d(a) - log Gamma_d(b) = sum_{j < d} lgamma(a - j/2) - lgamma(b - j/2)
__device__ double lmultigamma_diff(double a, double b, int d) {
  double s = 0.0;
  for (int j = 0; j < d; ++j) s += lgamma_d(a - 0.5 * j) - lgamma_d(b - 0.5 * j);
  return s;
}

// The merge bound (Gaussian family): for the pair (k1, k2) with union U,
//   Psi_n(U) >= X + Y + b b^T,  X = Psi/2 + C1, Y = Psi/2 + C2 (scatters about
//   the clusters' means), b = sqrt(n1 n2 / n) (xbar1 - xbar2);
//   log|X + Y| >= d log(|X|^(1/d) + |Y|^(1/d)) (Minkowski's determinant inequality),
//   b^T (X + Y)^-1 b >= |b|^2 / (lambda_max(Psi) + tr C1 + tr C2),
// give a lower bound LB on log|Psi_n(U)|, so an upper bound on the NIW
// marginal of U and on log H_merge.  A pair whose bound (plus a rounding
// margin) lies below log u is rejected here: exactly the decision its full
// ratio would give.  Every other pair is listed for its log marginal and
// k_merge_decide.  logdet_half[k] = log|Psi/2 + C_k|; lam_psi >= lambda_max(Psi).
__global__ void k_merge_prune(int n_pairs, const LogmlItem* __restrict__ pairs, int d, NiwPriorDev prior,
                              double logdet_psi, double lam_psi, const long long* __restrict__ counts,
                              const double* __restrict__ moments, const double* __restrict__ lml_cluster,
                              const double* __restrict__ logdet_half, double alpha, int paper_form, uint64_t seed,
                              uint32_t t, unsigned char* __restrict__ accept, int* __restrict__ list,
                              int* __restrict__ list_count) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const LogmlItem it = pairs[p];
  const int k1 = it.seg[0] >> 1, k2 = it.seg[2] >> 1;
  const int E = d + d * (d + 1) / 2;
  const double n1 = (double)(counts[2 * k1] + counts[2 * k1 + 1]);
  const double n2 = (double)(counts[2 * k2] + counts[2 * k2 + 1]);
  const double n = n1 + n2;
  const double* A0 = moments + (size_t)(2 * k1) * E;
  const double* A1 = A0 + E;
  const double* B0 = moments + (size_t)(2 * k2) * E;
  const double* B1 = B0 + E;
  // tr C_k = sum_i S_ii - |s|^2 / n_k, and |xbar1 - xbar2|^2
  double tr1 = 0.0, tr2 = 0.0, ss1 = 0.0, ss2 = 0.0, dx2 = 0.0;
  for (int i = 0; i < d; ++i) {
    const int di = d + tri_index(i, i, d);
    const double s1 = A0[i] + A1[i], s2 = B0[i] + B1[i];
    tr1 += A0[di] + A1[di];
    tr2 += B0[di] + B1[di];
    ss1 += s1 * s1;
    ss2 += s2 * s2;
    const double dd = s1 / n1 - s2 / n2;
    dx2 += dd * dd;
  }
  tr1 = fmax(tr1 - ss1 / n1, 0.0);
  tr2 = fmax(tr2 - ss2 / n2, 0.0);
  const double a = logdet_half[k1] / d, c = logdet_half[k2] / d;
  const double lb = d * (fmax(a, c) + log1p(exp(-fabs(a - c)))) + log1p(n1 * n2 / n * dx2 / (lam_psi + tr1 + tr2));
  const double nun = prior.nu + n, kn = prior.kappa + n;
  const double lmg = lmultigamma_diff(0.5 * nun, 0.5 * prior.nu, d);
  const double ub_u = -0.5 * n * d * 1.1447298858494002 + lmg + 0.5 * prior.nu * logdet_psi - 0.5 * nun * lb +
                      0.5 * d * (log(prior.kappa) - log(kn));
  double g = lgamma_d(n) - log(alpha) - lgamma_d(n1) - lgamma_d(n2);
  if (paper_form)
    g += lgamma_d(alpha) - lgamma_d(alpha + n) + lgamma_d(0.5 * alpha + n1) + lgamma_d(0.5 * alpha + n2) -
         2.0 * lgamma_d(0.5 * alpha);
  const double l1 = lml_cluster[3 * k1], l2 = lml_cluster[3 * k2];
  const double ub = g + ub_u - l1 - l2;
  // float64 rounding of the terms above (and of the Cholesky factorisations behind them)
  const double margin = 1e-9 * (fabs(g) + fabs(lmg) + 0.5 * nun * fabs(lb) + 0.5 * n * d * 1.15 + fabs(l1) + fabs(l2) +
                                0.5 * prior.nu * fabs(logdet_psi)) + 1e-6;
  const double u = uniform_d(rng_block(seed, t, merge_entity(k1, k2), TAG_MERGE, 0).x);
  if (ub + margin < log(u)) {
    accept[p] = 0;
  } else {
    list[atomicAdd(list_count, 1)] = p;  // the order of the list does not matter: one result per pair
  }
}

__global__ void k_merge_decide(int n_pairs, const LogmlItem* __restrict__ pairs, const long long* __restrict__ counts,
                               const double* __restrict__ lml_cluster, const double* __restrict__ lml_pair,
                               double alpha, int paper_form, uint64_t seed, uint32_t t,
                               unsigned char* __restrict__ accept, const int* __restrict__ list,
                               const int* __restrict__ list_count) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = list ? (q < *list_count ? list[q] : -1) : (q < n_pairs ? q : -1);
  if (p < 0) return;
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

// NT threads per item: 1024 for a large vocabulary (the log-Gamma calls of an
// item spread over 16 waves), BLOCK otherwise
template <int NT>
__global__ __launch_bounds__(NT) void k_logml_mult(int n_items, const LogmlItem* __restrict__ items, int V,
                                                   const double* __restrict__ beta, double beta_sum,
                                                   double lgamma_beta_sum, const double* __restrict__ lgamma_beta,
                                                   const long long* __restrict__ counts,
                                                   const long long* __restrict__ sums, double* __restrict__ out) {
  __shared__ double red[NT];
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
  for (int v = threadIdx.x; v < V; v += NT) {
    long long c = 0;
    for (int q = 0; q < 4; ++q)
      if (item.seg[q] >= 0) c += sums[(size_t)item.seg[q] * V + v];
    if (c == 0) continue;  // lgamma(beta_v) - lgamma(beta_v) = 0: most words of a large vocabulary
    acc += lgamma_d(beta[v] + (double)c) - lgamma_beta[v];
    tot += (double)c;
  }
  acc = reduce_sum(acc, red);
  tot = reduce_sum(tot, red);
  if (threadIdx.x == 0) out[it] = lgamma_beta_sum - lgamma_d(beta_sum + tot) + acc;
}

// Gamma-Poisson: sum_v [a_v log b_v - lgamma(a_v) + lgamma(a_v + c_v) -
// (a_v + c_v) log(b_v + n)] (the per-point 1 / x! factors left out: they
// cancel in every ratio); pconst holds the first two terms summed.
__global__ void k_logml_pois(int n_items, const LogmlItem* __restrict__ items, int V, const double* __restrict__ shape,
                             const double* __restrict__ rate, double pconst, const long long* __restrict__ counts,
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
  double acc = 0.0;
  for (int v = threadIdx.x; v < V; v += BLOCK) {
    long long c = 0;
    for (int q = 0; q < 4; ++q)
      if (item.seg[q] >= 0) c += sums[(size_t)item.seg[q] * V + v];
    const double ac = shape[v] + (double)c;
    acc += lgamma_d(ac) - ac * log(rate[v] + (double)npts);
  }
  acc = reduce_sum(acc, red);
  if (threadIdx.x == 0) out[it] = pconst + acc;
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

// cmom[k] = Psi / 2 + S_2k + S_2k+1, cluster k's scatter matrix plus half the
// prior's, in the tile kernel's register layout ([136 lower 8 x 8 tiles][8][8],
// tile u held by thread u, zero outside the lower d x d triangle), and in slot K
// Psi / 2 alone: a thread of the tile kernel reads its 64 entries contiguously.
__global__ void k_cluster_scatter(int K, int d, NiwPriorDev prior, const double* __restrict__ moments,
                                  double* __restrict__ cmom) {
  const int E = d + d * (d + 1) / 2;
  const int k = blockIdx.y;  // K: Psi / 2 alone
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < CMOM_TILE_ENTRIES; e += gridDim.x * blockDim.x) {
    int u = e >> 6, TR = 0;
    while (u > TR) {
      u -= TR + 1;
      ++TR;
    }
    const int i = 8 * TR + ((e >> 3) & 7), j = 8 * u + (e & 7);
    double v = 0.0;
    if (j <= i && i < d) {
      v = 0.5 * prior.psi[i * d + j];
      if (k < K) {
        const int t = tri_index(j, i, d);
        v += moments[(size_t)(2 * k) * E + d + t] + moments[(size_t)(2 * k + 1) * E + d + t];
      }
    }
    cmom[(size_t)k * CMOM_TILE_ENTRIES + e] = v;
  }
}

hipError_t launch_logml_gauss(int n_items, const LogmlItem* items, int d, NiwPriorDev prior, double logdet_psi,
                              const long long* counts, const double* moments, double* scratch, double* out,
                              int* err, hipStream_t s, const int* list, const int* list_count, int list_base,
                              double* cmom, int K) {
  if (n_items == 0) return hipSuccess;
  const dim3 wg((n_items + BLOCK / 64 - 1) / (BLOCK / 64));
#define DPMM_LOGML_WAVE(DD)                                                                                         \
  hipLaunchKernelGGL(k_logml_gauss_wave<DD>, wg, dim3(BLOCK), 0, s, n_items, items, d, prior, logdet_psi, counts, \
                     moments, out, err, list, list_count, list_base);                                             \
  return hipGetLastError();
  if (d <= 16) {
    DPMM_LOGML_WAVE(16)
  }
  if (d <= 32) {
    DPMM_LOGML_WAVE(32)
  }
  if (d <= 64) {
    DPMM_LOGML_WAVE(64)
  }
#undef DPMM_LOGML_WAVE
  if (d <= 128) {
    if (cmom && K > 0)
      hipLaunchKernelGGL(k_cluster_scatter, dim3((CMOM_TILE_ENTRIES + 255) / 256, K + 1), dim3(256), 0, s, K, d, prior,
                         moments, cmom);
    hipLaunchKernelGGL(k_logml_gauss_tile, dim3(n_items), dim3(CHOL_T), 0, s, n_items, items, d, prior, logdet_psi,
                       counts, moments, out, err, list, list_count, list_base, cmom, cmom ? K : 0);
    return hipGetLastError();
  }
  const size_t lds = d <= LOGML_LDS_MAX_D ? (size_t)d * d * sizeof(double) : 0;
  hipLaunchKernelGGL(k_logml_gauss, dim3(n_items), dim3(BLOCK), lds, s, n_items, items, d, prior, logdet_psi,
                     counts, moments, scratch, out, err, list, list_count, list_base);
  return hipGetLastError();
}

hipError_t launch_merge_prune(int n_pairs, const LogmlItem* pairs, int d, NiwPriorDev prior, double logdet_psi,
                              double lam_psi, const long long* counts, const double* moments, const double* lml_cluster,
                              const double* logdet_half, double alpha, bool paper_form, uint64_t seed, uint32_t t,
                              unsigned char* accept, int* list, int* list_count, hipStream_t s) {
  hipError_t e = launch_zero64(list_count, 1, s);
  if (e != hipSuccess || n_pairs == 0) return e;
  hipLaunchKernelGGL(k_merge_prune, dim3((n_pairs + 63) / 64), dim3(64), 0, s, n_pairs, pairs, d, prior, logdet_psi,
                     lam_psi, counts, moments, lml_cluster, logdet_half, alpha, paper_form ? 1 : 0, seed, t, accept,
                     list, list_count);
  return hipGetLastError();
}

hipError_t launch_logml_mult(int n_items, const LogmlItem* items, int V, const double* beta, double beta_sum,
                             double lgamma_beta_sum, const double* lgamma_beta, const long long* counts,
                             const long long* sums, double* out, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  if (V > 4096)
    hipLaunchKernelGGL(k_logml_mult<1024>, dim3(n_items), dim3(1024), 0, s, n_items, items, V, beta, beta_sum,
                       lgamma_beta_sum, lgamma_beta, counts, sums, out);
  else
    hipLaunchKernelGGL(k_logml_mult<BLOCK>, dim3(n_items), dim3(BLOCK), 0, s, n_items, items, V, beta, beta_sum,
                       lgamma_beta_sum, lgamma_beta, counts, sums, out);
  return hipGetLastError();
}

hipError_t launch_logml_pois(int n_items, const LogmlItem* items, int V, const double* shape, const double* rate,
                             double pconst, const long long* counts, const long long* sums, double* out,
                             hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_logml_pois, dim3(n_items), dim3(BLOCK), 0, s, n_items, items, V, shape, rate, pconst, counts,
                     sums, out);
  return hipGetLastError();
}

hipError_t launch_merge_decide(int n_pairs, const LogmlItem* pairs, const long long* counts, const double* lml_cluster,
                               const double* lml_pair, double alpha, bool paper_form, uint64_t seed, uint32_t t,
                               unsigned char* accept, hipStream_t s, const int* list, const int* list_count) {
  if (n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge_decide, dim3((n_pairs + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, n_pairs, pairs, counts,
                     lml_cluster, lml_pair, alpha, paper_form ? 1 : 0, seed, t, accept, list, list_count);
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
