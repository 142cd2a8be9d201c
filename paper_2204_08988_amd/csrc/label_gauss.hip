// Gaussian label step, float32 VALU path: Sec. 4.1 steps (e) and (f).
//
// One lane per point, points streamed with a grid-stride loop (x is
// point-major, so a wave reads 64 consecutive rows).  The cluster loop is
// uniform across the wave: the component record address depends only on the
// loop counter, so the compiler fetches means, whitener rows and constants
// with scalar loads and feeds them to the FMAs as scalar operands.
//
// Score of a component: l = c - 1/2 ||W (x - mu)||^2 with W lower triangular
// (W^T W = Sigma^-1), i.e. d(d+1)/2 FMAs for W (x - mu) and d for the norm.
//
// Label draw (eq. sample_labels) as a lazy Gumbel-max: pass 1 keeps the two
// best scores m1 >= m2.  If m2 < m1 - (G_max - G_min) no other cluster can
// beat the leader whatever the noise, so z is the leader and no random number
// is drawn.  Otherwise pass 2 draws the leader's Gumbel first and then the
// Gumbel of each other cluster k only if l_k + G_max can still exceed the
// best perturbed score; the result equals argmax_k (l_k + g_k) over all k.
// Sub-label (eq. sample_sub_labels), small d: the two sub-cluster records of
// z are gathered per lane; the logistic draw is skipped when the score gap
// exceeds the logistic's range.  For d >= 5 the kernel draws z only and the
// sub-labels are drawn in cluster-sorted order (sorted.hip), where the
// sub-cluster records are wave-uniform.
#include "kernels.hpp"
#include "score.hpp"

namespace dpmm {

namespace {

using namespace score;

template <int D, bool STAGED, int KM>
__global__ __launch_bounds__(BLOCK) void k_label_gauss(const float* __restrict__ x, long long n,
                                                       const float* __restrict__ packed, int K, int k_max,
                                                       uint32_t t, uint64_t seed, int* __restrict__ z,
                                                       unsigned char* __restrict__ zsub) {
  constexpr int S = (4 + D + D * (D + 1) / 2 + 3) & ~3;
  // STAGED: the K cluster records, then the 2K sub-cluster records, copied to
  // LDS once per workgroup (broadcast reads instead of a scalar load per
  // cluster and a per-lane global gather per point)
  extern __shared__ float recs[];
  const float* cl = packed;
  const float* sub = packed + (size_t)k_max * S;
  if constexpr (STAGED) {
    for (int q = threadIdx.x; q < K * S; q += BLOCK) recs[q] = packed[q];
    for (int q = threadIdx.x; q < 2 * K * S; q += BLOCK) recs[K * S + q] = packed[(size_t)k_max * S + q];
    __syncthreads();
    cl = recs;
    sub = recs + K * S;
  }
  const long long stride_pts = (long long)gridDim.x * BLOCK;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride_pts) {
    float xv[D];
#pragma unroll
    for (int j = 0; j < D; ++j) xv[j] = x[i * D + j];
    Top2 t2;
    t2.init();
    int zi;
    // the sub-label's word: the unused word of Gumbel block K / 4 when K % 4 != 0
    // (that block computed once, for every lane, and shared with the draw of z)
    uint32_t wsub = 0;
    if constexpr (KM > 0) {
      // K <= KM: the scores stay in registers for the draw
      float lk[KM];
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        lk[k] = k < K ? score_rec<D>(cl + (size_t)k * S, xv) : -INFINITY;
        if (k < K) t2.push(lk[k], k);
      }
      const u32x4 last = (K & 3) ? rng_block(seed, t, (uint32_t)i, TAG_GUMBEL, (uint32_t)(K >> 2)) : u32x4{0u, 0u, 0u, 0u};
      wsub = word_of(last, K & 3);
      zi = lazy_gumbel_max_regs<KM>(lk, t2, K, (uint32_t)i, t, seed, last);
    } else {
      for (int k = 0; k < K; ++k) t2.push(score_rec<D>(cl + (size_t)k * S, xv), k);
      zi = lazy_gumbel_max(t2, K, (uint32_t)i, t, seed, [&](int k) { return score_rec<D>(cl + (size_t)k * S, xv); });
    }
    const float* ps = sub + (size_t)(2 * zi) * S;
    const float delta = score_rec<D>(ps, xv) - score_rec<D>(ps + S, xv);
    z[i] = zi;
    if (KM > 0 && (K & 3))
      zsub[i] = delta > LOGISTIC_MAX_F ? 0 : (delta < -LOGISTIC_MAX_F ? 1 : sub_label_from_word(delta, wsub));
    else
      zsub[i] = draw_sub(delta, (uint32_t)i, t, seed, K);
  }
}

__global__ __launch_bounds__(BLOCK) void k_label_gauss_dyn(const float* __restrict__ x, long long n, int d,
                                                           const float* __restrict__ packed, int K,
                                                           int k_max, uint32_t t, uint64_t seed,
                                                           int* __restrict__ z,
                                                           unsigned char* __restrict__ zsub) {
  extern __shared__ float lds[];
  float* dx = lds + threadIdx.x;
  const int S = gauss_rec_stride(d);
  const long long stride_pts = (long long)gridDim.x * BLOCK;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride_pts) {
    const float* xi = x + i * d;
    Top2 t2;
    t2.init();
    for (int k = 0; k < K; ++k) t2.push(score_rec_dyn(packed + (size_t)k * S, xi, dx, d), k);
    const int zi = lazy_gumbel_max(t2, K, (uint32_t)i, t, seed,
                                   [&](int k) { return score_rec_dyn(packed + (size_t)k * S, xi, dx, d); });
    const float* ps = packed + (size_t)(k_max + 2 * zi) * S;
    const float delta = score_rec_dyn(ps, xi, dx, d) - score_rec_dyn(ps + S, xi, dx, d);
    z[i] = zi;
    zsub[i] = draw_sub(delta, (uint32_t)i, t, seed, K);
  }
}

// Cluster draw only, for the cluster-sorted path (d >= 5): block b labels the
// contiguous points [b per_block, (b + 1) per_block) and writes its histogram
// of z (hist[b][k]) and adds it to the cluster totals tot[k].
template <int D>
__global__ __launch_bounds__(BLOCK) void k_label_gauss_z(const float* __restrict__ x, long long n, long long per_block,
                                                         const float* __restrict__ packed, int K, uint32_t t,
                                                         uint64_t seed, int* __restrict__ z, int* __restrict__ hist,
                                                         int* __restrict__ tot) {
  extern __shared__ int h[];
  constexpr int S = (4 + D + D * (D + 1) / 2 + 3) & ~3;
  for (int k = threadIdx.x; k < K; k += BLOCK) h[k] = 0;
  __syncthreads();
  const long long begin = (long long)blockIdx.x * per_block;
  const long long end = begin + per_block < n ? begin + per_block : n;
  for (long long i = begin + threadIdx.x; i < end; i += BLOCK) {
    float xv[D];
#pragma unroll
    for (int j = 0; j < D; ++j) xv[j] = x[i * D + j];
    Top2 t2;
    t2.init();
    for (int k = 0; k < K; ++k) t2.push(score_rec<D>(packed + (size_t)k * S, xv), k);
    const int zi = lazy_gumbel_max(t2, K, (uint32_t)i, t, seed,
                                   [&](int k) { return score_rec<D>(packed + (size_t)k * S, xv); });
    z[i] = zi;
    atomicAdd(&h[zi], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += BLOCK) {
    hist[(size_t)blockIdx.x * K + k] = h[k];
    if (h[k]) atomicAdd(&tot[k], h[k]);
  }
}

__global__ __launch_bounds__(BLOCK) void k_label_gauss_z_dyn(const float* __restrict__ x, long long n, int d,
                                                             long long per_block, const float* __restrict__ packed,
                                                             int K, uint32_t t, uint64_t seed, int* __restrict__ z,
                                                             int* __restrict__ hist, int* __restrict__ tot) {
  extern __shared__ float lds[];
  float* dx = lds + threadIdx.x;
  int* h = reinterpret_cast<int*>(lds + (size_t)d * BLOCK);
  const int S = gauss_rec_stride(d);
  for (int k = threadIdx.x; k < K; k += BLOCK) h[k] = 0;
  __syncthreads();
  const long long begin = (long long)blockIdx.x * per_block;
  const long long end = begin + per_block < n ? begin + per_block : n;
  for (long long i = begin + threadIdx.x; i < end; i += BLOCK) {
    const float* xi = x + i * d;
    Top2 t2;
    t2.init();
    for (int k = 0; k < K; ++k) t2.push(score_rec_dyn(packed + (size_t)k * S, xi, dx, d), k);
    const int zi = lazy_gumbel_max(t2, K, (uint32_t)i, t, seed,
                                   [&](int k) { return score_rec_dyn(packed + (size_t)k * S, xi, dx, d); });
    z[i] = zi;
    atomicAdd(&h[zi], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += BLOCK) {
    hist[(size_t)blockIdx.x * K + k] = h[k];
    if (h[k]) atomicAdd(&tot[k], h[k]);
  }
}

// All 3K weighted log-likelihoods per point (parity / inspection entry).
__global__ __launch_bounds__(BLOCK) void k_loglik_gauss_dyn(const float* __restrict__ x, long long n, int d,
                                                            const float* __restrict__ packed, int K,
                                                            int k_max, float* __restrict__ out) {
  extern __shared__ float lds[];
  float* dx = lds + threadIdx.x;
  const int S = gauss_rec_stride(d);
  const long long stride_pts = (long long)gridDim.x * BLOCK;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride_pts) {
    const float* xi = x + i * d;
    float* o = out + i * 3 * K;
    for (int k = 0; k < K; ++k) o[k] = score_rec_dyn(packed + (size_t)k * S, xi, dx, d);
    for (int j = 0; j < 2 * K; ++j) o[K + j] = score_rec_dyn(packed + (size_t)(k_max + j) * S, xi, dx, d);
  }
}

int grid_for(long long n) {
  // enough workgroups to fill 256 CUs several times over, capped so the
  // grid-stride loop gives each lane a few points at large n
  long long g = (n + BLOCK - 1) / BLOCK;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_label_gauss(int d, const float* x, long long n, const float* packed, int K, int k_max,
                              uint32_t t, uint64_t seed, int* z, unsigned char* zsub, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int g = grid_for(n);
  // the 3K score records go to LDS when they fit in 48 KB
  const size_t rec_bytes = (size_t)3 * K * gauss_rec_stride(d) * sizeof(float);
  const bool staged = rec_bytes <= 48 * 1024;
#define DPMM_LABEL_CASE(DD)                                                                              \
  case DD:                                                                                               \
    if (staged && K <= 8)                                                                                \
      hipLaunchKernelGGL((k_label_gauss<DD, true, 8>), dim3(g), dim3(BLOCK), rec_bytes, s, x, n, packed, \
                         K, k_max, t, seed, z, zsub);                                                    \
    else if (staged)                                                                                     \
      hipLaunchKernelGGL((k_label_gauss<DD, true, 0>), dim3(g), dim3(BLOCK), rec_bytes, s, x, n, packed, \
                         K, k_max, t, seed, z, zsub);                                                    \
    else                                                                                                 \
      hipLaunchKernelGGL((k_label_gauss<DD, false, 0>), dim3(g), dim3(BLOCK), 0, s, x, n, packed, K,     \
                         k_max, t, seed, z, zsub);                                                       \
    break;
  switch (d) {
    DPMM_LABEL_CASE(1)
    DPMM_LABEL_CASE(2)
    DPMM_LABEL_CASE(3)
    DPMM_LABEL_CASE(4)
    DPMM_LABEL_CASE(8)
    DPMM_LABEL_CASE(16)
    DPMM_LABEL_CASE(32)
    default:
      hipLaunchKernelGGL(k_label_gauss_dyn, dim3(g), dim3(BLOCK), (size_t)d * BLOCK * sizeof(float), s,
                         x, n, d, packed, K, k_max, t, seed, z, zsub);
  }
#undef DPMM_LABEL_CASE
  return hipGetLastError();
}

// d = 128, FP32: a workgroup walks its point range in chunks of BLOCK rows,
// gathered coalesced into LDS columns (stride BLOCK + 1); each thread centres
// its column in registers and scores the clusters with wave-uniform records.
// The Gumbel-max runs as one streaming pass: cluster k's Gumbel is drawn only
// while l_k + G_max can still beat the running best perturbed score, which
// gives the argmax of l_k + g_k over all k with the same counter-based g_k.
constexpr int COL_LD = BLOCK + 1;

template <int D>
__global__ __launch_bounds__(BLOCK) void k_label_gauss_z_col(const float* __restrict__ x, long long n,
                                                             long long per_block, const float* __restrict__ packed,
                                                             int K, uint32_t t, uint64_t seed, int* __restrict__ z,
                                                             int* __restrict__ hist, int* __restrict__ tot) {
  constexpr int S = (4 + D + D * (D + 1) / 2 + 3) & ~3;
  extern __shared__ float xs[];  // [D][COL_LD], then the histogram
  int* h = reinterpret_cast<int*>(xs + D * COL_LD);
  for (int k = threadIdx.x; k < K; k += BLOCK) h[k] = 0;
  const long long begin = (long long)blockIdx.x * per_block;
  const long long end = begin + per_block < n ? begin + per_block : n;
  for (long long chunk = begin; chunk < end; chunk += BLOCK) {
    const int rows = (int)(end - chunk < BLOCK ? end - chunk : BLOCK);
    __syncthreads();  // the previous chunk's columns are read
    for (int e = threadIdx.x; e < rows * D; e += BLOCK) {
      const int r = e / D, c = e - r * D;
      xs[c * COL_LD + r] = x[(size_t)(chunk + r) * D + c];
    }
    __syncthreads();
    const int r = threadIdx.x;
    if (r < rows) {
      const long long i = chunk + r;
      const float* xc = xs + r;
      float best = -INFINITY;
      int win = 0, cached = -1;
      u32x4 blk{0u, 0u, 0u, 0u};
      for (int k = 0; k < K; ++k) {
        const float l = score_col<D, COL_LD>(packed + (size_t)k * S, xc);
        if (l + GUMBEL_MAX_F > best) {
          const int b = k >> 2;
          if (b != cached) {
            blk = rng_block(seed, t, (uint32_t)i, TAG_GUMBEL, (uint32_t)b);
            cached = b;
          }
          const float v = l + gumbel_f(word_of(blk, k & 3));
          if (v > best) {
            best = v;
            win = k;
          }
        }
      }
      z[i] = win;
      atomicAdd(&h[win], 1);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += BLOCK) {
    hist[(size_t)blockIdx.x * K + k] = h[k];
    if (h[k]) atomicAdd(&tot[k], h[k]);
  }
}

hipError_t launch_label_gauss_z(int d, const float* x, long long n, int G, long long per_block, const float* packed,
                                int K, uint32_t t, uint64_t seed, int* z, int* hist, int* tot, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipError_t e = launch_zero64(tot, (size_t)(K + 1) / 2 + 1, s);
  if (e != hipSuccess) return e;
  const size_t lh = (size_t)K * sizeof(int);
#define DPMM_LABELZ_CASE(DD)                                                                                  \
  case DD:                                                                                                    \
    hipLaunchKernelGGL(k_label_gauss_z<DD>, dim3(G), dim3(BLOCK), lh, s, x, n, per_block, packed, K, t, seed, z, \
                       hist, tot);                                                                            \
    break;
  switch (d) {
    DPMM_LABELZ_CASE(8)
    DPMM_LABELZ_CASE(16)
    DPMM_LABELZ_CASE(32)
    DPMM_LABELZ_CASE(64)
    case 128: {
      static bool attr_set = false;
      if (!attr_set) {  // the row block takes more than 64 KB of LDS
        e = hipFuncSetAttribute((const void*)k_label_gauss_z_col<128>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
      }
      hipLaunchKernelGGL(k_label_gauss_z_col<128>, dim3(G), dim3(BLOCK), (size_t)128 * COL_LD * sizeof(float) + lh, s,
                         x, n, per_block, packed, K, t, seed, z, hist, tot);
      break;
    }
    default:
      hipLaunchKernelGGL(k_label_gauss_z_dyn, dim3(G), dim3(BLOCK), (size_t)d * BLOCK * sizeof(float) + lh, s, x, n,
                         d, per_block, packed, K, t, seed, z, hist, tot);
  }
#undef DPMM_LABELZ_CASE
  return hipGetLastError();
}

hipError_t launch_loglik_gauss(int d, const float* x, long long n, const float* packed, int K, int k_max,
                               float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_loglik_gauss_dyn, dim3(grid_for(n)), dim3(BLOCK), (size_t)d * BLOCK * sizeof(float),
                     s, x, n, d, packed, K, k_max, out);
  return hipGetLastError();
}

}  // namespace dpmm
