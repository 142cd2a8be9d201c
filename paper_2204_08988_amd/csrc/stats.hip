// Sufficient statistics per sub-cluster (Sec. 4.4: counts, then the family's
// statistics, then aggregation), float64 accumulation of float32 data.
//
// Segment of a point: s = 2 z + zsub.  Gaussian statistics per segment:
// n, sum x (d) and the upper triangle of sum x x^T (d(d+1)/2, row-major),
// stored as [2K][d + d(d+1)/2] doubles plus a separate int64 count array.
// A product of two float32 values is exact in float64, so the only rounding
// is that of the float64 sums.
//
// Two Gaussian kernels:
//   small d  : lanes over points, per-workgroup LDS accumulators updated with
//              LDS atomics, flushed to global memory once per workgroup;
//   any d    : per chunk of up to 8192 points a local counting sort by segment in
//              LDS, then lanes over statistic entries accumulate each
//              segment's run from LDS tiles of 64 rows, one global atomic per
//              entry and segment and chunk.
// Multinomial: lanes over points, uint32 LDS accumulators (at most 65536
// points per workgroup, so count entries below 65536 cannot overflow), int64
// flush; all integer, so the result is exact and independent of the order.
#include "kernels.hpp"

namespace dpmm {

namespace {

constexpr int BLOCK = 256;
constexpr int CHUNK_MAX = 8192;
constexpr int LDS_MAX = 160 * 1024;
constexpr int TILE = 64;
constexpr int LDS_BUDGET = 64 * 1024;

__device__ __forceinline__ int tri_index(int a, int b, int d) {
  return a * d - (a * (a - 1)) / 2 + (b - a);
}

template <int D>
__global__ __launch_bounds__(BLOCK) void k_stats_gauss_lds(const float* __restrict__ x, long long n,
                                                           const int* __restrict__ z,
                                                           const unsigned char* __restrict__ zsub, int K,
                                                           long long* __restrict__ counts,
                                                           double* __restrict__ moments) {
  constexpr int E = D + D * (D + 1) / 2;
  extern __shared__ double lds_d[];
  double* acc = lds_d;                                        // [2K][E]
  unsigned int* cnt = reinterpret_cast<unsigned int*>(acc + 2 * K * E);  // [2K]
  for (int idx = threadIdx.x; idx < 2 * K * E; idx += BLOCK) acc[idx] = 0.0;
  for (int idx = threadIdx.x; idx < 2 * K; idx += BLOCK) cnt[idx] = 0u;
  __syncthreads();
  const long long stride_pts = (long long)gridDim.x * BLOCK;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride_pts) {
    const int zi = z[i];
    const int zs = zsub[i];
    if ((unsigned)zi >= (unsigned)K || zs > 1) continue;  // labels outside the table are ignored
    const int s = 2 * zi + zs;
    float xv[D];
#pragma unroll
    for (int j = 0; j < D; ++j) xv[j] = x[i * D + j];
    atomicAdd(&cnt[s], 1u);
    double* a = acc + s * E;
#pragma unroll
    for (int j = 0; j < D; ++j) atomicAdd(&a[j], (double)xv[j]);
#pragma unroll
    for (int p = 0; p < D; ++p)
#pragma unroll
      for (int q = p; q < D; ++q) atomicAdd(&a[D + tri_index(p, q, D)], (double)xv[p] * (double)xv[q]);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 2 * K * E; idx += BLOCK)
    if (acc[idx] != 0.0) atomicAdd(&moments[idx], acc[idx]);
  for (int idx = threadIdx.x; idx < 2 * K; idx += BLOCK)
    if (cnt[idx]) atomicAdd((unsigned long long*)&counts[idx], (unsigned long long)cnt[idx]);
}

// Entries per lane for d <= 128: (128 + 128*129/2) / 256 rounded up.
constexpr int EPT = 33;

__global__ __launch_bounds__(BLOCK) void k_stats_gauss_sorted(const float* __restrict__ x, long long n, int d,
                                                              int chunk, const int* __restrict__ z,
                                                              const unsigned char* __restrict__ zsub, int K,
                                                              long long* __restrict__ counts,
                                                              double* __restrict__ moments) {
  extern __shared__ int lds_i[];
  const int G = 2 * K;
  int* cnt = lds_i;            // [G]
  int* off = cnt + G;          // [G]
  int* cur = off + G;          // [G]
  int* perm = cur + G;         // [CHUNK]
  float* xs = reinterpret_cast<float*>(perm + chunk);  // [TILE][d]
  const int E = d + d * (d + 1) / 2;
  const int tid = threadIdx.x;
  // decode this lane's entries: e < d -> sum x_a; else upper-triangle (a, b)
  short ea[EPT], eb[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = tid + j * BLOCK;
    ea[j] = -1;
    eb[j] = -1;
    if (e < d) {
      ea[j] = (short)e;
    } else if (e < E) {
      int u = e - d, a = 0;
      while (u >= d - a) {
        u -= d - a;
        ++a;
      }
      ea[j] = (short)a;
      eb[j] = (short)(a + u);
    }
  }
  for (long long base = (long long)blockIdx.x * chunk; base < n; base += (long long)gridDim.x * chunk) {
    const int m = (int)((n - base) < chunk ? (n - base) : chunk);
    for (int g = tid; g < G; g += BLOCK) cnt[g] = 0;
    __syncthreads();
    for (int p = tid; p < m; p += BLOCK) {
      const int zi = z[base + p], zs = zsub[base + p];
      if ((unsigned)zi < (unsigned)K && zs <= 1) atomicAdd(&cnt[2 * zi + zs], 1);
    }
    __syncthreads();
    if (tid == 0) {
      int acc = 0;
      for (int g = 0; g < G; ++g) {
        off[g] = acc;
        cur[g] = acc;
        acc += cnt[g];
      }
    }
    __syncthreads();
    for (int p = tid; p < m; p += BLOCK) {
      const int zi = z[base + p], zs = zsub[base + p];
      if ((unsigned)zi < (unsigned)K && zs <= 1) perm[atomicAdd(&cur[2 * zi + zs], 1)] = p;
    }
    __syncthreads();
    for (int s = 0; s < G; ++s) {
      const int cs = cnt[s];
      if (cs == 0) continue;
      double acc[EPT];
#pragma unroll
      for (int j = 0; j < EPT; ++j) acc[j] = 0.0;
      const int beg = off[s];
      for (int r0 = 0; r0 < cs; r0 += TILE) {
        const int tn = (cs - r0) < TILE ? (cs - r0) : TILE;
        for (int idx = tid; idx < tn * d; idx += BLOCK) {
          const int pr = idx / d, col = idx - pr * d;
          xs[idx] = x[(base + perm[beg + r0 + pr]) * d + col];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const int a = ea[j], b = eb[j];
          if (a < 0) continue;
          double sacc = 0.0;
          if (b < 0) {
            for (int p = 0; p < tn; ++p) sacc += (double)xs[p * d + a];
          } else {
            for (int p = 0; p < tn; ++p) sacc += (double)xs[p * d + a] * (double)xs[p * d + b];
          }
          acc[j] += sacc;
        }
        __syncthreads();
      }
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int e = tid + j * BLOCK;
        if (e < E) atomicAdd(&moments[(size_t)s * E + e], acc[j]);
      }
      if (tid == 0) atomicAdd((unsigned long long*)&counts[s], (unsigned long long)cs);
    }
    __syncthreads();
  }
}

// Count sums of the multinomial segments in LDS (uint32 partial sums).  A wave
// takes 64 consecutive rows: lane r reads row r's label, then the lanes span
// the words of one row at a time (a coalesced load through a buffer descriptor
// that covers only rows below n, eight rows in flight) and add them to the
// row's segment, distinct addresses within each LDS instruction.
__global__ __launch_bounds__(BLOCK) void k_stats_mult_lds(const int* __restrict__ x, long long n, int V,
                                                          const int* __restrict__ z,
                                                          const unsigned char* __restrict__ zsub, int K,
                                                          long long* __restrict__ counts,
                                                          long long* __restrict__ sums) {
  extern __shared__ unsigned int lds_u[];
  unsigned int* acc = lds_u;           // [2K][V]
  unsigned int* cnt = acc + 2 * K * V;  // [2K]
  for (int idx = threadIdx.x; idx < 2 * K * V + 2 * K; idx += BLOCK) lds_u[idx] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long wstep = (long long)gridDim.x * (BLOCK / 64) * 64;
  for (long long base = ((long long)blockIdx.x * (BLOCK / 64) + wave) * 64; base < n; base += wstep) {
    const long long i = base + lane;
    int seg = -1;
    if (i < n) {
      const int zi = z[i], zs = zsub[i];
      if ((unsigned)zi < (unsigned)K && zs <= 1) seg = 2 * zi + zs;
    }
    if (seg >= 0) atomicAdd(&cnt[seg], 1u);
    const long long rows = n - base < 64 ? n - base : 64;
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc((void*)(x + base * V), (short)0, (int)(rows * V * 4), 0x00020000);
    for (int c0 = 0; c0 < V; c0 += 64) {
      const int c = c0 + lane;
      for (int r0 = 0; r0 < 64; r0 += 8) {
        int val[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) val[j] = __builtin_amdgcn_raw_buffer_load_b32(rx, ((r0 + j) * V + c) * 4, 0, 0);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int sj = __builtin_amdgcn_readlane(seg, r0 + j);
          if (sj >= 0 && c < V && val[j]) atomicAdd(&acc[sj * V + c], (unsigned int)val[j]);
        }
      }
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 2 * K * V; idx += BLOCK)
    if (acc[idx]) atomicAdd((unsigned long long*)&sums[idx], (unsigned long long)acc[idx]);
  for (int idx = threadIdx.x; idx < 2 * K; idx += BLOCK)
    if (cnt[idx]) atomicAdd((unsigned long long*)&counts[idx], (unsigned long long)cnt[idx]);
}

__global__ __launch_bounds__(BLOCK) void k_stats_mult_global(const int* __restrict__ x, long long n, int V,
                                                             const int* __restrict__ z,
                                                             const unsigned char* __restrict__ zsub, int K,
                                                             long long* __restrict__ counts,
                                                             long long* __restrict__ sums) {
  const long long stride_pts = (long long)gridDim.x * BLOCK;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride_pts) {
    const int zi = z[i];
    const int zs = zsub[i];
    if ((unsigned)zi >= (unsigned)K || zs > 1) continue;
    const int s = 2 * zi + zs;
    atomicAdd((unsigned long long*)&counts[s], 1ull);
    const int* xi = x + i * V;
    for (int v = 0; v < V; ++v) {
      const int c = xi[v];
      if (c) atomicAdd((unsigned long long*)&sums[(size_t)s * V + v], (unsigned long long)c);
    }
  }
}

int stats_grid(long long n, long long per_block) {
  long long g = (n + per_block - 1) / per_block;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_stats_gauss(int d, const float* x, long long n, const int* z, const unsigned char* zsub,
                              int K, long long* counts, double* moments, hipStream_t s) {
  const int E = d + d * (d + 1) / 2;
  hipError_t err = launch_zero64(counts, (size_t)2 * K, s);
  if (err != hipSuccess) return err;
  err = launch_zero64(moments, (size_t)2 * K * E, s);
  if (err != hipSuccess) return err;
  if (n == 0) return hipSuccess;
  const size_t lds_small = (size_t)2 * K * E * sizeof(double) + (size_t)2 * K * sizeof(unsigned);
  if (d <= 4 && lds_small <= LDS_BUDGET) {
    const int g = stats_grid(n, (long long)BLOCK * 16);
#define DPMM_STATS_CASE(DD)                                                                          \
  case DD:                                                                                           \
    hipLaunchKernelGGL(k_stats_gauss_lds<DD>, dim3(g), dim3(BLOCK), lds_small, s, x, n, z, zsub, K,  \
                       counts, moments);                                                             \
    break;
    switch (d) {
      DPMM_STATS_CASE(1)
      DPMM_STATS_CASE(2)
      DPMM_STATS_CASE(3)
      DPMM_STATS_CASE(4)
    }
#undef DPMM_STATS_CASE
    return hipGetLastError();
  }
  // chunk of points sorted in LDS: as large as CHUNK_MAX allows within the LDS limit
  const long long fixed = (long long)3 * 2 * K * sizeof(int) + (long long)TILE * d * sizeof(float);
  long long chunk = (LDS_MAX - fixed) / (long long)sizeof(int);
  chunk = chunk > CHUNK_MAX ? CHUNK_MAX : (chunk / BLOCK) * BLOCK;
  if (chunk < BLOCK) return hipErrorInvalidValue;
  const size_t lds = (size_t)fixed + (size_t)chunk * sizeof(int);
  hipLaunchKernelGGL(k_stats_gauss_sorted, dim3(stats_grid(n, chunk)), dim3(BLOCK), lds, s, x, n, d, (int)chunk,
                     z, zsub, K, counts, moments);
  return hipGetLastError();
}

hipError_t launch_stats_mult(int V, const int* x, long long n, const int* z, const unsigned char* zsub,
                             int K, long long* counts, long long* sums, hipStream_t s) {
  hipError_t err = launch_zero64(counts, (size_t)2 * K, s);
  if (err != hipSuccess) return err;
  err = launch_zero64(sums, (size_t)2 * K * V, s);
  if (err != hipSuccess) return err;
  if (n == 0) return hipSuccess;
  const size_t lds = ((size_t)2 * K * V + 2 * K) * sizeof(unsigned int);
  if (lds <= LDS_BUDGET) {
    // uint32 partial sums: at most 65536 points per workgroup, so entries below
    // 65536 cannot overflow a partial sum
    long long g = stats_grid(n, (long long)BLOCK * 32);
    if ((n + g - 1) / g > 65536) g = (n + 65535) / 65536;
    hipLaunchKernelGGL(k_stats_mult_lds, dim3((unsigned)g), dim3(BLOCK), lds, s, x, n, V, z, zsub, K, counts,
                       sums);
  } else {
    hipLaunchKernelGGL(k_stats_mult_global, dim3(stats_grid(n, (long long)BLOCK * 4)), dim3(BLOCK), 0, s, x, n,
                       V, z, zsub, K, counts, sums);
  }
  return hipGetLastError();
}

}  // namespace dpmm
