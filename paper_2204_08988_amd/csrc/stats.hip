// Sufficient statistics per sub-cluster (Sec. 4.4: counts, then the family's
// statistics, then aggregation), float64 accumulation of float32 data.
//
// Segment of a point: s = 2 z + zsub.  Gaussian statistics per segment:
// n, sum x (d) and the upper triangle of sum x x^T (d(d+1)/2, row-major),
// stored as [2K][d + d(d+1)/2] doubles plus a separate int64 count array.
// A product of two float32 values is exact in float64, so the only rounding
// is that of the float64 sums, and every sum here is taken in a fixed order:
// the same input gives the same bits whatever the timing of the waves.
//
// Gaussian, d <= 4 (d >= 5 and the large-K case take the cluster-sorted
// kernels): each lane owns float64 accumulators of every segment (in
// registers when d <= 2 and all segments' sums fit in 72 of them, in LDS
// otherwise) and adds its own points (a fixed grid-stride assignment); the
// workgroup then adds its lanes by a fixed tree and writes one partial row,
// and a second kernel adds the rows by a fixed tree (one wave per entry).
// Multinomial: lanes over points, uint32 LDS accumulators (at most 65536
// points per workgroup, so count entries below 65536 cannot overflow), int64
// flush; all integer, so the result is exact and independent of the order.
#include "kernels.hpp"

namespace dpmm {

namespace {

constexpr int BLOCK = 256;
constexpr int LDS_MAX = 160 * 1024;
constexpr int LDS_BUDGET = 64 * 1024;

// Per-lane float64 accumulators [2K][1 + E][L] (entry-major, so the lanes of
// one access hit distinct banks); lane l of workgroup g adds the points
// i = (g L + l) + j G L in increasing j.  The next U points' loads are issued
// before the current U are added (one workgroup per CU leaves few waves to
// hide the memory latency).  Then a fixed tree over the lanes, and the
// workgroup's row part[g][2K (1 + E)] (entry 0 of a segment is its count).
template <int D, int L>
__global__ __launch_bounds__(L) void k_stats_small(const float* __restrict__ x, long long n,
                                                   const int* __restrict__ z, const unsigned char* __restrict__ zsub,
                                                   int K, double* __restrict__ part) {
  constexpr int E1 = 1 + D + D * (D + 1) / 2;
  constexpr int U = 8;
  extern __shared__ double acc[];
  const int NE = 2 * K * E1;
  const int lane = threadIdx.x;
  for (int e = 0; e < NE; ++e) acc[(size_t)e * L + lane] = 0.0;
  const long long stride = (long long)gridDim.x * L;
  int seg[U];
  float xv[U][D];
  auto load = [&](long long i0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = i0 + u * stride;
      seg[u] = -1;
#pragma unroll
      for (int j = 0; j < D; ++j) xv[u][j] = 0.0f;
      if (i < n) {
        const int zi = z[i], zs = zsub[i];
        if ((unsigned)zi < (unsigned)K && zs <= 1) seg[u] = 2 * zi + zs;
#pragma unroll
        for (int j = 0; j < D; ++j) xv[u][j] = x[i * D + j];
      }
    }
  };
  long long i0 = (long long)blockIdx.x * L + lane;
  if (i0 < n) load(i0);
  for (; i0 < n; i0 += U * stride) {
    int cs[U];
    float cx[U][D];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cs[u] = seg[u];
#pragma unroll
      for (int j = 0; j < D; ++j) cx[u][j] = xv[u][j];
    }
    if (i0 + U * stride < n) load(i0 + U * stride);  // in flight while the current points are added
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (cs[u] < 0) continue;
      double* a = acc + (size_t)cs[u] * E1 * L + lane;
      a[0] += 1.0;
#pragma unroll
      for (int j = 0; j < D; ++j) a[(size_t)(1 + j) * L] += (double)cx[u][j];
      int e = 1 + D;
#pragma unroll
      for (int p = 0; p < D; ++p)
#pragma unroll
        for (int q = p; q < D; ++q, ++e) a[(size_t)e * L] += (double)cx[u][p] * (double)cx[u][q];
    }
  }
#pragma unroll
  for (int h = L / 2; h > 0; h >>= 1) {
    __syncthreads();
    if (lane < h)
      for (int e = 0; e < NE; ++e) acc[(size_t)e * L + lane] += acc[(size_t)e * L + lane + h];
  }
  __syncthreads();
  for (int e = lane; e < NE; e += L) part[(size_t)blockIdx.x * NE + e] = acc[(size_t)e * L];
}

// d <= 2 with at most REG_VALUES sums (2K (1 + E) <= 72): every lane keeps
// the sums of all segments in float64 registers and adds each of its points
// to its segment's (an add under the lane mask per segment: no data-dependent
// addressing, no LDS traffic).  Lane l of workgroup g adds the points
// i = (g L + l) + j G L in increasing j, the next U points' loads in flight
// while the current ones are added; then the wave's lanes by a fixed xor tree,
// the workgroup's waves in wave order, one partial row per workgroup.
constexpr int REG_VALUES = 72;
constexpr int REG_L = 256;
constexpr int REG_G = 512;  // at most two workgroups per CU

template <int D>
__global__ __launch_bounds__(REG_L) void k_stats_regs(const float* __restrict__ x, long long n,
                                                      const int* __restrict__ z,
                                                      const unsigned char* __restrict__ zsub, int K,
                                                      double* __restrict__ part) {
  constexpr int E1 = 1 + D + D * (D + 1) / 2;
  constexpr int SM = REG_VALUES / E1;  // segments held
  constexpr int U = 4;
  __shared__ double wsum[REG_L / 64][SM * E1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nseg = 2 * K;
  double acc[SM][E1];
#pragma unroll
  for (int q = 0; q < SM; ++q)
#pragma unroll
    for (int e = 0; e < E1; ++e) acc[q][e] = 0.0;
  const long long stride = (long long)gridDim.x * REG_L;
  int seg[U];
  float xv[U][D];
  auto load = [&](long long i0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = i0 + u * stride;
      seg[u] = -1;
#pragma unroll
      for (int j = 0; j < D; ++j) xv[u][j] = 0.0f;
      if (i < n) {
        const int zi = z[i], zs = zsub[i];
        if ((unsigned)zi < (unsigned)K && zs <= 1) seg[u] = 2 * zi + zs;
#pragma unroll
        for (int j = 0; j < D; ++j) xv[u][j] = x[i * D + j];
      }
    }
  };
  long long i0 = (long long)blockIdx.x * REG_L + threadIdx.x;
  if (i0 < n) load(i0);
  for (; i0 < n; i0 += U * stride) {
    int cs[U];
    float cx[U][D];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cs[u] = seg[u];
#pragma unroll
      for (int j = 0; j < D; ++j) cx[u][j] = xv[u][j];
    }
    if (i0 + U * stride < n) load(i0 + U * stride);  // in flight while the current points are added
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double v[E1];
      v[0] = 1.0;
#pragma unroll
      for (int j = 0; j < D; ++j) v[1 + j] = (double)cx[u][j];
      int e = 1 + D;
#pragma unroll
      for (int p = 0; p < D; ++p)
#pragma unroll
        for (int q = p; q < D; ++q, ++e) v[e] = (double)cx[u][p] * (double)cx[u][q];
#pragma unroll
      for (int q = 0; q < SM; ++q)
        if (q < nseg && cs[u] == q)
#pragma unroll
          for (int f = 0; f < E1; ++f) acc[q][f] += v[f];
    }
  }
  // the wave's lanes by a fixed xor tree, then its waves in order
#pragma unroll
  for (int q = 0; q < SM; ++q)
#pragma unroll
    for (int f = 0; f < E1; ++f) {
      double a = acc[q][f];
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) a += __shfl_xor(a, o);
      if (lane == 0) wsum[wave][q * E1 + f] = a;
    }
  __syncthreads();
  const int NE = nseg * E1;
  for (int e = threadIdx.x; e < NE; e += REG_L) {
    double a = wsum[0][e];
#pragma unroll
    for (int w = 1; w < REG_L / 64; ++w) a += wsum[w][e];
    part[(size_t)blockIdx.x * NE + e] = a;
  }
}

bool stats_regs_ok(int d, int K) { return (d == 1 || d == 2) && (size_t)2 * K * (1 + d + d * (d + 1) / 2) <= REG_VALUES; }

// counts[s] and moments[s][.] from the G partial rows: one wave per entry,
// lane l adding rows l, l + 64, ... in order, then the lanes by a fixed xor
// tree (the same bits whatever the timing).
__global__ __launch_bounds__(64) void k_stats_small_reduce(const double* __restrict__ part, int G, int K, int E,
                                                           long long* __restrict__ counts,
                                                           double* __restrict__ moments) {
  const int NE = 2 * K * (E + 1);
  const int e = blockIdx.x;
  if (e >= NE) return;
  double sum = 0.0;
  for (int g = threadIdx.x; g < G; g += 64) sum += part[(size_t)g * NE + e];
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) sum += __shfl_xor(sum, o);
  if (threadIdx.x != 0) return;
  const int sgm = e / (E + 1), f = e - sgm * (E + 1);
  if (f == 0)
    counts[sgm] = (long long)sum;  // a sum of integer counts below 2^53: exact
  else
    moments[(size_t)sgm * E + (f - 1)] = sum;
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

int stats_small_lanes(int d, int K) {
  if (d < 1 || d > 4 || K < 1) return 0;
  const size_t ne = (size_t)2 * K * (1 + d + d * (d + 1) / 2);
  for (int L = 256; L >= 64; L /= 2)
    if (ne * L * sizeof(double) <= (size_t)LDS_MAX) return L;
  return 0;
}

size_t stats_small_part_doubles(int d, int K) {
  const int L = stats_small_lanes(d, K);
  if (!L) return 0;
  const size_t row = (size_t)2 * K * (1 + d + d * (d + 1) / 2);
  const size_t lds_rows = (size_t)(STATS_SMALL_LANES / L);
  return (stats_regs_ok(d, K) && REG_G > (int)lds_rows ? (size_t)REG_G : lds_rows) * row;
}

hipError_t launch_stats_gauss(int d, const float* x, long long n, const int* z, const unsigned char* zsub,
                              int K, long long* counts, double* moments, double* part, hipStream_t s) {
  const int E = d + d * (d + 1) / 2;
  const int L = stats_small_lanes(d, K);
  if (!L || !part) return hipErrorInvalidValue;
  if (n == 0) {
    hipError_t err = launch_zero64(counts, (size_t)2 * K, s);
    if (err != hipSuccess) return err;
    return launch_zero64(moments, (size_t)2 * K * E, s);
  }
  if (stats_regs_ok(d, K)) {
    // at least 16 points per lane before the grid grows (small n: few partial rows)
    long long gl = (n + (long long)REG_L * 16 - 1) / ((long long)REG_L * 16);
    const int G = (int)(gl < 1 ? 1 : (gl > REG_G ? REG_G : gl));
    if (d == 1)
      hipLaunchKernelGGL(k_stats_regs<1>, dim3(G), dim3(REG_L), 0, s, x, n, z, zsub, K, part);
    else
      hipLaunchKernelGGL(k_stats_regs<2>, dim3(G), dim3(REG_L), 0, s, x, n, z, zsub, K, part);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int NE = 2 * K * (E + 1);
    hipLaunchKernelGGL(k_stats_small_reduce, dim3(NE), dim3(64), 0, s, part, G, K, E,
                       counts, moments);
    return hipGetLastError();
  }
  // STATS_SMALL_LANES lanes in all: one resident workgroup per CU at L = 256
  const int G = STATS_SMALL_LANES / L;
  const size_t lds = (size_t)2 * K * (E + 1) * L * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    const void* fns[] = {
        (const void*)k_stats_small<1, 256>, (const void*)k_stats_small<1, 128>, (const void*)k_stats_small<1, 64>,
        (const void*)k_stats_small<2, 256>, (const void*)k_stats_small<2, 128>, (const void*)k_stats_small<2, 64>,
        (const void*)k_stats_small<3, 256>, (const void*)k_stats_small<3, 128>, (const void*)k_stats_small<3, 64>,
        (const void*)k_stats_small<4, 256>, (const void*)k_stats_small<4, 128>, (const void*)k_stats_small<4, 64>};
    for (const void* f : fns) {
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_MAX);
      if (e != hipSuccess) return e;
    }
    attr_set = true;
  }
#define DPMM_SMALL_CASE(DD)                                                                                        \
  case DD:                                                                                                         \
    if (L == 256)                                                                                                  \
      hipLaunchKernelGGL((k_stats_small<DD, 256>), dim3(G), dim3(256), lds, s, x, n, z, zsub, K, part);            \
    else if (L == 128)                                                                                             \
      hipLaunchKernelGGL((k_stats_small<DD, 128>), dim3(G), dim3(128), lds, s, x, n, z, zsub, K, part);            \
    else                                                                                                           \
      hipLaunchKernelGGL((k_stats_small<DD, 64>), dim3(G), dim3(64), lds, s, x, n, z, zsub, K, part);              \
    break;
  switch (d) {
    DPMM_SMALL_CASE(1)
    DPMM_SMALL_CASE(2)
    DPMM_SMALL_CASE(3)
    DPMM_SMALL_CASE(4)
  }
#undef DPMM_SMALL_CASE
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int NE = 2 * K * (E + 1);
  hipLaunchKernelGGL(k_stats_small_reduce, dim3(NE), dim3(64), 0, s, part, G, K, E, counts,
                     moments);
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
