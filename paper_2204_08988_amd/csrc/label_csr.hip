// Count data in compressed sparse rows (multinomial and Poisson families):
// the label step (Sec. 4.1 steps (e) and (f)), the statistics update
// (Sec. 4.4) and the per-point log-likelihoods.
//
// A component's score is linear in the counts: l = c + sum_e val_e T[col_e]
// with T = log theta (multinomial; c = log w) or log lambda (Poisson;
// c = log w - sum_v lambda_v).  With a vocabulary in the tens of thousands
// and a hundred or so distinct words per row, a row touches a few hundred
// table rows, so the tables are laid out word-major: tcl[v][KS] holds the K
// cluster values of word v (KS = K rounded up to 4, the pad zero) and
// tsub[v][2K] the sub-cluster values (l, r of cluster 0, l, r of cluster 1,
// ...).  A nonzero then reads K consecutive floats, 16 bytes per lane.
//
// One wave per row.  The row's nonzeros are loaded 64 at a time (one per
// lane) and broadcast to groups of QP lanes (QP the power of two >= KS / 4,
// at most 64): group g takes nonzeros g, g + G, ... of the batch (G = 64 /
// QP), lane q of the group accumulates clusters 4q .. 4q + 3; the G partial
// sums are then added across groups.  More than 256 clusters run in chunks
// of 256.  The
// scores go to the wave's slice of LDS; the top-2 screen, the exact
// Gumbel-max over the clusters within the Gumbel range (the winner of
// max_k l_k + g_k, smaller k on ties) and the sub-label draw follow as in the
// dense kernels.  Every index read from the rows is checked: an entry out of
// range sets bit ERR_SPARSE_INPUT of the error flag and the row is skipped.
#include "kernels.hpp"

namespace dpmm {

namespace {

constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / 64;
constexpr float RGAP = GUMBEL_MAX_F - GUMBEL_MIN_F;

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// the row range of point i, or false (flag raised) when it lies outside [0, nnz]
__device__ __forceinline__ bool row_range(const long long* __restrict__ rp, long long i, long long nnz,
                                          long long& e0, long long& e1, int* err) {
  e0 = rp[i];
  e1 = rp[i + 1];
  if (e0 < 0 || e1 < e0 || e1 > nnz) {
    if ((threadIdx.x & 63) == 0) atomicOr(err, ERR_SPARSE_INPUT);
    return false;
  }
  return true;
}

// one nonzero per lane (lanes at or past m get word 0 with count 0)
__device__ __forceinline__ void load_batch(const int* __restrict__ col, const int* __restrict__ val, long long b,
                                           int m, int V, int lane, int& cl, float& vl, int* err) {
  cl = 0;
  vl = 0.0f;
  if (lane < m) {
    const int c = col[b + lane], v = val[b + lane];
    if (c >= 0 && c < V && v >= 0) {
      cl = c;
      vl = (float)v;
    } else {
      atomicOr(err, ERR_SPARSE_INPUT);
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_label_csr(const long long* __restrict__ rp, const int* __restrict__ col,
                                                     const int* __restrict__ val, long long nnz, long long n, int V,
                                                     const float* __restrict__ tcl, const float* __restrict__ tsub,
                                                     const float* __restrict__ cw, int K, int lg_qp, uint32_t t,
                                                     uint64_t seed, int* __restrict__ z,
                                                     unsigned char* __restrict__ zsub, int* __restrict__ err) {
  extern __shared__ float sc_all[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  float* sc = sc_all + (size_t)w * K;
  const int Q = (K + 3) >> 2;  // float4 per table row
  const int QP = 1 << lg_qp, G = 64 >> lg_qp;
  const int g = lane >> lg_qp, ql = lane & (QP - 1);
  const int NC = (Q + 63) >> 6;
  const float4* t4 = reinterpret_cast<const float4*>(tcl);
  for (long long i = (long long)blockIdx.x * WAVES + w; i < n; i += (long long)gridDim.x * WAVES) {
    long long e0, e1;
    if (!row_range(rp, i, nnz, e0, e1, err)) continue;
    // cluster scores into LDS
    for (int c = 0; c < NC; ++c) {
      const int q = 64 * c + ql;
      float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      for (long long b = e0; b < e1; b += 64) {
        const int m = (int)min(64LL, e1 - b);
        int cl;
        float vl;
        load_batch(col, val, b, m, V, lane, cl, vl, err);
        // uniform trip count: every lane takes part in each broadcast
        for (int u0 = 0; u0 < m; u0 += G) {
          const int u = u0 + g;  // < 64: u0 <= 64 - G
          const int cc = __shfl(cl, u);
          const float vv = __shfl(vl, u);
          if (q < Q) {
            const float4 tv = t4[(size_t)cc * Q + q];
            acc.x = fmaf(vv, tv.x, acc.x);
            acc.y = fmaf(vv, tv.y, acc.y);
            acc.z = fmaf(vv, tv.z, acc.z);
            acc.w = fmaf(vv, tv.w, acc.w);
          }
        }
      }
      for (int off = QP; off < 64; off <<= 1) {
        acc.x += __shfl_xor(acc.x, off);
        acc.y += __shfl_xor(acc.y, off);
        acc.z += __shfl_xor(acc.z, off);
        acc.w += __shfl_xor(acc.w, off);
      }
      if (g == 0 && q < Q) {
        const int k = 4 * q;
        sc[k] = cw[k] + acc.x;
        if (k + 1 < K) sc[k + 1] = cw[k + 1] + acc.y;
        if (k + 2 < K) sc[k + 2] = cw[k + 2] + acc.z;
        if (k + 3 < K) sc[k + 3] = cw[k + 3] + acc.w;
      }
    }
    wave_lds_sync();
    // top-2 screen (arg: the smallest k of the maximum)
    float m1 = -INFINITY, m2 = -INFINITY;
    int arg = 0x7fffffff;
    for (int k = lane; k < K; k += 64) {
      const float l = sc[k];
      if (l > m1) {
        m2 = m1;
        m1 = l;
        arg = k;
      } else if (l > m2) {
        m2 = l;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float o1 = __shfl_xor(m1, off), o2 = __shfl_xor(m2, off);
      const int oa = __shfl_xor(arg, off);
      const float s2 = fmaxf(fminf(m1, o1), fmaxf(m2, o2));
      if (o1 > m1 || (o1 == m1 && oa < arg)) {
        m1 = o1;
        arg = oa;
      }
      m2 = s2;
    }
    int zi = arg;
    if (m2 > m1 - RGAP) {
      // exact draw over the clusters within the Gumbel range of the leader
      const float th = m1 - RGAP;
      float best = -INFINITY;
      int win = 0x7fffffff;
      for (int k = lane; k < K; k += 64) {
        const float l = sc[k];
        if (l > th) {
          const u32x4 blk = rng_block(seed, t, (uint32_t)i, TAG_GUMBEL, (uint32_t)(k >> 2));
          const float s = l + gumbel_f(word_of(blk, k & 3));
          if (s > best || (s == best && k < win)) {
            best = s;
            win = k;
          }
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const float ob = __shfl_xor(best, off);
        const int ow = __shfl_xor(win, off);
        if (ob > best || (ob == best && ow < win)) {
          best = ob;
          win = ow;
        }
      }
      zi = win;
    }
    wave_lds_sync();  // the slice is rewritten by the next row
    // sub-cluster scores of the drawn cluster, one nonzero per lane
    const float* ts = tsub + 2 * zi;
    float al = 0.0f, ar = 0.0f;
    for (long long b = e0; b < e1; b += 64) {
      const int m = (int)min(64LL, e1 - b);
      int cl;
      float vl;
      load_batch(col, val, b, m, V, lane, cl, vl, err);
      if (lane < m) {
        const float2 r = *reinterpret_cast<const float2*>(ts + (size_t)cl * 2 * K);
        al = fmaf(vl, r.x, al);
        ar = fmaf(vl, r.y, ar);
      }
    }
    al = wave_sum(al);
    ar = wave_sum(ar);
    if (lane == 0) {
      const float delta = (cw[K + 2 * zi] + al) - (cw[K + 2 * zi + 1] + ar);
      z[i] = zi;
      zsub[i] = (unsigned char)sub_label_draw(delta, seed, t, (uint32_t)i, K);
    }
  }
}

// out[i][3K]: the K cluster scores, then l, r of every cluster
__global__ __launch_bounds__(BLOCK) void k_loglik_csr(const long long* __restrict__ rp, const int* __restrict__ col,
                                                      const int* __restrict__ val, long long nnz, long long n, int V,
                                                      const float* __restrict__ tcl, const float* __restrict__ tsub,
                                                      const float* __restrict__ cw, int K, float* __restrict__ out,
                                                      int* __restrict__ err) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int KS = (K + 3) & ~3;
  for (long long i = (long long)blockIdx.x * WAVES + w; i < n; i += (long long)gridDim.x * WAVES) {
    long long e0, e1;
    if (!row_range(rp, i, nnz, e0, e1, err)) continue;
    for (int j0 = 0; j0 < 3 * K; j0 += 64) {
      const int j = j0 + lane;
      float acc = 0.0f;
      for (long long e = e0; e < e1; ++e) {
        const int c = col[e], v = val[e];
        if (c < 0 || c >= V || v < 0) {
          if (lane == 0) atomicOr(err, ERR_SPARSE_INPUT);
          continue;
        }
        if (j < K)
          acc = fmaf((float)v, tcl[(size_t)c * KS + j], acc);
        else if (j < 3 * K)
          acc = fmaf((float)v, tsub[(size_t)c * 2 * K + (j - K)], acc);
      }
      if (j < 3 * K) out[i * 3 * K + j] = cw[j] + acc;
    }
  }
}

// counts[2K] and sums[2K][V] (zeroed by the caller): integer atomics, so the
// totals do not depend on the order of the additions
__global__ __launch_bounds__(BLOCK) void k_stats_csr(const long long* __restrict__ rp, const int* __restrict__ col,
                                                     const int* __restrict__ val, long long nnz, long long n, int V,
                                                     const int* __restrict__ z, const unsigned char* __restrict__ zsub,
                                                     int K, unsigned long long* __restrict__ counts,
                                                     unsigned long long* __restrict__ sums, int* __restrict__ err) {
  extern __shared__ int hist[];  // [2K]
  for (int s = threadIdx.x; s < 2 * K; s += BLOCK) hist[s] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (long long i = (long long)blockIdx.x * WAVES + w; i < n; i += (long long)gridDim.x * WAVES) {
    const int zi = z[i], zs = zsub[i];
    if (zi < 0 || zi >= K || zs > 1) continue;  // labels outside the clusters are not counted
    long long e0, e1;
    if (!row_range(rp, i, nnz, e0, e1, err)) continue;
    const int seg = 2 * zi + zs;
    if (lane == 0) atomicAdd(&hist[seg], 1);
    unsigned long long* srow = sums + (size_t)seg * V;
    for (long long e = e0 + lane; e < e1; e += 64) {
      const int c = col[e], v = val[e];
      if (c >= 0 && c < V && v >= 0) {
        if (v) atomicAdd(srow + c, (unsigned long long)v);
      } else {
        atomicOr(err, ERR_SPARSE_INPUT);
      }
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < 2 * K; s += BLOCK)
    if (hist[s]) atomicAdd(counts + s, (unsigned long long)hist[s]);
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// Word-major tables from the component records of k_pack_mult (slot k for
// cluster k, k_max + 2k + h for its sub-clusters; value 0 the constant c,
// values 4 .. 4 + V - 1 the log parameters): a 64 x 64 tile of (component,
// word) per workgroup, transposed through LDS; the pad of each tcl row is
// zeroed.
__global__ __launch_bounds__(BLOCK) void k_pack_csr(int K, int V, int k_max, const float* __restrict__ packed,
                                                    float* __restrict__ tcl, float* __restrict__ tsub,
                                                    float* __restrict__ cw) {
  __shared__ float tile[64][65];
  const int S = mult_rec_stride(V);
  const int KS = (K + 3) & ~3;
  const int v0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const int lane = threadIdx.x & 63, r0 = threadIdx.x >> 6;
  auto slot = [&](int j) { return j < K ? j : k_max + (j - K); };
  for (int r = r0; r < 64; r += WAVES) {
    const int j = j0 + r, v = v0 + lane;
    tile[r][lane] = (j < 3 * K && v < V) ? packed[(size_t)slot(j) * S + 4 + v] : 0.0f;
  }
  if (blockIdx.x == 0 && threadIdx.x < 64 && j0 + threadIdx.x < 3 * K)
    cw[j0 + threadIdx.x] = packed[(size_t)slot(j0 + threadIdx.x) * S];
  __syncthreads();
  for (int r = r0; r < 64; r += WAVES) {
    const int v = v0 + r, j = j0 + lane;
    if (v >= V) continue;
    if (blockIdx.y == 0 && lane < KS - K) tcl[(size_t)v * KS + K + lane] = 0.0f;
    if (j >= 3 * K) continue;
    if (j < K)
      tcl[(size_t)v * KS + j] = tile[lane][r];
    else
      tsub[(size_t)v * 2 * K + (j - K)] = tile[lane][r];
  }
}

int waves_grid(long long n) {
  long long g = (n + WAVES - 1) / WAVES;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_pack_csr(int K, int V, int k_max, const float* packed, float* tcl, float* tsub, float* cw,
                           hipStream_t s) {
  const dim3 grid((V + 63) / 64, (3 * K + 63) / 64);
  hipLaunchKernelGGL(k_pack_csr, grid, dim3(BLOCK), 0, s, K, V, k_max, packed, tcl, tsub, cw);
  return hipGetLastError();
}

hipError_t launch_label_csr(const SparseRows& x, long long n, int V, const float* tcl, const float* tsub,
                            const float* cw, int K, uint32_t t, uint64_t seed, int* z, unsigned char* zsub, int* err,
                            hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int Q = (K + 3) / 4;
  int lg = 0;
  while ((1 << lg) < Q && lg < 6) ++lg;
  const size_t lds = (size_t)WAVES * K * sizeof(float);
  hipLaunchKernelGGL(k_label_csr, dim3(waves_grid(n)), dim3(BLOCK), lds, s, x.row_ptr, x.col, x.val, x.nnz, n, V, tcl,
                     tsub, cw, K, lg, t, seed, z, zsub, err);
  return hipGetLastError();
}

hipError_t launch_loglik_csr(const SparseRows& x, long long n, int V, const float* tcl, const float* tsub,
                             const float* cw, int K, float* out, int* err, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_loglik_csr, dim3(waves_grid(n)), dim3(BLOCK), 0, s, x.row_ptr, x.col, x.val, x.nnz, n, V, tcl,
                     tsub, cw, K, out, err);
  return hipGetLastError();
}

hipError_t launch_stats_csr(const SparseRows& x, long long n, int V, const int* z, const unsigned char* zsub, int K,
                            long long* counts, long long* sums, int* err, hipStream_t s) {
  const size_t ns = 2 * (size_t)K * V;
  hipLaunchKernelGGL(k_zero_u64, dim3(std::min<size_t>((ns + 255) / 256, 4096)), dim3(256), 0, s,
                     (unsigned long long*)sums, ns);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, (unsigned long long*)counts, 2 * (size_t)K);
  if (n > 0)
    hipLaunchKernelGGL(k_stats_csr, dim3(waves_grid(n)), dim3(BLOCK), 2 * (size_t)K * sizeof(int), s, x.row_ptr,
                       x.col, x.val, x.nnz, n, V, z, zsub, K, (unsigned long long*)counts, (unsigned long long*)sums,
                       err);
  return hipGetLastError();
}

}  // namespace dpmm
