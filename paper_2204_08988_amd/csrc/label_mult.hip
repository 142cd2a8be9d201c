// Multinomial label step, float32 VALU path: Sec. 4.1 steps (e) and (f)
// with multinomial components (Sec. 2.1).
//
// Score of a component: l = log w + sum_v x_v log theta_v (the multinomial
// coefficient is the same for every component and is left out).  One lane per
// point; the count row is converted to float32 once (counts below 2^24 are
// exact) and held in registers, the uniform cluster loop reads log theta with
// scalar loads.  Label and sub-label draws as in the Gaussian kernel: top-2
// screen, lazy Gumbel-max, logistic skipped outside its range.
#include "kernels.hpp"

namespace dpmm {

namespace {

constexpr int BLOCK = 256;
constexpr float RGAP = GUMBEL_MAX_F - GUMBEL_MIN_F;
constexpr size_t MULT_MFMA_LDS_MAX = 96 * 1024;  // log theta staged for every cluster (two workgroups per CU)
constexpr int BUF_DWORD3 = 0x00020000;            // raw buffer descriptor word 3 (gfx9 family)

template <int VT>
__device__ __forceinline__ float score_mult(const float* __restrict__ p, const float (&x)[VT]) {
  float a0 = p[0], a1 = 0.0f;
#pragma unroll
  for (int v = 0; v < VT; v += 2) {
    a0 = fmaf(x[v], p[4 + v], a0);
    if (v + 1 < VT) a1 = fmaf(x[v + 1], p[5 + v], a1);
  }
  return a0 + a1;
}

template <int VT>
__global__ __launch_bounds__(BLOCK) void k_label_mult(const int* __restrict__ x, long long n, int V,
                                                      const float* __restrict__ packed, int K, int k_max,
                                                      uint32_t t, uint64_t seed, int* __restrict__ z,
                                                      unsigned char* __restrict__ zsub) {
  const int S = mult_rec_stride(V);
  const long long stride_pts = (long long)gridDim.x * BLOCK;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride_pts) {
    // unconditional loads (clamped word index, zeroed afterwards): all in flight together
    float xv[VT];
#pragma unroll
    for (int v = 0; v < VT; ++v) {
      const int c = x[i * V + (v < V ? v : V - 1)];
      xv[v] = v < V ? (float)c : 0.0f;
    }
    float m1 = -INFINITY, m2 = -INFINITY;
    int arg = 0;
    for (int k = 0; k < K; ++k) {
      const float l = score_mult<VT>(packed + (size_t)k * S, xv);
      if (l > m1) {
        m2 = m1;
        m1 = l;
        arg = k;
      } else if (l > m2) {
        m2 = l;
      }
    }
    int zi = arg;
    if (m2 > m1 - RGAP) {
      int cached = arg >> 2;
      u32x4 blk = rng_block(seed, t, (uint32_t)i, TAG_GUMBEL, (uint32_t)cached);
      float best = m1 + gumbel_f(word_of(blk, arg & 3));
      for (int k = 0; k < K; ++k) {
        if (k == arg) continue;
        const float l = score_mult<VT>(packed + (size_t)k * S, xv);
        if (l + GUMBEL_MAX_F > best) {
          const int b = k >> 2;
          if (b != cached) {
            blk = rng_block(seed, t, (uint32_t)i, TAG_GUMBEL, (uint32_t)b);
            cached = b;
          }
          const float s = l + gumbel_f(word_of(blk, k & 3));
          if (s > best || (s == best && k < zi)) {
            best = s;
            zi = k;
          }
        }
      }
    }
    const float* ps = packed + (size_t)(k_max + 2 * zi) * S;
    const float delta = score_mult<VT>(ps, xv) - score_mult<VT>(ps + S, xv);
    unsigned char zs;
    zs = sub_label_draw(delta, seed, t, (uint32_t)i, K);
    z[i] = zi;
    zsub[i] = zs;
  }
}

// The same draw with the scores on the FP32 matrix cores (v_mfma_f32_32x32x2_f32):
// a wave takes 64 points (two 32-point tiles) against blocks of 32 clusters,
// A = log theta of the block (staged in LDS for all K clusters once per
// workgroup, zero past V, row stride odd), B = the counts (word 2 s + h at step
// s on lane half h), and the accumulators start at log w (-inf for the padding
// clusters of the last block).  A lane ends with 16 of a point's K scores per
// block; the top-2 screen runs over the lane and its partner (lane ^ 32).  Only
// a wave holding a point whose runner-up lies within the Gumbel range computes
// its scores again and draws every cluster above m1 - RGAP: the winner of
// max (l_k + g_k), smaller k on ties, with the Philox words of the vector-ALU
// kernel (the same winner as its streaming draw, which skips only clusters
// that cannot beat the running best).  The sub-label then comes from the two
// sub-cluster scores of the point's cluster on the vector ALUs.
template <int VH>
__global__ __launch_bounds__(BLOCK) void k_label_mult_mfma(const int* __restrict__ x, long long n, int V,
                                                           const float* __restrict__ packed, int K, int k_max,
                                                           uint32_t t, uint64_t seed, int* __restrict__ z,
                                                           unsigned char* __restrict__ zsub) {
  typedef float f32x16 __attribute__((ext_vector_type(16)));
  constexpr int LDV = 2 * VH + 1;  // odd row stride
  const int S = mult_rec_stride(V);
  const int KB = (K + 31) / 32;
  extern __shared__ float th[];  // [32 KB][LDV] log theta, then [32 KB] log w
  float* cw = th + (size_t)KB * 32 * LDV;
  // eight loads in flight per thread (clamped addresses, zeroed afterwards)
  for (int i0 = threadIdx.x; i0 < KB * 32 * LDV; i0 += 8 * BLOCK) {
    float tv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = i0 + u * BLOCK, k = idx / LDV, v = idx - k * LDV;
      const bool in = idx < KB * 32 * LDV && k < K && v < V;
      const float val = packed[in ? (size_t)k * S + 4 + v : 0];
      tv[u] = in ? val : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u * BLOCK < KB * 32 * LDV) th[i0 + u * BLOCK] = tv[u];
  }
  for (int k = threadIdx.x; k < KB * 32; k += BLOCK) cw[k] = k < K ? packed[(size_t)k * S] : -INFINITY;
  __syncthreads();
  const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // scalar: the buffer descriptors below are too
  auto scores = [&](int b, const float (&xa)[VH], const float (&xb)[VH], f32x16& acca, f32x16& accb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float c0 = cw[32 * b + 8 * (r >> 2) + 4 * h + (r & 3)];
      acca[r] = c0;
      accb[r] = c0;
    }
    const float* ar = th + (size_t)(32 * b + col) * LDV + h;
#pragma unroll
    for (int st = 0; st < VH; ++st) {
      const float a = ar[2 * st];
      acca = __builtin_amdgcn_mfma_f32_32x32x2f32(a, xa[st], acca, 0, 0, 0);
      accb = __builtin_amdgcn_mfma_f32_32x32x2f32(a, xb[st], accb, 0, 0, 0);
    }
  };
  for (long long chunk = (long long)blockIdx.x * BLOCK; chunk < n; chunk += (long long)gridDim.x * BLOCK) {
    const long long base = chunk + wave * 64;
    const long long pA = base + col, pB = base + 32 + col;
    // the wave's 64 rows through a buffer descriptor that covers only rows below n
    // (loads past it return 0): one offset per lane, the word as an immediate, no
    // branches, so every load is in flight at once; words past V are zeroed
    const long long rows = n - base < 64 ? (n - base > 0 ? n - base : 0) : 64;
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(x + (rows > 0 ? base : 0) * V), (short)0, (int)(rows * V * 4), BUF_DWORD3);
    const int oA = (col * V + h) * 4, oB = ((32 + col) * V + h) * 4;
    float xa[VH], xb[VH];
#pragma unroll
    for (int st = 0; st < VH; ++st) {
      const int ia = __builtin_amdgcn_raw_buffer_load_b32(rx, oA + 8 * st, 0, 0);
      const int ib = __builtin_amdgcn_raw_buffer_load_b32(rx, oB + 8 * st, 0, 0);
      xa[st] = 2 * st + h < V ? (float)ia : 0.0f;
      xb[st] = 2 * st + h < V ? (float)ib : 0.0f;
    }
    // top-2 over this lane's clusters of each tile's point, then with the partner lane
    float a1 = -INFINITY, a2 = -INFINITY, b1 = -INFINITY, b2 = -INFINITY;
    int ka = 0, kb = 0;
    for (int b = 0; b < KB; ++b) {
      f32x16 acca, accb;
      scores(b, xa, xb, acca, accb);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int k = 32 * b + 8 * (r >> 2) + 4 * h + (r & 3);
        const float la = acca[r], lb = accb[r];
        if (la > a1) {
          a2 = a1;
          a1 = la;
          ka = k;
        } else if (la > a2) {
          a2 = la;
        }
        if (lb > b1) {
          b2 = b1;
          b1 = lb;
          kb = k;
        } else if (lb > b2) {
          b2 = lb;
        }
      }
    }
    auto merge2 = [&](float& m1, float& m2, int& kk) {
      const float o1 = __shfl_xor(m1, 32), o2 = __shfl_xor(m2, 32);
      const int ok = __shfl_xor(kk, 32);
      const float s2 = fmaxf(fminf(m1, o1), fmaxf(m2, o2));
      if (o1 > m1 || (o1 == m1 && ok < kk)) {
        m1 = o1;
        kk = ok;
      }
      m2 = s2;
    };
    merge2(a1, a2, ka);
    merge2(b1, b2, kb);
    const bool da = pA < n && a2 > a1 - RGAP, db = pB < n && b2 > b1 - RGAP;
    int za = ka, zb = kb;
    if (__ballot(da || db)) {
      // exact draw over the clusters above m1 - RGAP
      const float ta = a1 - RGAP, tb = b1 - RGAP;
      float sa = -INFINITY, sb = -INFINITY;
      int wa = 0x7fffffff, wb = 0x7fffffff;
      for (int b = 0; b < KB; ++b) {
        f32x16 acca, accb;
        scores(b, xa, xb, acca, accb);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int k0 = 32 * b + 8 * g + 4 * h;
          bool ca = false, cb = false;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            ca = ca || (k0 + j < K && acca[4 * g + j] > ta);
            cb = cb || (k0 + j < K && accb[4 * g + j] > tb);
          }
          if (da && ca) {
            const u32x4 blk = rng_block(seed, t, (uint32_t)pA, TAG_GUMBEL, (uint32_t)(k0 >> 2));
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (k0 + j < K && acca[4 * g + j] > ta) {
                const float sv = acca[4 * g + j] + gumbel_f(word_of(blk, j));
                if (sv > sa || (sv == sa && k0 + j < wa)) {
                  sa = sv;
                  wa = k0 + j;
                }
              }
          }
          if (db && cb) {
            const u32x4 blk = rng_block(seed, t, (uint32_t)pB, TAG_GUMBEL, (uint32_t)(k0 >> 2));
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (k0 + j < K && accb[4 * g + j] > tb) {
                const float sv = accb[4 * g + j] + gumbel_f(word_of(blk, j));
                if (sv > sb || (sv == sb && k0 + j < wb)) {
                  sb = sv;
                  wb = k0 + j;
                }
              }
          }
        }
      }
      auto merge_best = [&](float& sv, int& w) {
        const float os = __shfl_xor(sv, 32);
        const int ow = __shfl_xor(w, 32);
        if (os > sv || (os == sv && ow < w)) {
          sv = os;
          w = ow;
        }
      };
      merge_best(sa, wa);
      merge_best(sb, wb);
      if (da) za = wa;
      if (db) zb = wb;
    }
    // the lane's own point: tile A on the lower half, tile B on the upper
    const long long i = h ? pB : pA;
    if (i < n) {
      const int zi = h ? zb : za;
      float xv[2 * VH];
#pragma unroll
      for (int v = 0; v < 2 * VH; ++v) {
        const int c = __builtin_amdgcn_raw_buffer_load_b32(rx, lane * V * 4 + 4 * v, 0, 0);
        xv[v] = v < V ? (float)c : 0.0f;
      }
      const float* ps = packed + (size_t)(k_max + 2 * zi) * S;
      const float delta = score_mult<2 * VH>(ps, xv) - score_mult<2 * VH>(ps + S, xv);
      z[i] = zi;
      zsub[i] = (unsigned char)sub_label_draw(delta, seed, t, (uint32_t)i, K);
    }
  }
}

size_t label_mult_mfma_lds(int V, int K) {
  const int VH = V <= 32 ? 16 : (V <= 64 ? 32 : 64);
  const size_t kb = (size_t)(K + 31) / 32;
  return (kb * 32 * (2 * VH + 1) + kb * 32) * sizeof(float);
}

__global__ __launch_bounds__(BLOCK) void k_loglik_mult(const int* __restrict__ x, long long n, int V,
                                                       const float* __restrict__ packed, int K, int k_max,
                                                       float* __restrict__ out) {
  const int S = mult_rec_stride(V);
  const long long stride_pts = (long long)gridDim.x * BLOCK;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride_pts) {
    const int* xi = x + i * V;
    float* o = out + i * 3 * K;
    for (int j = 0; j < 3 * K; ++j) {
      const int slot = j < K ? j : k_max + (j - K);
      const float* p = packed + (size_t)slot * S;
      float a = p[0];
      for (int v = 0; v < V; ++v) a = fmaf((float)xi[v], p[4 + v], a);
      o[j] = a;
    }
  }
}

int grid_for(long long n) {
  long long g = (n + BLOCK - 1) / BLOCK;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_label_mult(int V, const int* x, long long n, const float* packed, int K, int k_max,
                             uint32_t t, uint64_t seed, int* z, unsigned char* zsub, hipStream_t s) {
  if (n == 0) return hipSuccess;
  // the matrix-core kernel while log theta of every cluster fits in LDS
  const size_t lds = label_mult_mfma_lds(V, K);
  if (V <= 128 && lds <= MULT_MFMA_LDS_MAX) {
    static bool attr_set = false;
    if (!attr_set) {
      const void* fns[3] = {(const void*)k_label_mult_mfma<16>, (const void*)k_label_mult_mfma<32>,
                            (const void*)k_label_mult_mfma<64>};
      for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)MULT_MFMA_LDS_MAX);
        if (e != hipSuccess) return e;
      }
      attr_set = true;
    }
    long long g = (n + BLOCK - 1) / BLOCK;
    if (g > 1024) g = 1024;
    if (V <= 32)
      hipLaunchKernelGGL(k_label_mult_mfma<16>, dim3(g), dim3(BLOCK), lds, s, x, n, V, packed, K, k_max, t, seed, z,
                         zsub);
    else if (V <= 64)
      hipLaunchKernelGGL(k_label_mult_mfma<32>, dim3(g), dim3(BLOCK), lds, s, x, n, V, packed, K, k_max, t, seed, z,
                         zsub);
    else
      hipLaunchKernelGGL(k_label_mult_mfma<64>, dim3(g), dim3(BLOCK), lds, s, x, n, V, packed, K, k_max, t, seed, z,
                         zsub);
    return hipGetLastError();
  }
  const int g = grid_for(n);
  if (V <= 32) {
    hipLaunchKernelGGL(k_label_mult<32>, dim3(g), dim3(BLOCK), 0, s, x, n, V, packed, K, k_max, t, seed, z, zsub);
  } else if (V <= 64) {
    hipLaunchKernelGGL(k_label_mult<64>, dim3(g), dim3(BLOCK), 0, s, x, n, V, packed, K, k_max, t, seed, z, zsub);
  } else if (V <= 128) {
    hipLaunchKernelGGL(k_label_mult<128>, dim3(g), dim3(BLOCK), 0, s, x, n, V, packed, K, k_max, t, seed, z,
                       zsub);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_loglik_mult(int V, const int* x, long long n, const float* packed, int K, int k_max,
                              float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_loglik_mult, dim3(grid_for(n)), dim3(BLOCK), 0, s, x, n, V, packed, K, k_max, out);
  return hipGetLastError();
}

}  // namespace dpmm
