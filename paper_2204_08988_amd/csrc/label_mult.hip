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
    float xv[VT];
#pragma unroll
    for (int v = 0; v < VT; ++v) xv[v] = v < V ? (float)x[i * V + v] : 0.0f;
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
    zs = sub_label_draw(delta, seed, t, (uint32_t)i);
    z[i] = zi;
    zsub[i] = zs;
  }
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
