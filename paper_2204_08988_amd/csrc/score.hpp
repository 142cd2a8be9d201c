// Device helpers shared by the Gaussian label kernels: FP32 component scores,
// the top-2 screen and the lazy Gumbel-max draw (Sec. 4.1 eq. sample_labels),
// and the sub-label draw (eq. sample_sub_labels).
#pragma once
#include "common.hpp"

namespace dpmm {
namespace score {

constexpr int BLOCK = 256;  // threads per workgroup of the label kernels
constexpr float RGAP = GUMBEL_MAX_F - GUMBEL_MIN_F;

template <int D>
__device__ __forceinline__ float score_rec(const float* __restrict__ p, const float (&x)[D]) {
  float dx[D];
#pragma unroll
  for (int j = 0; j < D; ++j) dx[j] = x[j] - p[4 + j];
  const float* w = p + 4 + D;
  float q = 0.0f;
#pragma unroll
  for (int r = 0; r < D; ++r) {
    float y = 0.0f;
#pragma unroll
    for (int c = 0; c <= r; ++c) y = fmaf(w[r * (r + 1) / 2 + c], dx[c], y);
    q = fmaf(y, y, q);
  }
  return fmaf(-0.5f, q, p[0]);
}

// Generic dimension: the centred vector lives in a per-thread LDS column.
__device__ __forceinline__ float score_rec_dyn(const float* __restrict__ p, const float* __restrict__ x,
                                               float* dx, int d) {
  for (int j = 0; j < d; ++j) dx[j * BLOCK] = x[j] - p[4 + j];
  const float* w = p + 4 + d;
  float q = 0.0f;
  for (int r = 0; r < d; ++r) {
    const float* wr = w + r * (r + 1) / 2;
    float y = 0.0f;
    for (int c = 0; c <= r; ++c) y = fmaf(wr[c], dx[c * BLOCK], y);
    q = fmaf(y, y, q);
  }
  return fmaf(-0.5f, q, p[0]);
}

// FP32 score of a row stored as an LDS column (element j at xc[j * LDC]) under
// the record p; the centred row is held in registers.  With a wave-uniform p
// the record's loads are scalar.
template <int D, int LDC>
__device__ __forceinline__ float score_col(const float* __restrict__ p, const float* __restrict__ xc) {
  float dx[D];
#pragma unroll
  for (int j = 0; j < D; ++j) dx[j] = xc[j * LDC] - p[4 + j];
  const float* w = p + 4 + D;
  float q = 0.0f;
#pragma unroll
  for (int r = 0; r < D; ++r) {
    float y = 0.0f;
#pragma unroll
    for (int c = 0; c <= r; ++c) y = fmaf(w[r * (r + 1) / 2 + c], dx[c], y);
    q = fmaf(y, y, q);
  }
  return fmaf(-0.5f, q, p[0]);
}

struct Top2 {
  float m1, m2;
  int arg;
  __device__ __forceinline__ void init() {
    m1 = -INFINITY;
    m2 = -INFINITY;
    arg = 0;
  }
  __device__ __forceinline__ void push(float l, int k) {
    if (l > m1) {
      m2 = m1;
      m1 = l;
      arg = k;
    } else if (l > m2) {
      m2 = l;
    }
  }
};

template <typename ScoreFn>
__device__ __forceinline__ int lazy_gumbel_max(const Top2& t2, int K, uint32_t i, uint32_t t, uint64_t seed,
                                               ScoreFn score_k) {
  if (!(t2.m2 > t2.m1 - RGAP)) return t2.arg;
  int cached = t2.arg >> 2;
  u32x4 blk = rng_block(seed, t, i, TAG_GUMBEL, (uint32_t)cached);
  float best = t2.m1 + gumbel_f(word_of(blk, t2.arg & 3));
  int win = t2.arg;
  for (int k = 0; k < K; ++k) {
    if (k == t2.arg) continue;
    const float l = score_k(k);
    if (l + GUMBEL_MAX_F > best) {
      const int b = k >> 2;
      if (b != cached) {
        blk = rng_block(seed, t, i, TAG_GUMBEL, (uint32_t)b);
        cached = b;
      }
      const float s = l + gumbel_f(word_of(blk, k & 3));
      if (s > best || (s == best && k < win)) {
        best = s;
        win = k;
      }
    }
  }
  return win;
}

// The same draw for K <= KM with the K scores already in registers: the
// candidates are the clusters within G_max - G_min of the leader (any other
// trails the leader's perturbed score whatever the noise); their Gumbel
// blocks are taken in increasing block order, each computed at most once
// per wave, and the winner is the largest l_k + g_k, the smaller k on ties.
// Clusters that lazy_gumbel_max skips cannot win, so the label is the same.
// `last` is block K / 4 when K % 4 != 0, computed by the caller (its unused
// word is the sub-label's), and is not computed again here.
template <int KM>
__device__ __forceinline__ int lazy_gumbel_max_regs(const float (&l)[KM], const Top2& t2, int K, uint32_t i,
                                                    uint32_t t, uint64_t seed, const u32x4& last) {
  if (!(t2.m2 > t2.m1 - RGAP)) return t2.arg;
  const float floor = t2.m1 - RGAP;
  const int bl = (K & 3) ? (K >> 2) : -1;
  float best = -INFINITY;
  int win = t2.arg;
#pragma unroll
  for (int b = 0; b < (KM + 3) / 4; ++b) {
    bool need = false;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (4 * b + j < K && l[4 * b + j] > floor) need = true;
    if (need) {
      const u32x4 blk = b == bl ? last : rng_block(seed, t, i, TAG_GUMBEL, (uint32_t)b);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 4 * b + j;
        if (k < K && l[k] > floor) {
          const float s = l[k] + gumbel_f(word_of(blk, j));
          if (s > best) {
            best = s;
            win = k;
          }
        }
      }
    }
  }
  return win;
}

__device__ __forceinline__ unsigned char draw_sub(float delta, uint32_t i, uint32_t t, uint64_t seed, int K) {
  return (unsigned char)sub_label_draw(delta, seed, t, i, K);
}

}  // namespace score
}  // namespace dpmm
