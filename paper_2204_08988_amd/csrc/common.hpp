// Shared device/host helpers of the DPMM HIP library (gfx950).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), keyed
// by the 64-bit seed and addressed by the counter (entity, t, tag, block).
// Each draw of the sampler is a pure function of that address, so the label
// kernels can evaluate Gumbel noise lazily, only for the clusters that can
// still win, and still reproduce the full Gumbel-max draw.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpmm {

constexpr uint32_t TAG_GUMBEL = 0;
constexpr uint32_t TAG_LOGISTIC = 1;
constexpr uint32_t TAG_SUBINIT = 2;
constexpr uint32_t TAG_BERN = 3;
constexpr uint32_t TAG_WEIGHTS = 16;
constexpr uint32_t TAG_SUBWEIGHTS = 17;
constexpr uint32_t TAG_NIW = 18;
constexpr uint32_t TAG_DIRTHETA = 19;
constexpr uint32_t TAG_SPLIT = 20;
constexpr uint32_t TAG_MERGE = 21;
constexpr uint32_t TAG_MOVE = 22;
constexpr uint32_t ATTEMPT_STRIDE = 256;

// Bounds of the float32 Gumbel and logistic values, widened by 1e-3 to
// cover the rounding of their float32 evaluations (exact values: 16.6355323, -2.8115409,
// 16.6355323).  A cluster whose score trails the leader's by more than
// GUMBEL_MAX_F - GUMBEL_MIN_F cannot win the Gumbel-max, and a sub-label
// whose score gap exceeds LOGISTIC_MAX_F cannot be flipped by the noise.
constexpr float GUMBEL_MAX_F = 16.6365f;
constexpr float GUMBEL_MIN_F = -2.8125f;
constexpr float LOGISTIC_MAX_F = 16.6365f;

struct u32x4 {
  uint32_t x, y, z, w;
};

__host__ __device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__host__ __device__ __forceinline__ u32x4 rng_block(uint64_t seed, uint32_t t, uint32_t entity,
                                                    uint32_t tag, uint32_t blk) {
  return philox4x32_10(u32x4{entity, t, tag, blk}, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__host__ __device__ __forceinline__ uint32_t word_of(const u32x4& b, int j) {
  return j == 0 ? b.x : (j == 1 ? b.y : (j == 2 ? b.z : b.w));
}

// u = ((w >> 9) + 1/2) 2^-23: exact in float32 and float64.
__host__ __device__ __forceinline__ float uniform_f(uint32_t w) {
  return ((float)(w >> 9) + 0.5f) * 1.1920928955078125e-07f;
}
__host__ __device__ __forceinline__ double uniform_d(uint32_t w) {
  return ((double)(w >> 9) + 0.5) * 1.1920928955078125e-07;
}

// Gumbel g = -log(-log u).  Inner e = -log u: for u <= 1/2 from the hardware
// base-2 logarithm (its result is at least 1 in magnitude there, so its error
// stays near one ulp of it); for u > 1/2 from v = 1 - u (exact for these
// uniforms) as -log(1 - v) = 2 atanh(s), s = v / (2 - v) <= 1/3, summed as
// 2 s (1 + s^2/3 + ... + s^12/13), the first omitted term below 2^-26 of the
// sum.  Outer logarithm by the hardware.  Over all 2^23 uniforms the result
// is within about 3.3 2^-24 (|g| + 1) of the exact Gumbel (checked against a
// float64 evaluation with the same steps in float32).
__device__ __forceinline__ float gumbel_f(uint32_t w) {
  constexpr float LN2 = 0.69314718f;
  const float u = uniform_f(w);
  const float v = 1.0f - u;
  const float s = v * __builtin_amdgcn_rcpf(2.0f - v);
  const float s2 = s * s;
  float p = 1.0f / 13.0f;
  p = fmaf(p, s2, 1.0f / 11.0f);
  p = fmaf(p, s2, 1.0f / 9.0f);
  p = fmaf(p, s2, 1.0f / 7.0f);
  p = fmaf(p, s2, 1.0f / 5.0f);
  p = fmaf(p, s2, 1.0f / 3.0f);
  p = fmaf(p, s2, 1.0f);
  const float e = u > 0.5f ? 2.0f * s * p : -LN2 * __builtin_amdgcn_logf(u);
  return -LN2 * __builtin_amdgcn_logf(e);
}

// Word of point i's sub-label logistic at step t with K clusters: the word of
// the last Gumbel block that no cluster uses (TAG_GUMBEL block K / 4, word
// K % 4) when K is not a multiple of 4, so that a point drawing both labels
// computes that block once; else word 0 of its own block (TAG_LOGISTIC).
__device__ __forceinline__ uint32_t sub_label_word(uint64_t seed, uint32_t t, uint32_t i, int K) {
  if (K & 3) return word_of(rng_block(seed, t, i, TAG_GUMBEL, (uint32_t)(K >> 2)), K & 3);
  return rng_block(seed, t, i, TAG_LOGISTIC, 0).x;
}

// Sub-label draw (eq. sample_sub_labels) from the score gap delta = l_l - l_r
// and the logistic's word w: l (0) iff delta + L > 0 for the logistic
// L = log u - log(1 - u); since the logit is increasing this is
// u > 1 / (1 + e^delta), one exp instead of two logs.
__device__ __forceinline__ int sub_label_from_word(float delta, uint32_t w) {
  const float u = uniform_f(w);
  return u > 1.0f / (1.0f + expf(delta)) ? 0 : 1;
}

// The same with the word drawn here; a gap beyond the logistic's range
// decides without a draw.
__device__ __forceinline__ int sub_label_draw(float delta, uint64_t seed, uint32_t t, uint32_t i, int K) {
  if (delta > LOGISTIC_MAX_F) return 0;
  if (delta < -LOGISTIC_MAX_F) return 1;
  return sub_label_from_word(delta, sub_label_word(seed, t, i, K));
}

__host__ __device__ __forceinline__ double box_muller_d(uint32_t w0, uint32_t w1) {
  const double u0 = uniform_d(w0), u1 = uniform_d(w1);
  return sqrt(-2.0 * log(u0)) * cos(6.283185307179586 * u1);
}

// Standard normal draw number q of (entity, tag): one block per draw.
__host__ __device__ __forceinline__ double normal_draw(uint64_t seed, uint32_t t, uint32_t entity,
                                                      uint32_t tag, uint32_t q) {
  const u32x4 b = rng_block(seed, t, entity, tag, q * ATTEMPT_STRIDE);
  return box_muller_d(b.x, b.y);
}

// log of a Gamma(shape, 1) draw: Marsaglia & Tsang (2000), acceptance test
// log u < x^2/2 + d - d v + d log v on attempt blocks 256 q + a, with the
// u^(1/shape) boost (word 3 of the accepted block) for shape < 1.
__host__ __device__ inline double log_gamma_draw(uint64_t seed, uint32_t t, uint32_t entity,
                                                 uint32_t tag, uint32_t q, double shape) {
  const bool boost = shape < 1.0;
  const double a = boost ? shape + 1.0 : shape;
  const double d = a - 1.0 / 3.0;
  const double c = 1.0 / sqrt(9.0 * d);
  for (uint32_t att = 0; att < ATTEMPT_STRIDE; ++att) {
    const u32x4 b = rng_block(seed, t, entity, tag, q * ATTEMPT_STRIDE + att);
    const double x = box_muller_d(b.x, b.y);
    double v = 1.0 + c * x;
    if (!(v > 0.0)) continue;
    v = v * v * v;
    const double lu = log(uniform_d(b.z));
    if (lu < 0.5 * x * x + d - d * v + d * log(v)) {
      double lg = log(d) + log(v);
      if (boost) lg += log(uniform_d(b.w)) / shape;
      return lg;
    }
  }
  return log(d);
}

__host__ __device__ __forceinline__ uint32_t merge_entity(int k1, int k2) {
  return ((uint32_t)k1 << 16) | (uint32_t)k2;
}

// Packed FP32 component record used by the Gaussian label kernels:
//   [0]            c = log w - 1/2 log|Sigma| - d/2 log(2 pi)
//   [1 .. 3]       padding
//   [4 .. 4+d)     mean mu
//   [4+d ..)       whitener W (lower triangular, W^T W = Sigma^-1), rows packed:
//                  row r holds W[r][0..r]
// The record stride is rounded up to a multiple of 4 floats.
__host__ __device__ __forceinline__ int gauss_rec_stride(int d) {
  const int n = 4 + d + d * (d + 1) / 2;
  return (n + 3) & ~3;
}

// Multinomial record: [0] c = log w, [1..3] padding, [4 .. 4+V) log theta.
__host__ __device__ __forceinline__ int mult_rec_stride(int v) { return (4 + v + 3) & ~3; }

}  // namespace dpmm
