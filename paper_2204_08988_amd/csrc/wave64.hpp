// Wave-level (64-lane) float64 helpers for kernels that give one wave to one
// small matrix: lane i owns row i, uniform values travel by v_readlane, and
// broadcast rows go through LDS with no workgroup barrier.
#pragma once
#include "common.hpp"

namespace dpmm {
namespace wave64 {

__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Keeps the compiler from hoisting the next rows' LDS reads above this point
// (a whole triangle of broadcast reads in flight would not fit in registers).
__device__ __forceinline__ void issue_fence() { __asm__ volatile("" ::: "memory"); }

// LDS writes of one lane made visible to the wave's other lanes
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1 / sqrt(s) from the hardware estimate and two Newton steps (within an ulp
// or two of the correctly rounded value)
__device__ __forceinline__ double rsqrt_refined(double s) {
  double y = __builtin_amdgcn_rsq(s);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-s * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Right-looking Cholesky of the matrix whose row `lane` is r (D x D): the
// pivot and the entries L_kj of the scaled column j come by v_readlane (into
// scalar registers, used directly as FMA operands) for the trailing update
// a_ik -= a_ij a_kj, so a step waits on no memory and the next pivot depends
// only on one read and one FMA.  Afterwards r is row `lane` of L (zero above
// the diagonal) and diag its pivot.  A pivot that is not positive and finite
// is replaced by 1 and reported by the (wave-uniform) return value.  Entries
// right of the diagonal are scratch during the loop and are cleared at the
// end.
template <int D>
__device__ __forceinline__ bool wave_cholesky(double (&r)[D], int lane, double& diag) {
  bool ok = true;
  diag = 1.0;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double s = readlane_d(r[j], j);
    if (!(s > 0.0) || !isfinite(s)) {
      ok = false;
      s = 1.0;
    }
    const double inv = rsqrt_refined(s), ljj = s * inv;
    if (lane == j) diag = ljj;
    r[j] = lane == j ? ljj : r[j] * inv;
#pragma unroll
    for (int k = j + 1; k < D; ++k) r[k] = fma(-r[j], readlane_d(r[j], k), r[k]);
  }
#pragma unroll
  for (int j = 0; j < D; ++j)
    if (j > lane) r[j] = 0.0;
  return ok;
}

}  // namespace wave64
}  // namespace dpmm
