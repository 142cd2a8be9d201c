// Workgroup-parallel float64 dense kernels for one small d x d matrix held in
// LDS (or global scratch), row-major.  All are right-looking: at step j the
// whole workgroup updates the trailing part in parallel, so every step costs a
// few barriers and independent LDS accesses instead of a serial dot product.
// Threads form rows of 32 (tx = column lane, ty = row lane), so the loops over
// a block of the matrix need no integer division (the workgroup size is a
// multiple of 32).  Every element receives the same sequence of updates as in
// a serial right-looking loop.
#pragma once
#include "common.hpp"

namespace dpmm {

// In-place lower Cholesky a = L L^T (row stride ld, d when 0); the strict
// upper triangle is zeroed.  Returns false (on every thread) if a pivot is not
// positive and finite.
__device__ inline bool wg_cholesky(double* a, int d, int* flag, int ld = 0) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int tx = tid & 31, ty = tid >> 5, nty = nt >> 5;
  if (ld == 0) ld = d;
  if (tid == 0) *flag = 1;
  __syncthreads();
  for (int j = 0; j < d; ++j) {
    if (tid == 0) {
      double s = a[j * ld + j];
      if (!(s > 0.0) || !isfinite(s)) {
        *flag = 0;
        s = 1.0;
      }
      a[j * ld + j] = sqrt(s);
    }
    __syncthreads();
    const double inv = 1.0 / a[j * ld + j];
    for (int i = j + 1 + tid; i < d; i += nt) a[i * ld + j] *= inv;
    __syncthreads();
    // trailing update of the lower triangle: a_ik -= a_ij a_kj, j < k <= i
    for (int i = j + 1 + ty; i < d; i += nty) {
      const double aij = a[i * ld + j];
      for (int k = j + 1 + tx; k <= i; k += 32) a[i * ld + k] -= aij * a[k * ld + j];
    }
    __syncthreads();
  }
  for (int i = ty; i < d; i += nty)
    for (int j = i + 1 + tx; j < d; j += 32) a[i * ld + j] = 0.0;
  __syncthreads();
  const bool ok = *flag != 0;
  __syncthreads();
  return ok;
}

// W = G^-1 for lower-triangular G (W lower triangular), W must not alias G.
__device__ inline void wg_lower_inverse(const double* G, double* W, int d) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int tx = tid & 31, ty = tid >> 5, nty = nt >> 5;
  for (int i = ty; i < d; i += nty)
    for (int c = tx; c < d; c += 32) W[i * d + c] = i == c ? 1.0 : 0.0;
  __syncthreads();
  // forward elimination on [G | I] one row at a time: row j of W is final
  // after dividing by G_jj; it is then eliminated from the rows below.
  for (int j = 0; j < d; ++j) {
    const double inv = 1.0 / G[j * d + j];
    for (int c = tid; c <= j; c += nt) W[j * d + c] *= inv;
    __syncthreads();
    for (int i = j + 1 + ty; i < d; i += nty) {
      const double gij = G[i * d + j];
      for (int c = tx; c <= j; c += 32) W[i * d + c] -= gij * W[j * d + c];
    }
    __syncthreads();
  }
}

// W = G^-1 in place for lower-triangular G (row stride ld), column by column
// from the last: W_jj = 1 / G_jj and, for i > j,
//   W_ij = -W_jj sum_{j < k <= i} W_ik G_kj,
// which reads the finished columns k > j of W and the untouched column j of G.
// Threads of a row of 32 split the sum over k and add their parts by
// shuffles; tmp holds d doubles (the new column before it is stored).
__device__ inline void wg_lower_inverse_inplace(double* a, int d, int ld, double* tmp) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int tx = tid & 31, ty = tid >> 5, nty = nt >> 5;
  for (int j = d - 1; j >= 0; --j) {
    const double wjj = 1.0 / a[j * ld + j];
    // every row block runs the same number of passes, so the shuffles see whole rows of 32
    const int rows = d - 1 - j, passes = (rows + nty - 1) / nty;
    for (int p = 0; p < passes; ++p) {
      const int i = j + 1 + ty + p * nty;
      double s = 0.0;
      if (i < d)
        for (int k = j + 1 + tx; k <= i; k += 32) s += a[i * ld + k] * a[k * ld + j];
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (i < d && tx == 0) tmp[i] = -wjj * s;
    }
    __syncthreads();
    if (tid == 0) a[j * ld + j] = wjj;
    for (int i = j + 1 + tid; i < d; i += nt) a[i * ld + j] = tmp[i];
    __syncthreads();
  }
}

// F = B A^-T for lower-triangular A, in place on F (F holds B on entry):
// column j of F is final after dividing by A_jj, then removed from the later
// columns, F[:, q] -= F[:, j] A[q][j] for q > j.
__device__ inline void wg_right_solve_lower_t(double* F, const double* A, int d) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int tx = tid & 31, ty = tid >> 5, nty = nt >> 5;
  for (int j = 0; j < d; ++j) {
    const double inv = 1.0 / A[j * d + j];
    for (int r = tid; r < d; r += nt) F[r * d + j] *= inv;
    __syncthreads();
    for (int r = ty; r < d; r += nty) {
      const double frj = F[r * d + j];
      for (int q = j + 1 + tx; q < d; q += 32) F[r * d + q] -= frj * A[q * d + j];
    }
    __syncthreads();
  }
}

}  // namespace dpmm
