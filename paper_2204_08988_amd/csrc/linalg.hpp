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

// ---- Blocked forms for one d x d matrix resident in LDS (d <= 128, row
// stride ld), eight-column panels: a panel costs two workgroup barriers
// instead of two or three per column.  The element updates of the Cholesky
// and of the right solve are the same fused multiply-adds, in the same order,
// as those of the column-by-column forms above.

constexpr int PNL = 8;  // panel width

// lower-triangle tile u (row-major over I >= J) of an nb x nb grid of tiles
__device__ __forceinline__ void tri_tile(int u, int& I, int& J) {
  int i = (int)((sqrtf(8.0f * (float)u + 1.0f) - 1.0f) * 0.5f);
  while (i * (i + 1) / 2 > u) --i;
  while ((i + 1) * (i + 2) / 2 <= u) ++i;
  I = i;
  J = u - i * (i + 1) / 2;
}

// In-place lower Cholesky a = L L^T (strict upper triangle zeroed); false on
// every thread if a pivot is not positive and finite.  Per panel: every
// thread of rows j0 ... d - 1 factors the diagonal block in registers and
// finishes its own row of the panel (the block's rows, or the solve against
// it); then each thread updates one 4 x 4 tile of the trailing lower triangle
// by the panel's columns.
__device__ inline bool wg_cholesky_panel(double* a, int d, int ld, int* flag) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) *flag = 1;
  __syncthreads();
  for (int j0 = 0; j0 < d; j0 += PNL) {
    const int w = d - j0 < PNL ? d - j0 : PNL;
    const int i = j0 + tid;
    double lrow[PNL];
    if (i < d) {
      double L[PNL][PNL];
      bool bad = false;
#pragma unroll
      for (int c = 0; c < PNL; ++c) {
        // columns past the matrix (last panel) factor as the identity
        const bool cin = c < w;
        double s = a[(j0 + (cin ? c : 0)) * ld + j0 + (cin ? c : 0)];
#pragma unroll
        for (int cc = 0; cc < PNL; ++cc)
          if (cc < c) s = fma(-L[c][cc], L[c][cc], s);
        if (cin && (!(s > 0.0) || !isfinite(s))) bad = true;
        if (!cin || !(s > 0.0) || !isfinite(s)) s = 1.0;
        L[c][c] = sqrt(s);
        const double inv = 1.0 / L[c][c];
#pragma unroll
        for (int r = 0; r < PNL; ++r) {
          if (r <= c) continue;
          const bool rin = cin && r < w;
          double v = a[(j0 + (rin ? r : 0)) * ld + j0 + (rin ? c : 0)];
          v = rin ? v : 0.0;
#pragma unroll
          for (int cc = 0; cc < PNL; ++cc)
            if (cc < c) v = fma(-L[r][cc], L[c][cc], v);
          L[r][c] = v * inv;
        }
      }
      if (tid < w) {
        // the block's rows are written after the barrier (other threads read the block first)
#pragma unroll
        for (int r = 0; r < PNL; ++r)
          if (r == tid) {
#pragma unroll
            for (int c = 0; c < PNL; ++c) lrow[c] = L[r][c];
          }
      } else {
        double v[PNL];
#pragma unroll
        for (int c = 0; c < PNL; ++c) v[c] = c < w ? a[i * ld + j0 + c] : 0.0;
#pragma unroll
        for (int c = 0; c < PNL; ++c) {
          double t = v[c];
#pragma unroll
          for (int cc = 0; cc < PNL; ++cc)
            if (cc < c) t = fma(-v[cc], L[c][cc], t);
          v[c] = c < w ? t * (1.0 / L[c][c]) : 0.0;
        }
#pragma unroll
        for (int c = 0; c < PNL; ++c)
          if (c < w) a[i * ld + j0 + c] = v[c];
      }
      if (tid == 0 && bad) *flag = 0;
    }
    __syncthreads();
    if (tid < w) {
#pragma unroll
      for (int c = 0; c < PNL; ++c)
        if (c <= tid) a[(j0 + tid) * ld + j0 + c] = lrow[c];
    }
    // trailing lower triangle [j0 + w, d)^2 in 4 x 4 tiles (rows below the block only)
    const int t0 = j0 + w, T = d - t0;
    if (T > 0) {
      const int nb = (T + 3) / 4, ntile = nb * (nb + 1) / 2;
      for (int u = tid; u < ntile; u += nt) {
        int I, J;
        tri_tile(u, I, J);
        double li[4][PNL], lj[4][PNL];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ra = min(t0 + 4 * I + r, d - 1), rb = min(t0 + 4 * J + r, d - 1);
#pragma unroll
          for (int c = 0; c < PNL; ++c) {
            li[r][c] = c < w ? a[ra * ld + j0 + c] : 0.0;
            lj[r][c] = c < w ? a[rb * ld + j0 + c] : 0.0;
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ra = t0 + 4 * I + r;
          if (ra >= d) continue;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int cb = t0 + 4 * J + q;
            if (cb > ra || cb >= d) continue;
            double v = a[ra * ld + cb];
#pragma unroll
            for (int c = 0; c < PNL; ++c)
              if (c < w) v = fma(-li[r][c], lj[q][c], v);
            a[ra * ld + cb] = v;
          }
        }
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < d * d; idx += nt) {
    const int r = idx / d, c = idx - r * d;
    if (c > r) a[r * ld + c] = 0.0;
  }
  __syncthreads();
  const bool ok = *flag != 0;
  __syncthreads();
  return ok;
}

// F = F A^-T in place for lower-triangular A given by rows of A^T (At[j d + i]
// = A[i][j], global memory), F full d x d: per panel the panel's columns of
// A^T go to LDS (apan, PNL x d doubles), each row of F is solved against the
// panel's diagonal block in registers, then the columns right of the panel
// lose the panel's contribution (4 x 4 tiles of F).  rdiag: d doubles, 1 / A_jj.
__device__ inline void wg_right_solve_lt_panel(double* F, int d, int ld, const double* __restrict__ At,
                                               double* apan, double* rdiag) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j = tid; j < d; j += nt) rdiag[j] = 1.0 / At[(size_t)j * d + j];
  for (int j0 = 0; j0 < d; j0 += PNL) {
    const int w = d - j0 < PNL ? d - j0 : PNL;
    // columns j0 ... j0 + w - 1 of A (rows of A^T) into LDS
    for (int idx = tid; idx < w * d; idx += nt) apan[idx] = At[(size_t)j0 * d + idx];
    __syncthreads();
    if (tid < d) {
      double v[PNL];
#pragma unroll
      for (int c = 0; c < PNL; ++c) v[c] = c < w ? F[tid * ld + j0 + c] : 0.0;
#pragma unroll
      for (int c = 0; c < PNL; ++c) {
        if (c < w) {
          v[c] *= rdiag[j0 + c];
#pragma unroll
          for (int q = 0; q < PNL; ++q)
            if (q > c && q < w) v[q] = fma(-v[c], apan[c * d + j0 + q], v[q]);
        }
      }
#pragma unroll
      for (int c = 0; c < PNL; ++c)
        if (c < w) F[tid * ld + j0 + c] = v[c];
    }
    __syncthreads();
    const int t0 = j0 + w, T = d - t0;
    if (T > 0) {
      const int nbr = (d + 3) / 4, nbc = (T + 3) / 4;
      for (int u = tid; u < nbr * nbc; u += nt) {
        const int I = u / nbc, J = u - I * nbc;
        double fr[4][PNL], aq[4][PNL];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rr = min(4 * I + r, d - 1), qq = min(t0 + 4 * J + r, d - 1);
#pragma unroll
          for (int c = 0; c < PNL; ++c) {
            fr[r][c] = c < w ? F[rr * ld + j0 + c] : 0.0;
            aq[r][c] = c < w ? apan[c * d + qq] : 0.0;
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rr = 4 * I + r;
          if (rr >= d) continue;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int cq = t0 + 4 * J + q;
            if (cq >= d) continue;
            double v = F[rr * ld + cq];
#pragma unroll
            for (int c = 0; c < PNL; ++c)
              if (c < w) v = fma(-fr[r][c], aq[q][c], v);
            F[rr * ld + cq] = v;
          }
        }
      }
    }
    __syncthreads();
  }
}

// W = G^-1 in place for lower-triangular G, panels from the last: with Q the
// rows below panel P (W_QQ already inverted in place),
//   W_PP = G_PP^-1,  W_QP = -W_QQ (G_QP W_PP),
// the inner product first into tbuf (up to (d - PNL) x PNL doubles).
__device__ inline void wg_lower_inverse_panel(double* a, int d, int ld, double* tbuf) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int npan = (d + PNL - 1) / PNL;
  for (int p = npan - 1; p >= 0; --p) {
    const int j0 = p * PNL, w = d - j0 < PNL ? d - j0 : PNL, q0 = j0 + w, nq = d - q0;
    // W_PP (every thread that needs it, in registers): forward substitution on G_PP X = I
    double Wp[PNL][PNL];
    const bool need = tid < (nq > w ? nq : w);
    if (need) {
#pragma unroll
      for (int c = 0; c < PNL; ++c) {
#pragma unroll
        for (int r = 0; r < PNL; ++r) Wp[r][c] = 0.0;
        if (c >= w) continue;
        Wp[c][c] = 1.0 / a[(j0 + c) * ld + j0 + c];
#pragma unroll
        for (int r = 0; r < PNL; ++r) {
          if (r <= c || r >= w) continue;
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < PNL; ++k)
            if (k >= c && k < r) s = fma(a[(j0 + r) * ld + j0 + k], Wp[k][c], s);
          Wp[r][c] = -s / a[(j0 + r) * ld + j0 + r];
        }
      }
    }
    // T = G_QP W_PP (row q0 + tid)
    if (tid < nq) {
      double g[PNL];
#pragma unroll
      for (int c = 0; c < PNL; ++c) g[c] = c < w ? a[(q0 + tid) * ld + j0 + c] : 0.0;
#pragma unroll
      for (int c = 0; c < PNL; ++c) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < PNL; ++k)
          if (k >= c && k < w) s = fma(g[k], Wp[k][c], s);
        if (c < w) tbuf[tid * PNL + c] = s;
      }
    }
    __syncthreads();
    // W_PP into the diagonal block; W_QP = -W_QQ T, one output per thread and pass
    if (tid < w) {
#pragma unroll
      for (int r = 0; r < PNL; ++r)
        if (r == tid) {
#pragma unroll
          for (int c = 0; c < PNL; ++c)
            if (c <= r) a[(j0 + r) * ld + j0 + c] = Wp[r][c];
        }
    }
    for (int o = tid; o < nq * w; o += nt) {
      const int qi = o / w, c = o - qi * w;
      const double* wr = a + (q0 + qi) * ld + q0;
      double s = 0.0;
      for (int k = 0; k <= qi; ++k) s = fma(wr[k], tbuf[k * PNL + c], s);
      a[(q0 + qi) * ld + j0 + c] = -s;
    }
    __syncthreads();
  }
}

}  // namespace dpmm
