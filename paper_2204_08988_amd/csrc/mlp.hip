// Learned split proposal: MLP F -> 128 -> 128 -> 1 (ReLU) on the matrix
// cores, its training kernels, set features, point selection, proposal sums
// and the statistics of a proposed partition.  (An added form; the paper has
// no learned component.)
//
// Every dense product of the forward and backward pass is one "NT" GEMM,
// C[M][N] = A[M][K] B^T with A and B^T both stored row-major with K
// contiguous (BF16), accumulated in FP32 on v_mfma_f32_32x32x16_bf16, one
// wave per 32 x 32 output tile, K masked to its true length:
//   forward  : H1 = relu(X W1 + b1)       A = X[n][Fp],   B^T = W1^T[128][Fp]
//              H2 = relu(H1 W2 + b2)      A = H1[n][128], B^T = W2^T[128][128]
//   backward : D1 = (D2 W2^T) . [H1 > 0]  A = D2[n][128], B^T = W2[128][128]
//              gW2 = H1^T D2              A = H1^T[128][n], B^T = D2^T[128][n]
//              gW1 = X^T D1               A = X^T[Fp][n],   B^T = D1^T[128][n]
// The 128 -> 1 layer, the loss gradient, bias gradients (column sums), Adam
// (FP32 master weights) and the set features run on the vector ALUs.
#include <cmath>

#include "kernels.hpp"

namespace dpmm {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

namespace {

constexpr int BLOCK = 256;
constexpr int H = MLP_HIDDEN;

// one wave computes the 32 x 32 tile (m0, n0) of C = A B^T; rows of A and B^T
// hold at least K rounded up to 16 elements (the tail is masked to zero)
__global__ __launch_bounds__(BLOCK) void k_gemm_nt(const __bf16* __restrict__ A, int lda, const __bf16* __restrict__ Bt,
                                                   int ldb, int M, int N, int K, const float* __restrict__ bias,
                                                   int relu, const __bf16* __restrict__ mask, int ldm,
                                                   float* __restrict__ out32, int ld32, int accumulate,
                                                   __bf16* __restrict__ out16, int ld16, __bf16* __restrict__ out16t,
                                                   int ld16t) {
  const int lane = threadIdx.x & 63;
  const int tiles_n = (N + 31) / 32;
  const long long tile = (long long)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
  const long long tiles = (long long)((M + 31) / 32) * tiles_n;
  if (tile >= tiles) return;
  const int m0 = (int)(tile / tiles_n) * 32, n0 = (int)(tile % tiles_n) * 32;
  const int row = m0 + (lane & 31), col = n0 + (lane & 31), kh = 8 * (lane >> 5);
  f32x16 acc = {0};
  const bf16x8 zero = {};
  // rows past M (columns past N) read row M - 1 (N - 1) and are zeroed: the loads
  // carry no branch, so the unrolled loop keeps several in flight
  const bool va = row < M, vb = col < N;
  const __bf16* pa = A + (size_t)(va ? row : M - 1) * lda + kh;
  const __bf16* pb = Bt + (size_t)(vb ? col : N - 1) * ldb + kh;
  const int kfull = K & ~15, nblk = kfull / 16;
  if (nblk > 0) {
    // four blocks of K in flight: ring slot j holds block i + j; the prefetch
    // index is clamped to the last full block (a harmless reload at the end)
    constexpr int PD = 4;
    bf16x8 ra[PD], rb[PD];
#pragma unroll
    for (int j = 0; j < PD; ++j) {
      const int kb = 16 * (j < nblk ? j : nblk - 1);
      ra[j] = *reinterpret_cast<const bf16x8*>(pa + kb);
      rb[j] = *reinterpret_cast<const bf16x8*>(pb + kb);
    }
    for (int i = 0; i < nblk; i += PD) {
#pragma unroll
      for (int j = 0; j < PD; ++j) {
        if (i + j < nblk) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va ? ra[j] : zero, vb ? rb[j] : zero, acc, 0, 0, 0);
        const int nx = i + j + PD < nblk ? i + j + PD : nblk - 1;
        ra[j] = *reinterpret_cast<const bf16x8*>(pa + 16 * nx);
        rb[j] = *reinterpret_cast<const bf16x8*>(pb + 16 * nx);
      }
    }
  }
  if (kfull < K) {
    bf16x8 a = *reinterpret_cast<const bf16x8*>(pa + kfull);
    bf16x8 b = *reinterpret_cast<const bf16x8*>(pb + kfull);
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (kfull + kh + q >= K) {
        a[q] = (__bf16)0.0f;
        b[q] = (__bf16)0.0f;
      }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va ? a : zero, vb ? b : zero, acc, 0, 0, 0);
  }
  if (col >= N) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
    if (m >= M) continue;
    float v = acc[r];
    if (bias) v += bias[col];
    if (relu) v = v > 0.0f ? v : 0.0f;
    if (mask && !((float)mask[(size_t)m * ldm + col] > 0.0f)) v = 0.0f;
    if (out32) {
      float* o = out32 + (size_t)m * ld32 + col;
      *o = accumulate ? *o + v : v;
    }
    if (out16) out16[(size_t)m * ld16 + col] = (__bf16)v;
    if (out16t) out16t[(size_t)col * ld16t + m] = (__bf16)v;
  }
}

// o[i] = H2[i] . w3 + b3
__global__ void k_out_layer(const float* __restrict__ H2, int n, const float* __restrict__ w3,
                            const float* __restrict__ b3, float* __restrict__ o) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* h = H2 + (size_t)i * H;
  float a = *b3;
  for (int j = 0; j < H; ++j) a = fmaf(h[j], w3[j], a);
  o[i] = a;
}

constexpr int OB_ROWS = 64;

// Loss gradient through the output layer for OB_ROWS rows per block, one
// thread per hidden unit: d_o = sigmoid(o) - y (BCE with logits);
// D2 = (d_o w3^T) . [H2 > 0] as BF16 row-major and transposed; the block's
// sums of gw3, gb3 and the loss sum(softplus(o) - y o) go to its row
// red[block][H + 2] (k_add_rows adds the rows in block order).
__global__ __launch_bounds__(H) void k_out_backward(const float* __restrict__ o, const float* __restrict__ y,
                                                    const float* __restrict__ H2, int n, int npad,
                                                    const float* __restrict__ w3, __bf16* __restrict__ D2,
                                                    __bf16* __restrict__ D2t, double* __restrict__ red) {
  const int j = threadIdx.x;
  const int r0 = blockIdx.x * OB_ROWS;
  const int r1 = r0 + OB_ROWS < n ? r0 + OB_ROWS : n;
  const float wj = w3[j];
  float gacc = 0.0f, bacc = 0.0f;
  double lacc = 0.0;
  for (int r = r0; r < r1; ++r) {
    const float orr = o[r];
    const float d_o = 1.0f / (1.0f + expf(-orr)) - y[r];
    const float h = H2[(size_t)r * H + j];
    const float d2 = h > 0.0f ? d_o * wj : 0.0f;
    D2[(size_t)r * H + j] = (__bf16)d2;
    D2t[(size_t)j * npad + r] = (__bf16)d2;
    gacc = fmaf(h, d_o, gacc);
    if (j == 0) {
      bacc += d_o;
      const double od = orr;
      const double sp = od > 0 ? od + log1p(exp(-od)) : log1p(exp(od));  // softplus, stable
      lacc += sp - (double)y[r] * od;
    }
  }
  double* row = red + (size_t)blockIdx.x * (H + 2);
  row[j] = gacc;
  if (j == 0) {
    row[H] = bacc;
    row[H + 1] = lacc;
  }
}

// Column sums of BF16 rows: block b sums rows b, b + G, ... of column c into
// red[b][ncol].
__global__ void k_colsum(const __bf16* __restrict__ A, int lda, int n, int ncol, double* __restrict__ red) {
  const int c = threadIdx.x;
  if (c >= ncol) return;
  float s = 0.0f;
  for (int i = blockIdx.x; i < n; i += gridDim.x) s += (float)A[(size_t)i * lda + c];
  red[(size_t)blockIdx.x * ncol + c] = s;
}

// out_c += sum over rows b < G of red[b][c] (in row order), for c < ncol;
// columns c >= nf go to the float64 outputs outd[c - nf] (the loss sum).
__global__ void k_add_rows(const double* __restrict__ red, int G, int ncol, int nf, float* __restrict__ outf,
                           double* __restrict__ outd) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  double s = 0.0;
  for (int b = 0; b < G; ++b) s += red[(size_t)b * ncol + c];
  if (c < nf)
    outf[c] += (float)s;
  else
    outd[c - nf] += s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 operand copies of the FP32 master weights: W1^T[128][Fp] (zero
// padding of the F columns), W2^T and W2 [128][128]
__global__ void k_refresh_weights(const float* __restrict__ p, int F, int Fp, __bf16* __restrict__ w1t,
                                  __bf16* __restrict__ w2t, __bf16* __restrict__ w2) {
  const float* W1 = p;
  const float* W2 = p + F * H + H;
  for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < H * Fp + H * H; id += gridDim.x * blockDim.x) {
    if (id < H * Fp) {
      const int j = id / Fp, f = id % Fp;
      w1t[id] = (__bf16)(f < F ? W1[f * H + j] : 0.0f);
    } else {
      const int q = id - H * Fp;
      const int u = q / H, v = q % H;
      w2[q] = (__bf16)W2[u * H + v];
      w2t[(size_t)v * H + u] = (__bf16)W2[u * H + v];
    }
  }
}

// Set features of the points idx[0..n) under the frame fr = [mu (d),
// P (m x d), ratios (m)] of cluster cl[q] (cl == nullptr: frame 0):
// row q = [P (x - mu), ratios, 0 ...] of width Fp (all zero when idx[q] does
// not name one of the npts points).  Outputs (each optional): X16 BF16
// [n][Fp], X16t BF16 [Fp][npad], X32 FP32 [n][F].
__global__ void k_features(const float* __restrict__ x, int d, long long npts, const int* __restrict__ idx,
                           const int* __restrict__ cl, int cl_by_point, int n, const float* __restrict__ frames, int m,
                           int F, int Fp, __bf16* __restrict__ X16, __bf16* __restrict__ X16t, int npad,
                           float* __restrict__ X32) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int fs = d + m * d + m;
  const bool valid = (unsigned long long)idx[q] < (unsigned long long)npts;  // rows past a short selection
  const float* fr = frames + (size_t)(cl ? cl[cl_by_point ? (valid ? idx[q] : 0) : q] : 0) * fs;
  const float* xi = x + (size_t)(valid ? idx[q] : 0) * d;
  for (int f = 0; f < Fp; ++f) {
    float v = 0.0f;
    if (!valid) {
    } else if (f < m) {
      const float* pr = fr + d + f * d;
      for (int c = 0; c < d; ++c) v = fmaf(pr[c], xi[c] - fr[c], v);
    } else if (f < 2 * m) {
      v = fr[d + m * d + (f - m)];
    }
    if (X16) X16[(size_t)q * Fp + f] = (__bf16)v;
    if (X16t) X16t[(size_t)f * npad + q] = (__bf16)v;
    if (X32 && f < F) X32[(size_t)q * F + f] = v;
  }
}

// FP32 feature rows [n][F] -> BF16 [n][Fp] (and optionally [Fp][npad])
__global__ void k_convert(const float* __restrict__ X32, int n, int F, int Fp, __bf16* __restrict__ X16,
                          __bf16* __restrict__ X16t, int npad) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  for (int f = 0; f < Fp; ++f) {
    const float v = f < F ? X32[(size_t)q * F + f] : 0.0f;
    X16[(size_t)q * Fp + f] = (__bf16)v;
    if (X16t) X16t[(size_t)f * npad + q] = (__bf16)v;
  }
}

// Training targets: 1 for sub-label l, flipped per cluster (flip[cl[q]], or
// flip[cl[idx[q]]] when cl is indexed by point).
__global__ void k_targets(const int* __restrict__ idx, const int* __restrict__ cl, int cl_by_point, int n,
                          const unsigned char* __restrict__ zsub, const int* __restrict__ flip, float* __restrict__ y) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int lft = zsub[idx[q]] == 0 ? 1 : 0;
  y[q] = (float)(lft ^ flip[cl[cl_by_point ? idx[q] : q]]);
}

// Proposal over rows idx[0..n): b = clip(sigmoid(o)); side A is
// u(i, t, TAG_BERN) < b (split) or z_i == merge_k1 (merge).  side[i] = 1 on
// side A, else 0; the block's sums of log b and log(1-b) over side A and over
// side B (a fixed tree) go to red[block][4] (k_add_rows adds the rows in
// block order).
__global__ __launch_bounds__(BLOCK) void k_proposal(const float* __restrict__ o, long long npts,
                                                    const int* __restrict__ idx, int n, int merge_k1,
                                                    const int* __restrict__ z, uint64_t seed, uint32_t t,
                                                    unsigned char* __restrict__ side, double* __restrict__ red) {
  __shared__ double sh[4][BLOCK];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (q < n && (unsigned long long)idx[q] < (unsigned long long)npts) {
    const int i = idx[q];
    float b = 1.0f / (1.0f + expf(-o[q]));
    b = fminf(fmaxf(b, MLP_CLIP), 1.0f - MLP_CLIP);
    const bool a = merge_k1 >= 0 ? z[i] == merge_k1 : uniform_f(rng_block(seed, t, (uint32_t)i, TAG_BERN, 0).x) < b;
    side[i] = a ? 1 : 0;
    const double lb = log((double)b), l1b = log1p(-(double)b);
    v[a ? 0 : 2] = lb;
    v[a ? 1 : 3] = l1b;
  }
  for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 4) red[(size_t)blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

// Accepted learned split: side-A points of the set go to cluster k_new, every
// point of the set gets a fresh sub-label (TAG_LEARNSUB).
__global__ void k_apply_split(long long npts, const int* __restrict__ idx, int n,
                              const unsigned char* __restrict__ side, int k_new, uint64_t seed, uint32_t t,
                              int* __restrict__ z, unsigned char* __restrict__ zsub) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int i = idx[q];
  if ((unsigned long long)i >= (unsigned long long)npts) return;
  if (side[i]) z[i] = k_new;
  zsub[i] = (unsigned char)(rng_block(seed, t, (uint32_t)i, TAG_LEARNSUB, 0).x & 1u);
}

// ---- stable selection of the points i with pred(i), in increasing order.
// Block b scans the contiguous range [b per, (b + 1) per).
struct SelectPred {
  const int* z;
  int k1, k2;       // mode 0: z == k1 or z == k2 (k2 < 0: unused)
  const int* elig;  // mode 1: z in [0, K) and elig[z] != 0
  int K;
  __device__ bool operator()(long long i) const {
    const int zi = z[i];
    if (elig) return (unsigned)zi < (unsigned)K && elig[zi] != 0;
    return zi == k1 || (k2 >= 0 && zi == k2);
  }
};

__global__ __launch_bounds__(BLOCK) void k_select_count(SelectPred pred, long long n, long long per,
                                                        int* __restrict__ cnt) {
  const long long begin = (long long)blockIdx.x * per;
  const long long end = begin + per < n ? begin + per : n;
  int total = 0;
  for (long long c0 = begin; c0 < end; c0 += BLOCK) {
    const long long i = c0 + threadIdx.x;
    total += __syncthreads_count(i < end && pred(i));
  }
  if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

// exclusive scan of cnt[0..G) in place; the total goes to cnt[G] and to
// cnt[total_at]
__global__ void k_select_scan(int* __restrict__ cnt, int G, int total_at) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int run = 0;
  for (int b = 0; b < G; ++b) {
    const int c = cnt[b];
    cnt[b] = run;
    run += c;
  }
  cnt[G] = run;
  cnt[total_at] = run;
}

__global__ __launch_bounds__(BLOCK) void k_select_write(SelectPred pred, long long n, long long per,
                                                        const int* __restrict__ base, int* __restrict__ out) {
  __shared__ int wtot[BLOCK / 64];
  const long long begin = (long long)blockIdx.x * per;
  const long long end = begin + per < n ? begin + per : n;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int run = base[blockIdx.x];
  for (long long c0 = begin; c0 < end; c0 += BLOCK) {
    const long long i = c0 + threadIdx.x;
    const bool p = i < end && pred(i);
    const unsigned long long mask = __ballot(p);
    const int pre = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wtot[w] = __popcll(mask);
    __syncthreads();
    int woff = 0, all = 0;
    for (int u = 0; u < BLOCK / 64; ++u) {
      woff += u < w ? wtot[u] : 0;
      all += wtot[u];
    }
    if (p) out[run + woff + pre] = (int)i;
    run += all;
    __syncthreads();
  }
}

// ---- float64 statistics of the two sides of a proposed partition.
// Entry e of a side: e = 0 the count, 1 <= e <= d sum x, then the upper
// triangle of sum x x^T row by row.  Block b reduces rows [b per, (b + 1) per)
// of idx into part[b][h][E + 1] (h = 0 side A, 1 side B); passes of
// SS_EPT BLOCK entries bound the registers for any d.
constexpr int SS_ROWS = 64;
constexpr int SS_EPT = 4;

__global__ __launch_bounds__(BLOCK) void k_set_stats(const float* __restrict__ x, int d, long long npts,
                                                     const int* __restrict__ idx, int n, int per,
                                                     const unsigned char* __restrict__ side,
                                                     double* __restrict__ part) {
  extern __shared__ float xs[];  // [SS_ROWS][d]
  __shared__ unsigned char sd[SS_ROWS];
  const int E1 = 1 + d + d * (d + 1) / 2;
  const int begin = blockIdx.x * per;
  const int end = begin + per < n ? begin + per : n;
  for (int e0 = 0; e0 < E1; e0 += SS_EPT * BLOCK) {
    int ea[SS_EPT], eb[SS_EPT];
    double accA[SS_EPT], accB[SS_EPT];
#pragma unroll
    for (int j = 0; j < SS_EPT; ++j) {
      const int e = e0 + j * BLOCK + threadIdx.x;
      accA[j] = accB[j] = 0.0;
      ea[j] = -2;  // no entry
      eb[j] = -1;
      if (e == 0) {
        ea[j] = -1;  // the count
      } else if (e <= d) {
        ea[j] = e - 1;
      } else if (e < E1) {
        int r = e - 1 - d, a = 0;
        while (r >= d - a) {
          r -= d - a;
          ++a;
        }
        ea[j] = a;
        eb[j] = a + r;
      }
    }
    for (int r0 = begin; r0 < end; r0 += SS_ROWS) {
      __syncthreads();
      for (int id = threadIdx.x; id < SS_ROWS * d; id += BLOCK) {
        const int rr = id / d, c = id % d;
        const int q = r0 + rr;
        const bool ok = q < end && (unsigned long long)idx[q] < (unsigned long long)npts;
        xs[id] = ok ? x[(size_t)idx[q] * d + c] : 0.0f;
      }
      if (threadIdx.x < SS_ROWS) {
        const int q = r0 + threadIdx.x;
        const bool ok = q < end && (unsigned long long)idx[q] < (unsigned long long)npts;
        sd[threadIdx.x] = ok ? side[idx[q]] : 2;
      }
      __syncthreads();
      const int rows = end - r0 < SS_ROWS ? end - r0 : SS_ROWS;
      for (int rr = 0; rr < rows; ++rr) {
        const bool A = sd[rr] == 1;
        const float* xr = xs + rr * d;
#pragma unroll
        for (int j = 0; j < SS_EPT; ++j) {
          if (ea[j] == -2) continue;
          const double v = ea[j] < 0 ? 1.0 : (eb[j] < 0 ? (double)xr[ea[j]] : (double)xr[ea[j]] * (double)xr[eb[j]]);
          if (A) accA[j] += v;
          else accB[j] += v;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < SS_EPT; ++j) {
      const int e = e0 + j * BLOCK + threadIdx.x;
      if (e < E1) {
        part[((size_t)blockIdx.x * 2 + 0) * E1 + e] = accA[j];
        part[((size_t)blockIdx.x * 2 + 1) * E1 + e] = accB[j];
      }
    }
  }
}

// part[G][2][E + 1] -> counts[slot + h], moments[(slot + h) E + e], summed in
// block order
__global__ void k_set_stats_reduce(const double* __restrict__ part, int G, int d, int slot,
                                   long long* __restrict__ counts, double* __restrict__ moments) {
  const int E1 = 1 + d + d * (d + 1) / 2;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 2 * E1) return;
  const int h = id / E1, e = id % E1;
  double s = 0.0;
  for (int b = 0; b < G; ++b) s += part[((size_t)b * 2 + h) * E1 + e];
  if (e == 0) counts[slot + h] = (long long)s;
  else moments[(size_t)(slot + h) * (E1 - 1) + (e - 1)] = s;
}

// Training batch: row j takes the selected point at position
// floor(w n_sel / 2^32), w = Philox word 0 of (entity j, counter, TAG_TRAIN).
__global__ void k_batch_pick(const int* __restrict__ sel, long long n_sel, int batch, uint64_t seed, uint32_t counter,
                             const int* __restrict__ z, int* __restrict__ bidx, int* __restrict__ bcl) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= batch) return;
  const uint32_t w = rng_block(seed, counter, (uint32_t)j, TAG_TRAIN, 0).x;
  const long long pos = (long long)(((unsigned long long)w * (unsigned long long)n_sel) >> 32);
  const int i = sel[pos];
  bidx[j] = i;
  bcl[j] = z[i];
}

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

}  // namespace

hipError_t launch_gemm_nt(const void* A, int lda, const void* Bt, int ldb, int M, int N, int K, const float* bias,
                          bool relu, const void* mask, int ldm, float* out32, int ld32, bool accumulate, void* out16,
                          int ld16, void* out16t, int ld16t, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  const long long tiles = (long long)cdiv(M, 32) * cdiv(N, 32);
  hipLaunchKernelGGL(k_gemm_nt, dim3(cdiv(tiles, BLOCK / 64)), dim3(BLOCK), 0, s, (const __bf16*)A, lda,
                     (const __bf16*)Bt, ldb, M, N, K, bias, relu ? 1 : 0, (const __bf16*)mask, ldm, out32, ld32,
                     accumulate ? 1 : 0, (__bf16*)out16, ld16, (__bf16*)out16t, ld16t);
  return hipGetLastError();
}

hipError_t launch_out_layer(const float* H2, int n, const float* w3, const float* b3, float* o, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_out_layer, dim3(cdiv(n, BLOCK)), dim3(BLOCK), 0, s, H2, n, w3, b3, o);
  return hipGetLastError();
}

hipError_t launch_out_backward(const float* o, const float* y, const float* H2, int n, int npad, const float* w3,
                               void* D2, void* D2t, float* gw3, float* gb3, double* loss, double* red,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (n > MLP_CHUNK || gb3 != gw3 + H) return hipErrorInvalidValue;  // red holds MLP_CHUNK / OB_ROWS rows
  const int G = cdiv(n, OB_ROWS);
  hipLaunchKernelGGL(k_out_backward, dim3(G), dim3(H), 0, s, o, y, H2, n, npad, w3, (__bf16*)D2, (__bf16*)D2t, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // gw3 and gb3 are adjacent in the parameter vector: columns 0 .. H of the rows, then the loss
  hipLaunchKernelGGL(k_add_rows, dim3(1), dim3(H + 64), 0, s, red, G, H + 2, H + 1, gw3, loss);
  return hipGetLastError();
}

hipError_t launch_colsum(const void* A, int lda, int n, int ncol, float* out, double* red, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (ncol > H) return hipErrorInvalidValue;
  const int G = n < 1024 ? n : 1024;
  hipLaunchKernelGGL(k_colsum, dim3(G), dim3(H), 0, s, (const __bf16*)A, lda, n, ncol, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_add_rows, dim3(1), dim3(H), 0, s, red, G, ncol, ncol, out, nullptr);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s) {
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
  hipLaunchKernelGGL(k_adam, dim3(cdiv(n, BLOCK)), dim3(BLOCK), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_refresh_weights(const float* p, int F, int Fp, void* w1t, void* w2t, void* w2, hipStream_t s) {
  hipLaunchKernelGGL(k_refresh_weights, dim3(64), dim3(BLOCK), 0, s, p, F, Fp, (__bf16*)w1t, (__bf16*)w2t,
                     (__bf16*)w2);
  return hipGetLastError();
}

hipError_t launch_features(const float* x, int d, long long npts, const int* idx, const int* cl, int n,
                           const float* frames, int m, int F, int Fp, void* X16, void* X16t, int npad, float* X32,
                           hipStream_t s, bool cl_by_point) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3(cdiv(n, BLOCK)), dim3(BLOCK), 0, s, x, d, npts, idx, cl, cl_by_point ? 1 : 0, n,
                     frames, m, F, Fp, (__bf16*)X16, (__bf16*)X16t, npad, X32);
  return hipGetLastError();
}

hipError_t launch_convert(const float* X32, int n, int F, int Fp, void* X16, void* X16t, int npad, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert, dim3(cdiv(n, BLOCK)), dim3(BLOCK), 0, s, X32, n, F, Fp, (__bf16*)X16, (__bf16*)X16t,
                     npad);
  return hipGetLastError();
}

hipError_t launch_targets(const int* idx, const int* cl, int n, const unsigned char* zsub, const int* flip, float* y,
                          hipStream_t s, bool cl_by_point) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_targets, dim3(cdiv(n, BLOCK)), dim3(BLOCK), 0, s, idx, cl, cl_by_point ? 1 : 0, n, zsub, flip,
                     y);
  return hipGetLastError();
}

hipError_t launch_proposal(const float* o, long long npts, const int* idx, int n, int merge_k1, const int* z,
                           uint64_t seed, uint32_t t, unsigned char* side, double* sums, double* red, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (n > MLP_CHUNK) return hipErrorInvalidValue;  // red holds MLP_CHUNK / BLOCK rows
  const int G = cdiv(n, BLOCK);
  hipLaunchKernelGGL(k_proposal, dim3(G), dim3(BLOCK), 0, s, o, npts, idx, n, merge_k1, z, seed, t, side, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_add_rows, dim3(1), dim3(64), 0, s, red, G, 4, 0, nullptr, sums);
  return hipGetLastError();
}

hipError_t launch_apply_split(long long npts, const int* idx, int n, const unsigned char* side, int k_new,
                              uint64_t seed, uint32_t t, int* z, unsigned char* zsub, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_apply_split, dim3(cdiv(n, BLOCK)), dim3(BLOCK), 0, s, npts, idx, n, side, k_new, seed, t, z,
                     zsub);
  return hipGetLastError();
}

hipError_t launch_select(const int* z, long long n, int k1, int k2, const int* elig, int K, int* cnt, int* out,
                         hipStream_t s) {
  SelectPred pred{z, k1, k2, elig, K};
  int G = n > 0 ? cdiv(n, 4096) : 1;
  if (G > SELECT_BLOCKS) G = SELECT_BLOCKS;
  const long long per = n > 0 ? (n + G - 1) / G : 0;
  hipLaunchKernelGGL(k_select_count, dim3(G), dim3(BLOCK), 0, s, pred, n, per, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_select_scan, dim3(1), dim3(64), 0, s, cnt, G, SELECT_BLOCKS);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_select_write, dim3(G), dim3(BLOCK), 0, s, pred, n, per, cnt, out);
  return hipGetLastError();
}

hipError_t launch_set_stats(const float* x, int d, long long npts, const int* idx, int n, const unsigned char* side,
                            double* part, int slot, long long* counts, double* moments, hipStream_t s) {
  int G = cdiv(n, 1024);
  if (G < 1) G = 1;
  if (G > SET_STATS_BLOCKS) G = SET_STATS_BLOCKS;
  const int per = n > 0 ? cdiv(n, G) : 0;
  hipLaunchKernelGGL(k_set_stats, dim3(G), dim3(BLOCK), (size_t)SS_ROWS * d * sizeof(float), s, x, d, npts, idx, n,
                     per, side, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int E1 = 1 + d + d * (d + 1) / 2;
  hipLaunchKernelGGL(k_set_stats_reduce, dim3(cdiv(2 * E1, BLOCK)), dim3(BLOCK), 0, s, part, G, d, slot, counts,
                     moments);
  return hipGetLastError();
}

hipError_t launch_batch_pick(const int* sel, long long n_sel, int batch, uint64_t seed, uint32_t counter, const int* z,
                             int* bidx, int* bcl, hipStream_t s) {
  if (batch == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_pick, dim3(cdiv(batch, BLOCK)), dim3(BLOCK), 0, s, sel, n_sel, batch, seed, counter, z,
                     bidx, bcl);
  return hipGetLastError();
}

}  // namespace dpmm
