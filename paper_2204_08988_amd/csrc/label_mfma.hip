// Gaussian cluster draw on the matrix cores (BF16 inputs, FP32 accumulation):
// Sec. 4.1 step (e), eq. sample_labels, for d in {32, 64, 128}.
//
// For cluster k the whitened, centred points of a tile are Y^T = W_k (X - mu_k)^T
// with W_k lower triangular (W^T W = Sigma^-1).  W_k is the MFMA A operand
// (pre-packed BF16 fragments, identical for every wave), the per-cluster centred
// points (x - mu_k) rounded to BF16 are the B operand, so after
// v_mfma_f32_32x32x16_bf16 a lane holds 16 whitened coordinates of one point
// and the squared norm needs one cross-lane add.  A wave scores 64 points (two
// 32-point tiles) and each lane ends up owning one point for the draw.
//
// BF16X3 adds the two cross terms of the hi/lo split, W_hi dx_lo + W_lo dx_hi,
// for about 16 mantissa bits.
//
// Precision guard: if the runner-up is within the Gumbel range of the leader,
// widened by an allowance for the BF16 rounding of both scores, the point is
// deferred to k_rescore_flagged, which re-scores it in FP32 on the vector ALUs
// and draws it exactly as the FP32 kernel draws it; otherwise no other cluster
// can win and the leader is the label.
#include "kernels.hpp"
#include "score.hpp"

namespace dpmm {

using namespace score;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

namespace {

// allowance on |l_bf16 - l_fp32| of a score with squared norm q
constexpr float BF16_TOL_REL = 1.0f / 32.0f;
constexpr float BF16X3_TOL_REL = 1.0f / 4096.0f;
constexpr float TOL_ABS = 0.05f;
constexpr int NCAND = RESCORE_CAND;

// Candidate clusters of one point for the FP32 re-score.  A BF16 score l with
// squared norm q stands for an FP32 score within rel q + TOL_ABS / 2 of it, so
// the FP32 maximum is at least lo_max - TOL_ABS / 2, lo_max = max (l - rel q),
// and a cluster can only win the FP32 Gumbel-max if its bound u = l + rel q
// exceeds T = lo_max - RGAP - TOL_ABS.  T only grows as clusters are scored,
// so a cluster at or below the running T never becomes a candidate: only the
// others enter the list (the NCAND largest u, in decreasing order), and the
// largest bound ever pushed out of it tells whether the list is complete.
struct Cands {
  float u[NCAND];
  int k[NCAND];
  float lo_max, ev_max;
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int j = 0; j < NCAND; ++j) {
      u[j] = -INFINITY;
      k[j] = -1;
    }
    lo_max = -INFINITY;
    ev_max = -INFINITY;
  }
  __device__ __forceinline__ float threshold() const { return lo_max - RGAP - TOL_ABS; }
  __device__ __forceinline__ void push(float l, float q, float rel, int kk) {
    lo_max = fmaxf(lo_max, fmaf(-rel, q, l));
    const float uu = fmaf(rel, q, l);
    if (uu > threshold() && uu > u[NCAND - 1]) {
      ev_max = fmaxf(ev_max, u[NCAND - 1]);
      float cu = uu;
      int ck = kk;
#pragma unroll
      for (int j = 0; j < NCAND; ++j) {
        const bool sw = cu > u[j];
        const float tu = u[j];
        const int tk = k[j];
        u[j] = sw ? cu : tu;
        k[j] = sw ? ck : tk;
        cu = sw ? tu : cu;
        ck = sw ? tk : ck;
      }
    } else if (uu > threshold()) {
      ev_max = fmaxf(ev_max, uu);  // a bound inside the window that the full list has no room for
    }
  }
};

// The main pass keeps, per point, the two largest bounds u1 >= u2 (cluster k1)
// and lo_max: exactly one cluster can win in FP32 unless u2 > T.
struct Top2U {
  float u1, u2, lo_max;
  int k1;
  __device__ __forceinline__ void init() {
    u1 = u2 = lo_max = -INFINITY;
    k1 = 0;
  }
  __device__ __forceinline__ void push(float l, float q, float rel, int kk) {
    lo_max = fmaxf(lo_max, fmaf(-rel, q, l));
    const float u = fmaf(rel, q, l);
    const bool gt1 = u > u1, gt2 = u > u2;
    u2 = gt1 ? u1 : (gt2 ? u : u2);
    u1 = gt1 ? u : u1;
    k1 = gt1 ? kk : k1;
  }
};

// Main pass, point p: certain (z = k1, the only cluster that can win) unless
// another bound reaches T; then appended to `flagged` (z = -1, not in the
// histogram) for the candidate pass and k_rescore_flagged.
__device__ __forceinline__ void finish_main(bool valid, long long p, const Top2U& t2, int* z, int* h, int* flagged,
                                            int* n_flagged, int lane) {
  const bool doubt = valid && t2.u2 > t2.lo_max - RGAP - TOL_ABS;
  const unsigned long long dm = __ballot(doubt);
  if (dm) {
    const int leader = __ffsll((long long)dm) - 1;
    int slot0 = 0;
    if (lane == leader) slot0 = atomicAdd(n_flagged, __popcll(dm));
    slot0 = __shfl(slot0, leader);
    if (doubt) flagged[slot0 + __popcll(dm & ((1ull << lane) - 1ull))] = (int)p;
  }
  if (valid) {
    z[p] = doubt ? -1 : t2.k1;
    if (!doubt) atomicAdd(&h[t2.k1], 1);
  }
}

// Candidate pass, deferred slot r: the listed clusters above T, -1 elsewhere,
// or -2 in slot 0 when a cluster above T may be missing from the list.
__device__ __forceinline__ void finish_cands(bool valid, long long r, const Cands& cd, int* cand) {
  if (!valid) return;
  const float T = cd.threshold();
  const bool complete = !(cd.ev_max > T);
  int* cs = cand + (size_t)r * NCAND;
#pragma unroll
  for (int j = 0; j < NCAND; ++j) cs[j] = complete ? (cd.u[j] > T ? cd.k[j] : -1) : (j == 0 ? -2 : -1);
}

constexpr int BLOCK32 = 512;  // threads per workgroup of the d = 32 kernel

// d = 32: the whitener fragments, means and constants of a group of up to CG
// clusters are staged in LDS once and shared by the workgroup's eight waves
// (when K <= CG, once per workgroup).  A wave scores 64 points (two 32-point
// tiles) against each cluster of the group: the per-cluster centring in FP32,
// the BF16 B operand, v_mfma_f32_32x32x16_bf16 with the W_k fragment as A, and
// the squared norm; the top-2 update is branch-free so that two clusters'
// work interleaves.  Points whose top-2 gap leaves any doubt are appended to
// `flagged` (z = -1, not in the histogram) for k_rescore_flagged.
template <bool X3, bool CANDS>
__global__ __launch_bounds__(BLOCK32) void k_label_gauss_mfma32(const float* __restrict__ x, long long n,
                                                                long long per_block, const float* __restrict__ packed,
                                                                const bf16x8* __restrict__ whi,
                                                                const bf16x8* __restrict__ wlo, int K,
                                                                int* __restrict__ z, int* __restrict__ hist,
                                                                int* __restrict__ tot, int* __restrict__ flagged,
                                                                int* __restrict__ cand, int* __restrict__ n_flagged) {
  constexpr int D = 32, KS = 2, NF = KS * 64;  // 16-byte fragments per cluster and table
  constexpr float REL = X3 ? BF16X3_TOL_REL : BF16_TOL_REL;
  constexpr int NB = X3 ? 2 : 1;               // tables per cluster (hi, lo)
  constexpr int CG = X3 ? 16 : 32;             // clusters per LDS stage (64 KB of fragments)
  constexpr int MUS = D + 4;                   // mu[D], c, padding
  constexpr int S = (4 + D + D * (D + 1) / 2 + 3) & ~3;
  extern __shared__ __align__(16) unsigned char smem[];
  bf16x8* s_w = reinterpret_cast<bf16x8*>(smem);              // [CG][NB][NF]
  float* s_mu = reinterpret_cast<float*>(s_w + CG * NB * NF);  // [CG][MUS]
  int* h = reinterpret_cast<int*>(s_mu + CG * MUS);            // [K]
  for (int k = threadIdx.x; k < K; k += BLOCK32) h[k] = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5, col = lane & 31;
  // main pass: the workgroup's points; candidate pass: the deferred slots, grid-strided
  const long long nf = CANDS ? (long long)*n_flagged : 0;
  const long long begin = CANDS ? (long long)blockIdx.x * BLOCK32 : (long long)blockIdx.x * per_block;
  const long long end = CANDS ? nf : (begin + per_block < n ? begin + per_block : n);
  const long long step = CANDS ? (long long)gridDim.x * BLOCK32 : BLOCK32;
  auto stage = [&](int g0, int cnt) {
    for (int e = threadIdx.x; e < cnt * NB * NF; e += BLOCK32) {
      const int c = e / (NB * NF), r = e - c * (NB * NF);
      const int tb = r / NF, f = r - tb * NF;
      s_w[e] = (X3 && tb ? wlo : whi)[(size_t)(g0 + c) * NF + f];
    }
    for (int e = threadIdx.x; e < cnt * MUS; e += BLOCK32) {
      const int c = e / MUS, j = e - c * MUS;
      const float* rec = packed + (size_t)(g0 + c) * S;
      s_mu[e] = j < D ? rec[4 + j] : (j == D ? rec[0] : 0.0f);
    }
  };
  const bool single = K <= CG;
  if (single && begin < end) stage(0, K);
  __syncthreads();
  for (long long chunk = begin; chunk < end; chunk += step) {
    const long long base = chunk + wave * 64;
    const long long rA = base + col, rB = base + 32 + col;
    const long long pA = rA < end ? (CANDS ? (long long)flagged[rA] : rA) : 0;
    const long long pB = rB < end ? (CANDS ? (long long)flagged[rB] : rB) : 0;
    // this lane's k-slices of the two tiles' points: dims 16 ks + 8 half + q
    float xa[KS][8], xb[KS][8];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const float4* ra = reinterpret_cast<const float4*>(x + pA * D + 16 * ks + 8 * half);
      const float4* rb = reinterpret_cast<const float4*>(x + pB * D + 16 * ks + 8 * half);
      const float4 a0 = rA < end ? ra[0] : float4{0.f, 0.f, 0.f, 0.f};
      const float4 a1 = rA < end ? ra[1] : float4{0.f, 0.f, 0.f, 0.f};
      const float4 b0 = rB < end ? rb[0] : float4{0.f, 0.f, 0.f, 0.f};
      const float4 b1 = rB < end ? rb[1] : float4{0.f, 0.f, 0.f, 0.f};
      xa[ks][0] = a0.x; xa[ks][1] = a0.y; xa[ks][2] = a0.z; xa[ks][3] = a0.w;
      xa[ks][4] = a1.x; xa[ks][5] = a1.y; xa[ks][6] = a1.z; xa[ks][7] = a1.w;
      xb[ks][0] = b0.x; xb[ks][1] = b0.y; xb[ks][2] = b0.z; xb[ks][3] = b0.w;
      xb[ks][4] = b1.x; xb[ks][5] = b1.y; xb[ks][6] = b1.z; xb[ks][7] = b1.w;
    }
    Top2U t2;
    Cands cd;
    if (CANDS)
      cd.init();
    else
      t2.init();
    for (int g0 = 0; g0 < K; g0 += CG) {
      const int cnt = K - g0 < CG ? K - g0 : CG;
      if (!single) {
        __syncthreads();  // every wave is done with the previous group
        stage(g0, cnt);
        __syncthreads();
      }
#pragma unroll 2
      for (int c = 0; c < cnt; ++c) {
        const bf16x8* cw = s_w + c * NB * NF;
        const float* cmu = s_mu + c * MUS;
        bf16x8 ba[KS], bb[KS], bal[KS], bbl[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const float4 u0 = *reinterpret_cast<const float4*>(cmu + 16 * ks + 8 * half);
          const float4 u1 = *reinterpret_cast<const float4*>(cmu + 16 * ks + 8 * half + 4);
          const float mu[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const float da = xa[ks][q] - mu[q], db = xb[ks][q] - mu[q];
            ba[ks][q] = (__bf16)da;
            bb[ks][q] = (__bf16)db;
            if (X3) {
              bal[ks][q] = (__bf16)(da - (float)ba[ks][q]);
              bbl[ks][q] = (__bf16)(db - (float)bb[ks][q]);
            }
          }
        }
        f32x16 acca = {0}, accb = {0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const bf16x8 w = cw[ks * 64 + lane];
          acca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, ba[ks], acca, 0, 0, 0);
          accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, bb[ks], accb, 0, 0, 0);
          if (X3) {
            const bf16x8 wl = cw[NF + ks * 64 + lane];
            acca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wl, ba[ks], acca, 0, 0, 0);
            accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wl, bb[ks], accb, 0, 0, 0);
            acca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, bal[ks], acca, 0, 0, 0);
            accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, bbl[ks], accb, 0, 0, 0);
          }
        }
        float qa = 0.0f, qb = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          qa = fmaf(acca[r], acca[r], qa);
          qb = fmaf(accb[r], accb[r], qb);
        }
        // lane l owns point base + l (tile A for l < 32, tile B for l >= 32):
        // it keeps its own tile's half-sum and receives the partner's
        const float qm = (half ? qb : qa) + __shfl_xor(half ? qa : qb, 32);
        const float l = fmaf(-0.5f, qm, cmu[D]);
        if (CANDS)
          cd.push(l, qm, REL, g0 + c);
        else
          t2.push(l, qm, REL, g0 + c);
      }
    }
    const long long r = base + lane;
    if (CANDS)
      finish_cands(r < end, r, cd, cand);
    else
      finish_main(r < end, r, t2, z, h, flagged, n_flagged, lane);
  }
  if (CANDS) return;
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += BLOCK32) {
    hist[(size_t)blockIdx.x * K + k] = h[k];
    if (h[k]) atomicAdd(&tot[k], h[k]);
  }
}

// d = 128: the cluster's whitener fragments (and mu, c) are staged in LDS once
// per workgroup and shared by its four waves, double-buffered: cluster k + 1 is
// fetched into registers while cluster k computes; MFMA tiles entirely above the
// diagonal of W (16 ks > 32 mt + 31) are skipped, so the matrix cores execute
// 1.25 d^2 instead of 2 d^2 flops per point-cluster.  Points whose top-2 gap
// leaves any doubt are not drawn here: they are appended to `flagged` (z = -1,
// not in the histogram) and drawn by k_rescore_flagged in FP32.
template <int D, bool X3, bool CANDS>
__global__ __launch_bounds__(BLOCK) void k_label_gauss_mfma_lds(const float* __restrict__ x, long long n,
                                                                long long per_block, const float* __restrict__ packed,
                                                                const bf16x8* __restrict__ whi,
                                                                const bf16x8* __restrict__ wlo, int K,
                                                                int* __restrict__ z, int* __restrict__ hist,
                                                                int* __restrict__ tot, int* __restrict__ flagged,
                                                                int* __restrict__ cand, int* __restrict__ n_flagged) {
  constexpr int S = (4 + D + D * (D + 1) / 2 + 3) & ~3;
  constexpr int MT = D / 32, KS = D / 16, NF = MT * KS * 64;
  constexpr float REL = X3 ? BF16X3_TOL_REL : BF16_TOL_REL;
  constexpr int PF = NF / BLOCK;  // fragments each thread stages per cluster
  constexpr int NB = X3 ? 2 : 1;  // fragment tables per cluster (hi, lo)
  constexpr int MUS = D + 4;      // mu[D], c
  static_assert(NF % BLOCK == 0 && D < BLOCK, "staging layout");
  // two staging buffers: [buf][NB][NF] fragments, then [buf][MUS] floats, then the histogram
  extern __shared__ __align__(16) unsigned char smem[];
  bf16x8* s_w = reinterpret_cast<bf16x8*>(smem);
  float* s_mu = reinterpret_cast<float*>(s_w + 2 * NB * NF);
  int* h = reinterpret_cast<int*>(s_mu + 2 * MUS);
  for (int k = threadIdx.x; k < K; k += BLOCK) h[k] = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5, col = lane & 31;
  // main pass: the workgroup's points; candidate pass: the deferred slots, grid-strided
  const long long nf = CANDS ? (long long)*n_flagged : 0;
  const long long begin = CANDS ? (long long)blockIdx.x * BLOCK : (long long)blockIdx.x * per_block;
  const long long end = CANDS ? nf : (begin + per_block < n ? begin + per_block : n);
  const long long step = CANDS ? (long long)gridDim.x * BLOCK : BLOCK;
  // staging of cluster k into buffer b: global -> registers (pf*), registers -> LDS
  bf16x8 pf[NB][PF];
  float pfmu = 0.0f;
  auto fetch = [&](int k) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      pf[0][j] = whi[(size_t)k * NF + threadIdx.x + j * BLOCK];
      if (X3) pf[NB - 1][j] = wlo[(size_t)k * NF + threadIdx.x + j * BLOCK];
    }
    const float* rec = packed + (size_t)k * S;
    pfmu = threadIdx.x < D ? rec[4 + threadIdx.x] : (threadIdx.x == D ? rec[0] : 0.0f);
  };
  auto store = [&](int b) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      s_w[(b * NB) * NF + threadIdx.x + j * BLOCK] = pf[0][j];
      if (X3) s_w[(b * NB + NB - 1) * NF + threadIdx.x + j * BLOCK] = pf[NB - 1][j];
    }
    if (threadIdx.x <= D) s_mu[b * MUS + threadIdx.x] = pfmu;
  };
  const bool any = begin < end;
  if (any) {
    fetch(0);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  // every wave runs the same number of chunks and clusters: one barrier per cluster
  for (long long chunk = begin; chunk < end; chunk += step) {
    const long long base = chunk + wave * 64;
    const long long rA = base + col, rB = base + 32 + col;
    const long long pA = rA < end ? (CANDS ? (long long)flagged[rA] : rA) : 0;
    const long long pB = rB < end ? (CANDS ? (long long)flagged[rB] : rB) : 0;
    float xa[KS][8], xb[KS][8];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = 16 * ks + 8 * half + q;
        xa[ks][q] = rA < end ? x[pA * D + j] : 0.0f;
        xb[ks][q] = rB < end ? x[pB * D + j] : 0.0f;
      }
    const bool more = chunk + step < end;
    Top2U t2;
    Cands cd;
    if (CANDS)
      cd.init();
    else
      t2.init();
    for (int k = 0; k < K; ++k) {
      // the next cluster (or the next chunk's first) is fetched while this one computes
      const bool next = k + 1 < K || more;
      if (next) fetch(k + 1 < K ? k + 1 : 0);
      const bf16x8* cw = s_w + (buf * NB) * NF;
      const bf16x8* cwl = s_w + (buf * NB + NB - 1) * NF;
      const float* cmu = s_mu + buf * MUS;
      bf16x8 ba[KS], bb[KS], bal[KS], bbl[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float mu = cmu[16 * ks + 8 * half + q];
          const float da = xa[ks][q] - mu, db = xb[ks][q] - mu;
          ba[ks][q] = (__bf16)da;
          bb[ks][q] = (__bf16)db;
          if (X3) {
            bal[ks][q] = (__bf16)(da - (float)ba[ks][q]);
            bbl[ks][q] = (__bf16)(db - (float)bb[ks][q]);
          }
        }
      float qa = 0.0f, qb = 0.0f;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        f32x16 acca = {0}, accb = {0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          if (16 * ks > 32 * mt + 31) continue;  // W is lower triangular: an all-zero tile
          const bf16x8 a = cw[(mt * KS + ks) * 64 + lane];
          acca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, ba[ks], acca, 0, 0, 0);
          accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb[ks], accb, 0, 0, 0);
          if (X3) {
            const bf16x8 al = cwl[(mt * KS + ks) * 64 + lane];
            acca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, ba[ks], acca, 0, 0, 0);
            accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bb[ks], accb, 0, 0, 0);
            acca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bal[ks], acca, 0, 0, 0);
            accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bbl[ks], accb, 0, 0, 0);
          }
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          qa = fmaf(acca[r], acca[r], qa);
          qb = fmaf(accb[r], accb[r], qb);
        }
      }
      qa += __shfl_xor(qa, 32);
      qb += __shfl_xor(qb, 32);
      const float qm = half ? qb : qa;
      const float l = fmaf(-0.5f, qm, cmu[D]);
      if (CANDS)
        cd.push(l, qm, REL, k);
      else
        t2.push(l, qm, REL, k);
      // the other buffer was last read before the previous barrier
      if (next) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
    const long long r = base + lane;
    if (CANDS)
      finish_cands(r < end, r, cd, cand);
    else
      finish_main(r < end, r, t2, z, h, flagged, n_flagged, lane);
  }
  if (CANDS) return;
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += BLOCK) {
    hist[(size_t)blockIdx.x * K + k] = h[k];
    if (h[k]) atomicAdd(&tot[k], h[k]);
  }
}

constexpr int RS_BLOCK = 64;

// FP32 re-score and lazy Gumbel-max draw of the deferred points, exactly the
// FP32 kernel's draw; the centred vector of a thread lives in an LDS column.
// With a complete candidate list only the candidates are scored (in
// increasing k, the order of the full draw): every other cluster's FP32 score
// is below the leader's by more than the Gumbel range, so the full draw skips
// it too.  Adds each drawn point to the histogram of the label-kernel block
// that owns it.
__global__ __launch_bounds__(RS_BLOCK) void k_rescore_flagged(const float* __restrict__ x, int d,
                                                              const int* __restrict__ flagged,
                                                              const int* __restrict__ cand,
                                                              const int* __restrict__ n_flagged, long long per_block,
                                                              const float* __restrict__ packed, int K, uint32_t t,
                                                              uint64_t seed, int* __restrict__ z,
                                                              int* __restrict__ hist, int* __restrict__ tot) {
  extern __shared__ float dxs[];  // [d][RS_BLOCK]
  float* dx = dxs + threadIdx.x;
  const int S = gauss_rec_stride(d);
  const int cnt = *n_flagged;
  for (int q = blockIdx.x * RS_BLOCK + threadIdx.x; q < cnt; q += gridDim.x * RS_BLOCK) {
    const long long p = flagged[q];
    const float* xp = x + p * d;
    auto score = [&](int k) {
      const float* rp = packed + (size_t)k * S;
      for (int j = 0; j < d; ++j) dx[j * RS_BLOCK] = xp[j] - rp[4 + j];
      const float* w = rp + 4 + d;
      float qq = 0.0f;
      for (int r = 0; r < d; ++r) {
        const float* wr = w + r * (r + 1) / 2;
        float y = 0.0f;
        for (int c = 0; c <= r; ++c) y = fmaf(wr[c], dx[c * RS_BLOCK], y);
        qq = fmaf(y, y, qq);
      }
      return fmaf(-0.5f, qq, rp[0]);
    };
    int ids[NCAND];
#pragma unroll
    for (int j = 0; j < NCAND; ++j) ids[j] = cand[(size_t)q * NCAND + j];
    int zi;
    if (ids[0] == -2) {
      Top2 f;
      f.init();
      for (int k = 0; k < K; ++k) f.push(score(k), k);
      zi = lazy_gumbel_max(f, K, (uint32_t)p, t, seed, score);
    } else {
      // candidates in increasing k (empty slots last)
#pragma unroll
      for (int a = 0; a < NCAND; ++a)
#pragma unroll
        for (int b = 0; b + 1 < NCAND - a; ++b) {
          const unsigned ka = (unsigned)ids[b], kb = (unsigned)ids[b + 1];
          ids[b] = ka < kb ? (int)ka : (int)kb;
          ids[b + 1] = ka < kb ? (int)kb : (int)ka;
        }
      float sc[NCAND];
      Top2 f;
      f.init();
#pragma unroll
      for (int j = 0; j < NCAND; ++j) {
        sc[j] = ids[j] >= 0 ? score(ids[j]) : -INFINITY;
        if (ids[j] >= 0) f.push(sc[j], ids[j]);
      }
      zi = f.arg;
      if (f.m2 > f.m1 - RGAP) {
        int cached = f.arg >> 2;
        u32x4 blk = rng_block(seed, t, (uint32_t)p, TAG_GUMBEL, (uint32_t)cached);
        float best = f.m1 + gumbel_f(word_of(blk, f.arg & 3));
#pragma unroll
        for (int j = 0; j < NCAND; ++j) {
          const int k = ids[j];
          if (k < 0 || k == f.arg) continue;
          if (sc[j] + GUMBEL_MAX_F > best) {
            const int b = k >> 2;
            if (b != cached) {
              blk = rng_block(seed, t, (uint32_t)p, TAG_GUMBEL, (uint32_t)b);
              cached = b;
            }
            const float s = sc[j] + gumbel_f(word_of(blk, k & 3));
            if (s > best || (s == best && k < zi)) {
              best = s;
              zi = k;
            }
          }
        }
      }
    }
    z[p] = zi;
    atomicAdd(&hist[(size_t)(p / per_block) * K + zi], 1);
    atomicAdd(&tot[zi], 1);
  }
}

// Fragment table of cluster k's whitener: element (mt, ks, lane, q) =
// W[32 mt + lane % 32][16 ks + 8 (lane / 32) + q] (zero above the diagonal).
__global__ void k_pack_wfrag(int K, int d, int k_max, const float* __restrict__ packed, __bf16* __restrict__ whi,
                             __bf16* __restrict__ wlo) {
  const int k = blockIdx.x;
  if (k >= K) return;
  const int S = gauss_rec_stride(d);
  const float* w = packed + (size_t)k * S + 4 + d;
  const int KS = d / 16;
  for (int idx = threadIdx.x; idx < d * d; idx += blockDim.x) {
    const int q = idx & 7, lane = (idx >> 3) & 63, f = idx >> 9;
    const int ks = f % KS, mt = f / KS;
    const int r = 32 * mt + (lane & 31), c = 16 * ks + 8 * (lane >> 5) + q;
    const float v = c <= r ? w[r * (r + 1) / 2 + c] : 0.0f;
    const __bf16 hi = (__bf16)v;
    whi[(size_t)k * d * d + idx] = hi;
    if (wlo) wlo[(size_t)k * d * d + idx] = (__bf16)(v - (float)hi);
  }
}

}  // namespace

bool mfma_supported(int d) { return d == 32 || d == 64 || d == 128; }

hipError_t launch_pack_wfrag(int K, int d, int k_max, const float* packed, void* whi, void* wlo, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_wfrag, dim3(K), dim3(256), 0, s, K, d, k_max, packed, (__bf16*)whi, (__bf16*)wlo);
  return hipGetLastError();
}

hipError_t launch_label_gauss_mfma(int d, bool x3, const float* x, long long n, int G, long long per_block,
                                   const float* packed, const void* whi, const void* wlo, int K, uint32_t t,
                                   uint64_t seed, int* z, int* hist, int* tot, int* flagged, int* cand,
                                   int* n_flagged, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipError_t e = launch_zero64(tot, (size_t)(K + 1) / 2 + 1, s);
  if (e != hipSuccess) return e;
  const size_t lh = (size_t)K * sizeof(int);
  const bf16x8* hi = (const bf16x8*)whi;
  const bf16x8* lo = (const bf16x8*)wlo;
  e = launch_zero64(n_flagged, 1, s);
  if (e != hipSuccess) return e;
  static bool attr_set = false;
  if (!attr_set) {  // more than 64 KB of dynamic LDS (160 KB per CU on gfx950)
    const void* fns[12] = {
        (const void*)k_label_gauss_mfma_lds<128, true, false>, (const void*)k_label_gauss_mfma_lds<128, false, false>,
        (const void*)k_label_gauss_mfma_lds<64, true, false>,  (const void*)k_label_gauss_mfma_lds<64, false, false>,
        (const void*)k_label_gauss_mfma32<true, false>,        (const void*)k_label_gauss_mfma32<false, false>,
        (const void*)k_label_gauss_mfma_lds<128, true, true>,  (const void*)k_label_gauss_mfma_lds<128, false, true>,
        (const void*)k_label_gauss_mfma_lds<64, true, true>,   (const void*)k_label_gauss_mfma_lds<64, false, true>,
        (const void*)k_label_gauss_mfma32<true, true>,         (const void*)k_label_gauss_mfma32<false, true>};
    for (const void* f : fns) {
      e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      if (e != hipSuccess) return e;
    }
    attr_set = true;
  }
  // the main pass, then the candidate pass over the points it deferred (same grid)
  for (int pass = 0; pass < 2; ++pass) {
    const bool cands = pass == 1;
    if (d == 64 || d == 128) {
      const int NF = (d / 32) * (d / 16) * 64;
      const size_t lds = 2 * ((size_t)(x3 ? 2 : 1) * NF * sizeof(bf16x8) + (d + 4) * sizeof(float)) + lh;
#define DPMM_MFMA_LDS(DD, XX, CC)                                                                           \
  hipLaunchKernelGGL((k_label_gauss_mfma_lds<DD, XX, CC>), dim3(G), dim3(BLOCK), lds, s, x, n, per_block, packed, \
                     hi, lo, K, z, hist, tot, flagged, cand, n_flagged)
      if (d == 128 && x3) {
        if (cands) DPMM_MFMA_LDS(128, true, true); else DPMM_MFMA_LDS(128, true, false);
      } else if (d == 128) {
        if (cands) DPMM_MFMA_LDS(128, false, true); else DPMM_MFMA_LDS(128, false, false);
      } else if (x3) {
        if (cands) DPMM_MFMA_LDS(64, true, true); else DPMM_MFMA_LDS(64, true, false);
      } else {
        if (cands) DPMM_MFMA_LDS(64, false, true); else DPMM_MFMA_LDS(64, false, false);
      }
#undef DPMM_MFMA_LDS
    } else if (d == 32) {
      // [CG][NB][NF] fragments (64 KB), [CG][d + 4] means and constants, the histogram
      const size_t lds = (size_t)65536 + (size_t)(x3 ? 16 : 32) * (d + 4) * sizeof(float) + lh;
#define DPMM_MFMA32(XX, CC)                                                                                 \
  hipLaunchKernelGGL((k_label_gauss_mfma32<XX, CC>), dim3(G), dim3(BLOCK32), lds, s, x, n, per_block, packed, hi, \
                     lo, K, z, hist, tot, flagged, cand, n_flagged)
      if (x3) {
        if (cands) DPMM_MFMA32(true, true); else DPMM_MFMA32(true, false);
      } else {
        if (cands) DPMM_MFMA32(false, true); else DPMM_MFMA32(false, false);
      }
#undef DPMM_MFMA32
    } else {
      return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_rescore_flagged, dim3(1024), dim3(RS_BLOCK), (size_t)d * RS_BLOCK * sizeof(float), s, x, d,
                     flagged, cand, n_flagged, per_block, packed, K, t, seed, z, hist, tot);
  return hipGetLastError();
}

}  // namespace dpmm
