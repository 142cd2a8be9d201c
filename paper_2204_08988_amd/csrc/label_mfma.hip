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
// The BF16 main pass at d = 64, 128 (k_label_gauss_mfma_uc) centres the points
// once on a centre common to all clusters and starts each cluster's
// accumulators at W_k (c - mu_k), so that the rows are rounded to BF16 once per
// step instead of once per cluster; each of its scores carries an interval
// that bounds the BF16 and FP32 rounding errors.
//
// Precision guard: if the runner-up is within the Gumbel range of the leader,
// widened by an allowance for the BF16 rounding of both scores, the point is
// deferred to k_rescore_flagged, which re-scores it in FP32 on the vector ALUs
// and draws it exactly as the FP32 kernel draws it; otherwise no other cluster
// can win and the leader is the label.
#include <hip/hip_ext.h>

#include <climits>

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

// arr[bucket] += 1 for every active lane, as one atomic per distinct bucket of
// the wave (deferred points pile onto few clusters; per-lane atomics on a
// handful of addresses serialise).  Call with every lane of the wave.
__device__ __forceinline__ void wave_count_add(bool active, long long bucket, int* arr) {
  const int lane = threadIdx.x & 63;
  unsigned long long pend = __ballot(active);
  while (pend) {
    const int l0 = __ffsll((long long)pend) - 1;
    const long long b0 = __shfl(bucket, l0);
    const unsigned long long m = __ballot(active && bucket == b0);
    if (lane == l0) atomicAdd(&arr[b0], __popcll(m));
    pend &= ~m;
  }
}

// Candidate clusters of one point for the FP32 re-score.  A BF16 score l with
// squared norm q stands for an FP32 score within rel q + TOL_ABS / 2 of it, so
// the FP32 maximum is at least lo_max - TOL_ABS / 2, lo_max = max (l - rel q),
// and a cluster can only win the FP32 Gumbel-max if its bound u = l + rel q
// exceeds T = lo_max - RGAP - TOL_ABS.  T only grows as clusters are scored,
// so a cluster at or below the running T never becomes a candidate: only the
// others enter the list (the NCAND largest u, in decreasing order), and the
// largest bound ever pushed out of it tells whether the list is complete.
struct Cands {
  float u[NCAND], q[NCAND];
  int k[NCAND];
  float lo_max, ev_max;
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int j = 0; j < NCAND; ++j) {
      u[j] = -INFINITY;
      q[j] = 0.0f;
      k[j] = -1;
    }
    lo_max = -INFINITY;
    ev_max = -INFINITY;
  }
  __device__ __forceinline__ float threshold() const { return lo_max - RGAP - TOL_ABS; }
  __device__ __forceinline__ void push(float l, float q, float rel, int kk) {
    lo_max = fmaxf(lo_max, fmaf(-rel, q, l));
    push_u(fmaf(rel, q, l), q, kk);
  }
  // a bound uu (squared norm q, cluster kk) against the current lo_max
  __device__ __forceinline__ void push_u(float uu, float q, int kk) {
    if (uu > threshold() && uu > u[NCAND - 1]) {
      ev_max = fmaxf(ev_max, u[NCAND - 1]);
      float cu = uu, cq = q;
      int ck = kk;
#pragma unroll
      for (int j = 0; j < NCAND; ++j) {
        const bool sw = cu > u[j];
        const float tu = u[j], tq = this->q[j];
        const int tk = k[j];
        u[j] = sw ? cu : tu;
        this->q[j] = sw ? cq : tq;
        k[j] = sw ? ck : tk;
        cu = sw ? tu : cu;
        cq = sw ? tq : cq;
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
    push_bounds(fmaf(-rel, q, l), fmaf(rel, q, l), kk);
  }
  // a score known to lie in [lo, u]
  __device__ __forceinline__ void push_bounds(float lo, float u, int kk) {
    lo_max = fmaxf(lo_max, lo);
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

// Candidate pass (bf16x3 scores, allowance rel q + TOL_ABS / 2 each), deferred
// slot r of point p: with a complete list the candidates' Gumbel values are
// drawn here (the same words as the FP32 draw).  If the perturbed leader's
// lower bound beats every other candidate's upper bound, the FP32 draw picks
// the same cluster: z[p] is written and the point counted, and slot 0 of the
// list becomes -3.  Otherwise the list holds the candidates (-1 elsewhere) or
// -2 in slot 0 when a cluster above T may be missing, for k_rescore_flagged.
__device__ __forceinline__ void finish_cands(bool valid, long long r, long long p, const Cands& cd, float rel,
                                             int K, long long per_block, uint32_t t, uint64_t seed, int* z,
                                             int* hist, int* tot, int* cand) {
  const float T = cd.threshold();
  const bool complete = !(cd.ev_max > T);
  bool sure = false;
  int kb = -1;
  if (valid && complete) {
    float pb = -INFINITY, tb = 0.0f;
    float pv[NCAND], tv[NCAND];
#pragma unroll
    for (int j = 0; j < NCAND; ++j) {
      pv[j] = -INFINITY;
      tv[j] = 0.0f;
      if (cd.k[j] >= 0 && cd.u[j] > T) {
        const int k = cd.k[j];
        const float l = fmaf(-rel, cd.q[j], cd.u[j]);
        const u32x4 blk = rng_block(seed, t, (uint32_t)p, TAG_GUMBEL, (uint32_t)(k >> 2));
        pv[j] = l + gumbel_f(word_of(blk, k & 3));
        tv[j] = fmaf(rel, cd.q[j], 0.5f * TOL_ABS);
        if (pv[j] > pb || (pv[j] == pb && k < kb)) {
          pb = pv[j];
          tb = tv[j];
          kb = k;
        }
      }
    }
    sure = kb >= 0;
#pragma unroll
    for (int j = 0; j < NCAND; ++j)
      if (cd.k[j] >= 0 && cd.k[j] != kb && cd.u[j] > T) sure = sure && (pb - tb > pv[j] + tv[j]);
  }
  if (valid) {
    int* cs = cand + (size_t)r * NCAND;
    if (sure) {
      z[p] = kb;
      cs[0] = -3;
    } else {
#pragma unroll
      for (int j = 0; j < NCAND; ++j) cs[j] = complete ? (cd.u[j] > T ? cd.k[j] : -1) : (j == 0 ? -2 : -1);
    }
  }
  wave_count_add(sure, sure ? (p / per_block) * K + kb : 0, hist);
  wave_count_add(sure, sure ? kb : 0, tot);
}

// The split candidate pass's lists of deferred point r (one per cluster group)
// merged in group order: lo_max and the evicted bound are the groups' maxima,
// and every listed bound above the merged threshold enters one list (a bound a
// group dropped lay below its own threshold, at most the merged one).  The
// result holds every cluster that can win, as the single pass's list does, and
// finish_cands draws or lists from it.  Lanes of a wave take consecutive points.
__global__ __launch_bounds__(256) void k_cands_merge(const int* __restrict__ n_flagged, int ng, int cap,
                                                     const float* __restrict__ cst, float rel, int K,
                                                     long long per_block, uint32_t t, uint64_t seed,
                                                     const int* __restrict__ flagged, int* __restrict__ z,
                                                     int* __restrict__ hist, int* __restrict__ tot,
                                                     int* __restrict__ cand) {
  const long long nf = *n_flagged;
  if (nf > cap) return;
  const int lane = threadIdx.x & 63;
  for (long long base = (long long)blockIdx.x * 256 + (threadIdx.x & ~63); base < nf;
       base += (long long)gridDim.x * 256) {
    const long long r = base + lane;
    const bool valid = r < nf;
    Cands m;
    m.init();
    if (valid) {
      const float* o = cst + (size_t)r * ng * CAND_STATE;
      for (int g = 0; g < ng; ++g) {
        m.lo_max = fmaxf(m.lo_max, o[g * CAND_STATE + 3 * NCAND]);
        m.ev_max = fmaxf(m.ev_max, o[g * CAND_STATE + 3 * NCAND + 1]);
      }
      for (int g = 0; g < ng; ++g)
#pragma unroll
        for (int j = 0; j < NCAND; ++j) {
          const int kk = __float_as_int(o[g * CAND_STATE + 2 * NCAND + j]);
          if (kk >= 0) m.push_u(o[g * CAND_STATE + j], o[g * CAND_STATE + NCAND + j], kk);
        }
    }
    finish_cands(valid, r, valid ? (long long)flagged[r] : 0, m, rel, K, per_block, t, seed, z, hist, tot, cand);
  }
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
                                                                const bf16x8* __restrict__ wlo, int K, uint32_t t,
                                                                uint64_t seed, int* __restrict__ z, int* __restrict__ hist,
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
      finish_cands(r < end, r, r < end ? (long long)flagged[r] : 0, cd, REL, K, per_block, t, seed, z, hist, tot,
                   cand);
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

typedef __attribute__((address_space(3))) void lds_void;

// The 32 x 16 tiles of a lower-triangular D x D whitener that are not all
// zero: row block mt (rows 32 mt ... 32 mt + 31) needs ks <= 2 mt + 1.
template <int D>
struct TriTiles {
  static constexpr int MT = D / 32, KS = D / 16;
  static constexpr int tiles(int m) { return 2 * m + 2 < KS ? 2 * m + 2 : KS; }
  static constexpr int off(int m) { return m == 0 ? 0 : off(m - 1) + tiles(m - 1); }
  static constexpr int NT = off(MT);
};

constexpr int BLOCK_W32 = 512;  // threads of k_label_gauss_mfma_w32: 8 waves of 32 points

// d = 64, 128 in bf16x3, and the candidate pass of either form (the BF16
// main pass is k_label_gauss_mfma_uc below): a cluster's non-zero whitener
// tiles (only those on or below
// the diagonal), its mean and its constant are copied from global memory
// straight into LDS (global_load_lds, no registers) into one of two
// statically allocated buffers, while the workgroup scores its points against
// the previous clusters from the other (in BF16 four clusters per buffer and
// barrier at d = 64, two at d = 128; one in bf16x3, whose tables are twice as
// large); the matrix cores
// execute 1.25 d^2 instead of 2 d^2 flops per point-cluster at d = 128.  A
// wave scores a single 32-point tile: lanes l and l + 32 hold the two halves
// of the K slice of point l % 32, so a lane keeps d / 2 FP32 coordinates and
// one 16-register accumulator.  Two waves then share a SIMD and one wave's
// centring and squared norms on the vector ALUs overlap the other's
// matrix-core tiles.  A workgroup step covers 256 points, as for the other
// label kernels (the per-workgroup histogram blocks are the same).  Points
// whose top-2 gap leaves any doubt are appended to `flagged` (z = -1, not in
// the histogram) for the candidate pass and k_rescore_flagged.
template <int D, bool X3, bool CANDS>
__global__ __launch_bounds__(BLOCK_W32) void k_label_gauss_mfma_w32(const float* __restrict__ x, long long n,
                                                                   long long per_block, const float* __restrict__ packed,
                                                                   const bf16x8* __restrict__ whi,
                                                                   const bf16x8* __restrict__ wlo, int K, uint32_t t,
                                                                   uint64_t seed, int* __restrict__ z,
                                                                   int* __restrict__ hist, int* __restrict__ tot,
                                                                   int* __restrict__ flagged, int* __restrict__ cand,
                                                                   int* __restrict__ n_flagged, int ng, int cap,
                                                                   float* __restrict__ cst) {
  using TT = TriTiles<D>;
  constexpr int S = (4 + D + D * (D + 1) / 2 + 3) & ~3;
  constexpr int MT = TT::MT, KS = TT::KS, NF = MT * KS * 64;  // fragments per cluster in global memory
  constexpr int NFZ = TT::NT * 64;                              // fragments per cluster staged (non-zero tiles)
  constexpr int NJ = (NFZ + BLOCK_W32 - 1) / BLOCK_W32;
  constexpr float REL = X3 ? BF16X3_TOL_REL : BF16_TOL_REL;
  constexpr int NB = X3 ? 2 : 1;  // fragment tables per cluster (hi, lo)
  constexpr int MUS = D + 4;      // mu[D], c
  constexpr int CHUNK = BLOCK_W32 / 2;
  constexpr int CPB = X3 ? 1 : (D == 64 ? 4 : 2);  // clusters per staging buffer (per barrier)
  static_assert(D < BLOCK_W32 && CHUNK == BLOCK && NFZ % 64 == 0, "staging layout, histogram blocks");
  __shared__ __align__(16) bf16x8 s_w0[CPB * NB * NFZ], s_w1[CPB * NB * NFZ];
  __shared__ __align__(16) float s_mu0[CPB * MUS], s_mu1[CPB * MUS];
  extern __shared__ int h[];  // K counters
  for (int k = threadIdx.x; k < K; k += BLOCK_W32) h[k] = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int wbase = threadIdx.x & ~63;
  // main pass: the workgroup's points; candidate pass: the deferred slots, grid-strided
  const long long nf = CANDS ? (long long)*n_flagged : 0;
  // candidate pass, split form (ng > 1): workgroup (chunk, g) scores clusters
  // [g kg, (g + 1) kg) of its points and stores their lists; it runs only while at
  // most cap points are deferred, and the single form only beyond that
  if (CANDS && (ng > 1 ? nf > cap : (cap > 0 && nf <= cap))) return;
  const int grp = CANDS ? (int)blockIdx.y : 0;
  const int kg = (K + ng - 1) / ng;
  const int kb0 = grp * kg < K ? grp * kg : K;
  const int kb1 = kb0 + kg < K ? kb0 + kg : K;
  const long long begin = CANDS ? (long long)blockIdx.x * CHUNK : (long long)blockIdx.x * per_block;
  const long long end = CANDS ? nf : (begin + per_block < n ? begin + per_block : n);
  const long long step = CANDS ? (long long)gridDim.x * CHUNK : CHUNK;
  // copies of clusters k0 ... k0 + nk - 1 into slots 0 ... nk - 1 of (dw, dmu): fragment
  // f of a slot's table is tile f / 64 in (row block, ks) order, lane f % 64; each wave
  // fills 64 consecutive entries
  auto stage = [&](bf16x8* dws, float* dmus, int k0, int nk) {
#pragma unroll
    for (int c = 0; c < CPB; ++c) {
      if (c >= nk) break;
      const int k = k0 + c;
      bf16x8* dw = dws + c * NB * NFZ;
      float* dmu = dmus + c * MUS;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int f = j * BLOCK_W32 + threadIdx.x;
        if (f < NFZ) {
          const int tt = f >> 6;
          int mt = 0, o = 0;
#pragma unroll
          for (int m = 1; m < MT; ++m)
            if (tt >= TT::off(m)) mt = m, o = TT::off(m);
          const size_t g = (size_t)k * NF + (size_t)(mt * KS + tt - o) * 64 + (f & 63);
          __builtin_amdgcn_global_load_lds((const void*)(whi + g), (lds_void*)(dw + j * BLOCK_W32 + wbase), 16, 0, 0);
          if (X3)
            __builtin_amdgcn_global_load_lds((const void*)(wlo + g), (lds_void*)(dw + NFZ + j * BLOCK_W32 + wbase), 16,
                                             0, 0);
        }
      }
      if (threadIdx.x <= D) {
        const float* rec = packed + (size_t)k * S;
        __builtin_amdgcn_global_load_lds((const void*)(threadIdx.x < D ? rec + 4 + threadIdx.x : rec),
                                         (lds_void*)(dmu + wbase), 4, 0, 0);
      }
    }
  };
  if (begin < end && kb0 < kb1) stage(s_w0, s_mu0, kb0, kb1 - kb0 < CPB ? kb1 - kb0 : CPB);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int buf = 0;
  // every wave runs the same number of chunks and clusters: one barrier per CPB clusters
  for (long long chunk = begin; chunk < end; chunk += step) {
    const long long r = chunk + wave * 32 + col;
    const bool ok = r < end;
    const long long p = ok ? (CANDS ? (long long)flagged[r] : r) : 0;
    // the lane's half of the point's coordinates: 8 per K slice of 16 (a lane
    // past the end reads row 0 and keeps zeros)
    float xv[KS][8];
    const float4* xr = reinterpret_cast<const float4*>(x + p * D) + 2 * half;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const float4 v0 = xr[4 * ks], v1 = xr[4 * ks + 1];
      xv[ks][0] = ok ? v0.x : 0.0f;
      xv[ks][1] = ok ? v0.y : 0.0f;
      xv[ks][2] = ok ? v0.z : 0.0f;
      xv[ks][3] = ok ? v0.w : 0.0f;
      xv[ks][4] = ok ? v1.x : 0.0f;
      xv[ks][5] = ok ? v1.y : 0.0f;
      xv[ks][6] = ok ? v1.z : 0.0f;
      xv[ks][7] = ok ? v1.w : 0.0f;
    }
    const bool more = chunk + step < end;
    Top2U t2;
    Cands cd;
    if (CANDS)
      cd.init();
    else
      t2.init();
    // score cluster k from (cw, cmu)
    auto score = [&](const bf16x8* cw, const float* cmu, int k) {
      float q0 = 0.0f, q1 = 0.0f;
      const bf16x8* cwl = cw + (NB - 1) * NFZ;
      bf16x8 b[KS], bl[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float dv = xv[ks][q] - cmu[16 * ks + 8 * half + q];
          b[ks][q] = (__bf16)dv;
          if (X3) bl[ks][q] = (__bf16)(dv - (float)b[ks][q]);
        }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        f32x16 acc = {0};
#pragma unroll
        for (int ks = 0; ks < TT::tiles(mt); ++ks) {
          const int tile = TT::off(mt) + ks;
          const bf16x8 a = cw[tile * 64 + lane];
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[ks], acc, 0, 0, 0);
          if (X3) {
            const bf16x8 al = cwl[tile * 64 + lane];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b[ks], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bl[ks], acc, 0, 0, 0);
          }
        }
#pragma unroll
        for (int e = 0; e < 16; e += 2) {
          q0 = fmaf(acc[e], acc[e], q0);
          q1 = fmaf(acc[e + 1], acc[e + 1], q1);
        }
      }
      // lane l holds rows 4 (l / 32) + ... of every 8: the other half has the rest
      float qm = q0 + q1;
      qm += __shfl_xor(qm, 32);
      const float l = fmaf(-0.5f, qm, cmu[D]);
      if (CANDS)
        cd.push(l, qm, REL, k);
      else
        t2.push(l, qm, REL, k);
    };
    // score clusters k0 ... k0 + nk - 1 from (cw, cmu) while the next group (kn, nkn)
    // is copied into (nw, nmu)
    auto group = [&](const bf16x8* cw, const float* cmu, bf16x8* nw, float* nmu, int k0, int nk, bool next, int kn,
                     int nkn) {
      if (next) stage(nw, nmu, kn, nkn);
#pragma unroll
      for (int c = 0; c < CPB; ++c)
        if (c < nk) score(cw + c * NB * NFZ, cmu + c * MUS, k0 + c);
      // this wave's copies into the other buffer have landed; after the barrier all have
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    };
    for (int k = kb0; k < kb1; k += CPB) {
      const int nk = kb1 - k < CPB ? kb1 - k : CPB;
      const bool last = k + CPB >= kb1;
      const bool next = !last || more;
      const int kn = last ? kb0 : k + CPB;
      const int nkn = last ? (kb1 - kb0 < CPB ? kb1 - kb0 : CPB) : (kb1 - kn < CPB ? kb1 - kn : CPB);
      if (buf == 0)
        group(s_w0, s_mu0, s_w1, s_mu1, k, nk, next, kn, nkn);
      else
        group(s_w1, s_mu1, s_w0, s_mu0, k, nk, next, kn, nkn);
      buf ^= 1;
    }
    // lanes 0-31 own the points (lanes 32-63 hold the same state)
    if (CANDS && ng > 1) {
      if (ok && half == 0) {  // this group's list of point r (r < nf <= cap)
        float* o = cst + ((size_t)r * ng + grp) * CAND_STATE;
#pragma unroll
        for (int j = 0; j < NCAND; ++j) {
          o[j] = cd.u[j];
          o[NCAND + j] = cd.q[j];
          o[2 * NCAND + j] = __int_as_float(cd.k[j]);
        }
        o[3 * NCAND] = cd.lo_max;
        o[3 * NCAND + 1] = cd.ev_max;
      }
    } else if (CANDS) {
      finish_cands(ok && half == 0, r, p, cd, REL, K, per_block, t, seed, z, hist, tot, cand);
    } else {
      finish_main(ok && half == 0, r, t2, z, h, flagged, n_flagged, lane);
    }
  }
  if (CANDS) return;
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += BLOCK_W32) {
    hist[(size_t)blockIdx.x * K + k] = h[k];
    if (h[k]) atomicAdd(&tot[k], h[k]);
  }
}


// Two partial top-2 states over disjoint cluster sets combined: the same state
// as one sequential pass over both (maximum bounds, the smallest cluster index
// among equal maxima, the second largest bound of the union).
__device__ __forceinline__ void top2_merge(Top2U& a, float u1, float u2, float lo, int k1) {
  const bool take = u1 > a.u1 || (u1 == a.u1 && k1 < a.k1);
  const float s2 = fmaxf(fminf(a.u1, u1), fmaxf(a.u2, u2));
  a.k1 = take ? k1 : a.k1;
  a.u1 = fmaxf(a.u1, u1);
  a.u2 = s2;
  a.lo_max = fmaxf(a.lo_max, lo);
}


// Bounds on the score of the uncentred form below.  l = c_k - q / 2 is the
// score of the FP32 record (W, mu, c_k), q = ||y||^2, y = W (x - mu).  With
// x' = x - c (c a centre common to all clusters) and beta = -W (mu - c),
// y = W x' + beta; the matrix cores form Y = bf16(W) bf16(x') + beta with exact
// products and FP32 sums.  Each rounding to BF16 is within 2^-8 relative, so
//   |Y_j - y_j| <= g sum_i |W_ji| |x'_i| + g2 sum_i |W_ji| (|x'_i| + |mu_i - c_i|)
// with g = 2^-7 (plus a margin) for the two BF16 roundings and g2 = 2^-14 for
// the FP32 sums and roundings of both this form and the FP32 draw it stands
// for ((3d + 5) 2^-24 at most, d <= 128).  By Cauchy-Schwarz
//   E = ||Y - y|| <= (g + g2) ||W||_F ||x'|| + g2 ||W||_F ||mu - c||.
// The computed s = sqrt(q_bf16) is within 2^-16 s of ||Y||, so with
// E' = E + 2^-16 s the exact q lies in [max(0, s - E')^2, (s + E')^2]: the
// score lies in [c_k - (s + E')^2 / 2, c_k - max(0, s - E')^2 / 2].
constexpr int UC_BUF_DWORD3 = 0x00020000;  // raw buffer descriptor word 3 (gfx9 family)
constexpr int UC_NT = 2;                    // cache policy of the row loads: non-temporal
constexpr float UC_GAMMA = 1.02f / 128.0f;
constexpr float UC_GAMMA2 = 1.0f / 16384.0f;
constexpr float UC_EPSS = 1.0f / 65536.0f;

// Main pass for d = 64, 128 in BF16, cluster-stationary and uncentred: the
// workgroup's NWAVE waves (eight, or four with two workgroups per CU) take PTS
// rows per step (512 with eight waves while they and the counters fit in LDS,
// else 256), centred once per step on the common centre c,
// rounded to BF16 and stored in LDS (rows padded by 16 bytes, so that the
// sixteen-byte reads of 32 rows fall on distinct banks), with each row's norm
// ||x'||.  Each wave takes every NWAVE-th cluster and holds its
// whitener fragments (non-zero tiles only) and its offset beta = -W (mu - c),
// in the accumulator layout, in registers while it sweeps the step's 32-point
// tiles: a row block's accumulators start at beta (the matrix cores add it),
// so a tile costs its MFMAs, its B operands read from LDS and the squared
// norms, and none of the per-cluster centring and rounding of the rows.  Each
// score comes with its own interval (above) in place of the allowance of the
// centred kernels: a point is drawn here only if a single cluster can win the
// FP32 draw, so the labels are those of the FP32 draw.
// The partial top-2 states of the waves are merged through LDS at the end of
// the step (top2_merge).
template <int D, int PTS, int NWAVE>
__global__ __launch_bounds__(64 * NWAVE, 8 / NWAVE) void k_label_gauss_mfma_uc(const float* __restrict__ x, long long n,
                                                                     long long per_block,
                                                                     const bf16x8* __restrict__ whi,
                                                                     const float* __restrict__ wbias, int K, int k_max,
                                                                     int* __restrict__ z, int* __restrict__ hist,
                                                                     int* __restrict__ tot, int* __restrict__ flagged,
                                                                     int* __restrict__ n_flagged) {
  using TT = TriTiles<D>;
  constexpr int MT = TT::MT, KS = TT::KS, NF = MT * KS * 64, NT = TT::NT;
  constexpr int RB = D / 8 + 1;  // LDS row stride in 16-byte units
  constexpr int TILES = PTS / 32;
  constexpr int UC_T2 = TILES / 2;  // first tile read from the second base
  constexpr int NW = NWAVE, BLK = 64 * NWAVE;
  constexpr int P4 = D / 4;       // float4 pieces of a row
  constexpr int RPI = 64 / P4;    // rows per wave and staging pass
  constexpr int WROWS = PTS / NW;  // rows staged per wave
  constexpr int ITER = WROWS / RPI;  // staging passes for the wave's rows
  static_assert(D % 64 == 0 && PTS % (32 * NW) == 0 && PTS <= BLK, "step, row copies");
  static_assert(NW * PTS * 4 * sizeof(float) <= PTS * RB * 16, "partial states alias the rows");
  typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
  extern __shared__ __align__(16) unsigned char smem[];
  bf16x8* xb = reinterpret_cast<bf16x8*>(smem);                 // [PTS][RB] centred BF16 rows
  float* rxs = reinterpret_cast<float*>(smem + PTS * RB * 16);  // [PTS] ||x'||
  int* h = reinterpret_cast<int*>(rxs + PTS);                  // [K] counters
  const float4* cst = reinterpret_cast<const float4*>(wbias + (size_t)k_max * D);  // (c_k, (g + g2) ||W||_F, g2 ||W||_F ||mu - c||, 0)
  const float* centre = wbias + (size_t)k_max * (D + 4);
  for (int k = threadIdx.x; k < K; k += BLK) h[k] = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int sub = lane / P4, part = lane % P4;
  const long long begin = (long long)blockIdx.x * per_block;
  const long long end = begin + per_block < n ? begin + per_block : n;
  for (long long chunk = begin; chunk < end; chunk += PTS) {
    const int rows = end - chunk < PTS ? (int)(end - chunk) : PTS;
    // the lane's slice of the centre, read again each step (an L2 hit) rather
    // than held in registers across the cluster loop
    const float* cp = centre + 4 * part;
    asm volatile("" : "+v"(cp));
    const float4 c4 = *reinterpret_cast<const float4*>(cp);
    __syncthreads();  // the previous step's merge is done with the rows' space
    // the wave's rows: x' = x - c rounded to BF16, and ||x'|| (rows past the end
    // are zero), sixteen loads in flight per batch
    {
      // the rows are read once: non-temporal loads, so that they do not evict
      // the whitener tables from L2
      typedef float f32x4 __attribute__((ext_vector_type(4)));
      constexpr int SB = ITER < 16 ? ITER : 16;
      static_assert(ITER % SB == 0, "staging batches");
      // one buffer descriptor per step over its rows (loads past them return
      // zero), one lane offset and a constant offset per row: no 64-bit
      // address per load to keep live
      const __amdgpu_buffer_rsrc_t rx =
          __builtin_amdgcn_make_buffer_rsrc((void*)(x + chunk * D), (short)0, rows * D * 4, UC_BUF_DWORD3);
      const int vo = ((wave * WROWS + sub) * D + 4 * part) * 4;
#pragma unroll
      for (int i0 = 0; i0 < ITER; i0 += SB) {
        float4 v[SB];
#pragma unroll
        for (int j = 0; j < SB; ++j) {
          const int r = wave * WROWS + (i0 + j) * RPI + sub;
          const f32x4 u = __builtin_amdgcn_raw_buffer_load_b128(rx, vo, (i0 + j) * RPI * D * 4, UC_NT);
          v[j] = r < rows ? make_float4(u.x, u.y, u.z, u.w) : c4;
        }
        float ss[SB];
#pragma unroll
        for (int j = 0; j < SB; ++j) {
          const int r = wave * WROWS + (i0 + j) * RPI + sub;
          const float d0 = v[j].x - c4.x, d1 = v[j].y - c4.y, d2 = v[j].z - c4.z, d3 = v[j].w - c4.w;
          ss[j] = fmaf(d3, d3, fmaf(d2, d2, fmaf(d1, d1, d0 * d0)));
          bf16x4 b4;
          b4[0] = (__bf16)d0;
          b4[1] = (__bf16)d1;
          b4[2] = (__bf16)d2;
          b4[3] = (__bf16)d3;
          reinterpret_cast<bf16x4*>(xb + r * RB)[part] = b4;
        }
#pragma unroll
        for (int o = P4 / 2; o > 0; o >>= 1)
#pragma unroll
          for (int j = 0; j < SB; ++j) ss[j] += __shfl_xor(ss[j], o);
        if (part == 0)
#pragma unroll
          for (int j = 0; j < SB; ++j) rxs[wave * WROWS + (i0 + j) * RPI + sub] = __builtin_amdgcn_sqrtf(ss[j]);
      }
    }
    __syncthreads();

    Top2U st[TILES / 2];
#pragma unroll
    for (int j = 0; j < TILES / 2; ++j) st[j].init();
    typedef __attribute__((address_space(3))) const bf16x8 lds_bf16x8;
    lds_bf16x8* xr_lo = (lds_bf16x8*)(xb + col * RB + half);
    for (int k = wave; k < K; k += NW) {
      const int ku = __builtin_amdgcn_readfirstlane(k);
      bf16x8 a[NT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ks = 0; ks < TT::tiles(mt); ++ks)
          a[TT::off(mt) + ks] = whi[(size_t)ku * NF + (size_t)(mt * KS + ks) * 64 + lane];
      // beta in the accumulator layout: element r of row block mt is output row
      // 32 mt + 8 (r / 4) + 4 half + r % 4
      f32x16 bs[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const float4* bp = reinterpret_cast<const float4*>(wbias + ((size_t)ku * MT + mt) * 32 + half * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 u = bp[q];
          bs[mt][4 * q] = u.x;
          bs[mt][4 * q + 1] = u.y;
          bs[mt][4 * q + 2] = u.z;
          bs[mt][4 * q + 3] = u.w;
        }
      }
      const float4 kc = cst[ku];
      float qa;  // the lane's half of the squared norms of the even tile of a pair
      // a second base for the second half of the tiles, opaque to the compiler,
      // so that every B-operand read takes its offset as an immediate (at most
      // 16 bits) instead of an address add of its own
      lds_bf16x8* xr_hi;
#pragma unroll
      for (int t = 0; t < TILES; ++t) {
        if (t == UC_T2) {
          xr_hi = xr_lo + UC_T2 * 32 * RB;
          asm volatile("" : "+v"(xr_hi));
        }
        lds_bf16x8* xr = (t < UC_T2 ? xr_lo + t * 32 * RB : xr_hi + (t - UC_T2) * 32 * RB);
        bf16x8 b[KS];
        float q0 = 0.0f, q1 = 0.0f, q2 = 0.0f, q3 = 0.0f;
        f32x16 acc;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
          for (int ks = (mt == 0 ? 0 : TT::tiles(mt - 1)); ks < TT::tiles(mt); ++ks) b[ks] = xr[2 * ks];
          if (mt > 0) {
#pragma unroll
            for (int e = 0; e < 16; e += 4) {
              q0 = fmaf(acc[e], acc[e], q0);
              q1 = fmaf(acc[e + 1], acc[e + 1], q1);
              q2 = fmaf(acc[e + 2], acc[e + 2], q2);
              q3 = fmaf(acc[e + 3], acc[e + 3], q3);
            }
          }
          acc = bs[mt];
#pragma unroll
          for (int ks = 0; ks < TT::tiles(mt); ++ks)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[TT::off(mt) + ks], b[ks], acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 16; e += 4) {
          q0 = fmaf(acc[e], acc[e], q0);
          q1 = fmaf(acc[e + 1], acc[e + 1], q1);
          q2 = fmaf(acc[e + 2], acc[e + 2], q2);
          q3 = fmaf(acc[e + 3], acc[e + 3], q3);
        }
        // the lane's half of the squared norm of point t * 32 + col
        const float qh = (q0 + q1) + (q2 + q3);
        if ((t & 1) == 0) {
          qa = qh;
        } else {
          // tiles t - 1 and t together: one swap of the upper half of the first
          // tile's partial sums with the lower half of the second's leaves the
          // full norm of tile t - 1 in lanes 0-31 and of tile t in lanes 32-63,
          // so each half takes the bounds of its own tile's points only
          const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(qa), __float_as_uint(qh), false, false);
          const float qm = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
          const float sq = __builtin_amdgcn_sqrtf(qm);
          const float e = fmaf(UC_EPSS, sq, fmaf(kc.y, rxs[(t - 1) * 32 + lane], kc.z));
          const float sp = sq + e, sm = sq - e;
          const float lo = fmaf(-0.5f * sp, sp, kc.x);
          const float up = sm > 0.0f ? fmaf(-0.5f * sm, sm, kc.x) : kc.x;
          st[t >> 1].push_bounds(lo, up, k);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    __syncthreads();  // every wave is done with the rows
    float* ps = reinterpret_cast<float*>(smem);  // partial states [wave][point]: u1, u2, lo_max, k1
#pragma unroll
    for (int j = 0; j < TILES / 2; ++j) {
      const int p = (2 * j + half) * 32 + col;
      float* o = ps + ((size_t)wave * PTS + p) * 4;
      o[0] = st[j].u1;
      o[1] = st[j].u2;
      o[2] = st[j].lo_max;
      o[3] = __int_as_float(st[j].k1);
    }
    __syncthreads();
    if (threadIdx.x < PTS) {
      Top2U m;
      m.init();
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const float* o = ps + ((size_t)w * PTS + threadIdx.x) * 4;
        top2_merge(m, o[0], o[1], o[2], __float_as_int(o[3]));
      }
      finish_main(threadIdx.x < rows, chunk + threadIdx.x, m, z, h, flagged, n_flagged, lane);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += BLK) {
    hist[(size_t)blockIdx.x * K + k] = h[k];
    if (h[k]) atomicAdd(&tot[k], h[k]);
  }
}

size_t label_uc_lds(int d, int K, int pts) {
  return (size_t)pts * (d / 8 + 1) * 16 + (size_t)pts * sizeof(float) + (size_t)K * sizeof(int);
}

constexpr int RS_BLOCK = 256;

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

// FP32 draw of the deferred points, exactly the FP32 kernel's draw: the
// winner of max_k (l_k + g_k) with the smaller k on ties, here as a streaming
// lazy Gumbel-max over the point's candidates in increasing k (or over all K
// when its list is incomplete).  Each candidate k that is not already beaten
// by more than the Gumbel range gets its Gumbel value, so the result equals
// the full draw.  A wave takes 64 deferred points and walks the union of their
// cluster sequences in increasing k: at each step every lane scores the same
// cluster (the record comes through scalar loads) and the lanes whose next
// cluster it is use the score.  Adds each drawn point to the histogram of the
// label-kernel block that owns it.
template <int D>
__global__ __launch_bounds__(RS_BLOCK) void k_rescore_flagged(const float* __restrict__ x,
                                                              const int* __restrict__ flagged,
                                                              const int* __restrict__ cand,
                                                              const int* __restrict__ n_flagged, long long per_block,
                                                              const float* __restrict__ packed, int K, uint32_t t,
                                                              uint64_t seed, int* __restrict__ z,
                                                              int* __restrict__ hist, int* __restrict__ tot) {
  constexpr int S = (4 + D + D * (D + 1) / 2 + 3) & ~3;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nf = *n_flagged;
  for (int base = (blockIdx.x * (RS_BLOCK / 64) + wave) * 64; base < nf; base += gridDim.x * RS_BLOCK) {
    const int q = base + lane;
    const bool valid = q < nf;
    const long long p = valid ? flagged[q] : 0;
    // the row is re-read (from cache) for every cluster: only the centred copy stays in registers
    const float4* xr = reinterpret_cast<const float4*>(x + p * D);
    int ids[NCAND];
#pragma unroll
    for (int j = 0; j < NCAND; ++j) ids[j] = valid ? cand[(size_t)q * NCAND + j] : -1;
    const bool done = valid && ids[0] == -3;  // drawn by the candidate pass
    const bool all = valid && ids[0] == -2;
    // candidates in increasing k, empty slots (-1) last
#pragma unroll
    for (int a = 0; a < NCAND; ++a)
#pragma unroll
      for (int b = 0; b + 1 < NCAND - a; ++b) {
        const unsigned ka = (unsigned)ids[b], kb = (unsigned)ids[b + 1];
        ids[b] = ka < kb ? (int)ka : (int)kb;
        ids[b + 1] = ka < kb ? (int)kb : (int)ka;
      }
    if (done) ids[0] = -1;
    int pos = 0;                  // next candidate slot (list lanes)
    int nxt_all = all ? 0 : K;    // next cluster (all-K lanes)
    float best = -INFINITY;
    int win = -1, cached = -1;
    u32x4 blk = {0u, 0u, 0u, 0u};
    for (;;) {
      int mine_k = INT_MAX;
      if (all) {
        mine_k = nxt_all < K ? nxt_all : INT_MAX;
      } else if (valid) {
#pragma unroll
        for (int j = 0; j < NCAND; ++j)
          if (j == pos && ids[j] >= 0) mine_k = ids[j];
      }
      // uniform by construction; readfirstlane lets the compiler see it (scalar record loads)
      const int kk = __builtin_amdgcn_readfirstlane(wave_min_i(mine_k));
      if (kk == INT_MAX) break;
      float l;
      {
        const float* rec = packed + (size_t)kk * S;
        float dx[D];
#pragma unroll
        for (int j = 0; j < D / 4; ++j) {
          const float4 v = xr[j];
          dx[4 * j] = v.x - rec[4 + 4 * j];
          dx[4 * j + 1] = v.y - rec[5 + 4 * j];
          dx[4 * j + 2] = v.z - rec[6 + 4 * j];
          dx[4 * j + 3] = v.w - rec[7 + 4 * j];
        }
        const float* w = rec + 4 + D;
        float qq = 0.0f;
#pragma unroll
        for (int r = 0; r < D; ++r) {
          float y = 0.0f;
#pragma unroll
          for (int c = 0; c <= r; ++c) y = fmaf(w[r * (r + 1) / 2 + c], dx[c], y);
          qq = fmaf(y, y, qq);
        }
        l = fmaf(-0.5f, qq, rec[0]);
      }
      if (mine_k == kk) {
        if (l + GUMBEL_MAX_F > best) {
          const int b = kk >> 2;
          if (b != cached) {
            blk = rng_block(seed, t, (uint32_t)p, TAG_GUMBEL, (uint32_t)b);
            cached = b;
          }
          const float sv = l + gumbel_f(word_of(blk, kk & 3));
          if (sv > best) {
            best = sv;
            win = kk;
          }
        }
        if (all)
          ++nxt_all;
        else
          ++pos;
      }
    }
    const bool drew = valid && !done;
    if (drew) z[p] = win;
    wave_count_add(drew, drew ? (p / per_block) * K + win : 0, hist);
    wave_count_add(drew, drew ? win : 0, tot);
  }
}

// Fragment table of record rec0 + k's whitener: element (mt, ks, lane, q) =
// W[32 mt + lane % 32][16 ks + 8 (lane / 32) + q] (zero above the diagonal).
__global__ void k_pack_wfrag(int K, int d, int rec0, const float* __restrict__ packed, __bf16* __restrict__ whi,
                             __bf16* __restrict__ wlo) {
  const int k = blockIdx.x;
  if (k >= K) return;
  const int S = gauss_rec_stride(d);
  const float* w = packed + (size_t)(rec0 + k) * S + 4 + d;
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

// Sub-label draw of cluster-sorted rows in bf16x3 on the BF16 matrix cores
// (d = 64, 128), Sec. 4.1 step (f), in front of the FP32 kernel
// k_sub_labels_mfma: the same scores (rows centred on sub-cluster 0's mean,
// sub-cluster 1's accumulators started at W_1 (mu_0 - mu_1)) from the hi/lo
// BF16 parts of W_h and of the centred rows, three products each (W_hi x_hi +
// W_hi x_lo + W_lo x_hi), for about 16 mantissa bits at a sixteenth of the FP32
// matrix cores' time.  The score difference delta = l_0 - l_1 then carries the
// allowance rel (q_0 + q_1) + TOL_ABS of the bf16x3 form against the FP32 one;
// a row is drawn here when the logistic draw gives the same sub-label at both
// ends of that interval (the draw is monotone in delta), else it is flagged for
// the FP32 kernel, which draws it as it draws every row in the FP32 form.
// A workgroup of eight waves walks a contiguous range of sorted rows; the
// hi/lo fragments of the current cluster's two sub-clusters (non-zero tiles)
// are staged in LDS whenever the cluster changes; a wave scores 64 rows (two
// 32-row tiles that share each fragment read), a lane holding the hi and lo
// BF16 parts of half the coordinates of one row of each tile.
constexpr int SUBX_BLOCK = 512;

__device__ __forceinline__ int logistic_pick(float delta, float u) {
  if (delta > LOGISTIC_MAX_F) return 0;
  if (delta < -LOGISTIC_MAX_F) return 1;
  return u > 1.0f / (1.0f + expf(delta)) ? 0 : 1;
}

template <int D>
__global__ __launch_bounds__(SUBX_BLOCK, 1) void k_sub_labels_x3(
    const float* __restrict__ x, long long n_sorted, long long per_block, const int* __restrict__ perm,
    const int* __restrict__ z, const int* __restrict__ zrow, unsigned char* __restrict__ zsub,
    const float* __restrict__ packed, const bf16x8* __restrict__ shi, const bf16x8* __restrict__ slo, int K,
    int k_max, uint32_t t, uint64_t seed, unsigned char* __restrict__ flag, int* __restrict__ cnt) {
  using TT = TriTiles<D>;
  constexpr int S = (4 + D + D * (D + 1) / 2 + 3) & ~3;
  constexpr int MT = TT::MT, KS = TT::KS, NF = MT * KS * 64, NT = TT::NT;
  constexpr int NFZ = NT * 64;  // staged fragments per sub-cluster and part
  extern __shared__ __align__(16) unsigned char smem[];
  bf16x8* s_fr = reinterpret_cast<bf16x8*>(smem);  // [sub][hi, lo][NFZ]
  float* s_mu0 = reinterpret_cast<float*>(s_fr + 4 * NFZ);
  float* s_dmu = s_mu0 + D;
  float* s_corr = s_dmu + D;  // W_1 (mu_0 - mu_1)
  float* s_c = s_corr + D;    // c_0, c_1
  int* s_cnt = reinterpret_cast<int*>(s_c + 4);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, col = lane & 31;
  if (threadIdx.x == 0) *s_cnt = 0;
  const long long begin = (long long)blockIdx.x * per_block;
  const long long end = begin + per_block < n_sorted ? begin + per_block : n_sorted;
  auto kof = [&](long long g) { return __builtin_amdgcn_readfirstlane(zrow ? zrow[g] : z[perm[g]]); };
  int staged = -1, nflag = 0;
  for (long long chunk = begin; chunk < end; chunk += SUBX_BLOCK) {
    const long long cend = chunk + SUBX_BLOCK < end ? chunk + SUBX_BLOCK : end;
    const long long base = chunk + wave * 64;
    const long long rA = base + col, rB = base + 32 + col;
    const bool vA = rA < cend, vB = rB < cend;
    const long long iA = vA ? perm[rA] : 0, iB = vB ? perm[rB] : 0;
    const int kA = vA ? (zrow ? zrow[rA] : z[iA]) : -1, kB = vB ? (zrow ? zrow[rB] : z[iB]) : -1;
    const int kmine = h ? kB : kA;
    float delta = 0.0f, allow = 0.0f;
    int cur = kof(chunk);
    const int last = kof(cend - 1);
    for (;;) {
      if (cur != staged) {
        __syncthreads();  // every wave is done with the previous tables
        for (int f = threadIdx.x; f < 4 * NFZ; f += SUBX_BLOCK) {
          const int part = f / NFZ, g = f - part * NFZ;  // part = 2 sub + (lo)
          const int tt = g >> 6;
          int mt = 0, o = 0;
#pragma unroll
          for (int m = 1; m < MT; ++m)
            if (tt >= TT::off(m)) mt = m, o = TT::off(m);
          const size_t src = (size_t)(2 * cur + (part >> 1)) * NF + (size_t)(mt * KS + tt - o) * 64 + (g & 63);
          s_fr[f] = (part & 1) ? slo[src] : shi[src];
        }
        const float* r0 = packed + (size_t)(k_max + 2 * cur) * S;
        const float* r1 = r0 + S;
        if (threadIdx.x < D) {
          s_mu0[threadIdx.x] = r0[4 + threadIdx.x];
          s_dmu[threadIdx.x] = r0[4 + threadIdx.x] - r1[4 + threadIdx.x];
        }
        if (threadIdx.x == 0) {
          s_c[0] = r0[0];
          s_c[1] = r1[0];
        }
        __syncthreads();
        if (threadIdx.x < D) {
          const int i = threadIdx.x;
          const float* w1 = r1 + 4 + D + i * (i + 1) / 2;
          float c = 0.0f;
          for (int k = 0; k <= i; ++k) c = fmaf(w1[k], s_dmu[k], c);
          s_corr[i] = c;
        }
        __syncthreads();
        staged = cur;
      }
      if (__ballot(kA == cur || kB == cur)) {
        // this lane's half of rows A and B (k = 16 ks + 8 h + q), centred on mu_0, hi and lo parts
        bf16x8 ah[KS], al[KS], bh[KS], bl[KS];
        const float4* pa = reinterpret_cast<const float4*>(x + (size_t)iA * D + 8 * h);
        const float4* pb = reinterpret_cast<const float4*>(x + (size_t)iB * D + 8 * h);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const float4 a0 = vA ? pa[4 * ks] : make_float4(0.f, 0.f, 0.f, 0.f);
          const float4 a1 = vA ? pa[4 * ks + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
          const float4 b0 = vB ? pb[4 * ks] : make_float4(0.f, 0.f, 0.f, 0.f);
          const float4 b1 = vB ? pb[4 * ks + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
          const float va[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
          const float vb[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const float m = s_mu0[16 * ks + 8 * h + q];
            const float da = va[q] - m, db = vb[q] - m;
            ah[ks][q] = (__bf16)da;
            al[ks][q] = (__bf16)(da - (float)ah[ks][q]);
            bh[ks][q] = (__bf16)db;
            bl[ks][q] = (__bf16)(db - (float)bh[ks][q]);
          }
        }
        float sc[2], qq[2];
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
          const bf16x8* fh = s_fr + (2 * sub) * NFZ;
          const bf16x8* fl = fh + NFZ;
          float qa = 0.0f, qb = 0.0f;
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            f32x16 acca, accb;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const float c0 = sub ? s_corr[32 * mt + 8 * (r >> 2) + 4 * h + (r & 3)] : 0.0f;
              acca[r] = c0;
              accb[r] = c0;
            }
#pragma unroll
            for (int ks = 0; ks < TT::tiles(mt); ++ks) {
              const int tile = TT::off(mt) + ks;
              const bf16x8 wh = fh[tile * 64 + lane], wl = fl[tile * 64 + lane];
              acca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, ah[ks], acca, 0, 0, 0);
              accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, bh[ks], accb, 0, 0, 0);
              acca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, al[ks], acca, 0, 0, 0);
              accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, bl[ks], accb, 0, 0, 0);
              acca = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wl, ah[ks], acca, 0, 0, 0);
              accb = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wl, bh[ks], accb, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              qa = fmaf(acca[r], acca[r], qa);
              qb = fmaf(accb[r], accb[r], qb);
            }
          }
          qa += __shfl_xor(qa, 32);
          qb += __shfl_xor(qb, 32);
          qq[sub] = h ? qb : qa;
          sc[sub] = fmaf(-0.5f, qq[sub], s_c[sub]);
        }
        if (kmine == cur) {
          delta = sc[0] - sc[1];
          allow = fmaf(BF16X3_TOL_REL, qq[0] + qq[1], TOL_ABS);
        }
      }
      if (cur == last) break;
      long long lo = chunk, hi = cend - 1;
      while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (kof(mid) > cur)
          hi = mid;
        else
          lo = mid + 1;
      }
      cur = kof(lo);
    }
    const long long rme = base + lane;
    if (rme < cend) {
      const int i = (int)(h ? iB : iA);
      const float u = uniform_f(sub_label_word(seed, t, (uint32_t)i, K));
      const int s0 = logistic_pick(delta - allow, u), s1 = logistic_pick(delta + allow, u);
      if (s0 == s1) zsub[i] = (unsigned char)s0;
      flag[rme] = s0 != s1;
      nflag += s0 != s1;
    }
  }
  // the workgroup's count of flagged rows
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nflag += __shfl_xor(nflag, o);
  if (lane == 0 && nflag) atomicAdd(s_cnt, nflag);
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = *s_cnt;
}

// Exclusive prefix of the G workgroup counts (G <= SUBX_GROUPS): offs[g]; the total in offs[SUBX_GROUPS].
__global__ __launch_bounds__(1024) void k_subx_scan(const int* __restrict__ cnt, int G, int* __restrict__ offs) {
  __shared__ int buf[1024];
  const int tid = threadIdx.x;
  buf[tid] = tid < G ? cnt[tid] : 0;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = tid >= o ? buf[tid - o] : 0;
    __syncthreads();
    buf[tid] += v;
    __syncthreads();
  }
  if (tid < G) offs[tid] = buf[tid] - cnt[tid];
  if (tid == 0) offs[SUBX_GROUPS] = buf[1023];
}

// The flagged rows of workgroup g's range, in sorted order, at offs[g]: their
// point indices and clusters (the FP32 kernel's row list).
__global__ __launch_bounds__(256) void k_subx_scatter(long long n_sorted, long long per_block,
                                                      const unsigned char* __restrict__ flag,
                                                      const int* __restrict__ perm, const int* __restrict__ z,
                                                      const int* __restrict__ zrow, const int* __restrict__ offs,
                                                      int* __restrict__ perm_c, int* __restrict__ zrow_c) {
  __shared__ int wsum[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long begin = (long long)blockIdx.x * per_block;
  const long long end = begin + per_block < n_sorted ? begin + per_block : n_sorted;
  int at = offs[blockIdx.x];
  for (long long c = begin; c < end; c += 256) {
    const long long g = c + threadIdx.x;
    const bool f = g < end && flag[g];
    const unsigned long long m = __ballot(f);
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      before += w < wave ? wsum[w] : 0;
      tot += wsum[w];
    }
    if (f) {
      const int o = at + before + __popcll(m & ((1ull << lane) - 1ull));
      const int p = perm[g];
      perm_c[o] = p;
      zrow_c[o] = zrow ? zrow[g] : z[p];
    }
    at += tot;
    __syncthreads();
  }
}

// The common centre of the uncentred main pass: the mean of the K cluster
// means (any centre keeps the draw exact; one near the data keeps ||x'|| and
// so the error bounds small).
__global__ void k_pack_centre(int K, int d, const float* __restrict__ packed, float* __restrict__ centre) {
  const int S = gauss_rec_stride(d);
  for (int j = threadIdx.x; j < d; j += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += (double)packed[(size_t)k * S + 4 + j];
    centre[j] = (float)(s / K);
  }
}

// Cluster k's offset beta = -W (mu - c) in the accumulator layout of
// k_label_gauss_mfma_uc ([k][row block][lane half][16]) and its constants
// (c_k, (g + g2) ||W||_F, g2 ||W||_F ||mu - c||, 0), rounded up; float64 sums
// of the record's float32 values.  One thread per output row.
template <int D>
__global__ __launch_bounds__(D) void k_pack_bias(int K, int k_max, const float* __restrict__ packed,
                                                 float* __restrict__ wbias) {
  constexpr int S = (4 + D + D * (D + 1) / 2 + 3) & ~3;
  constexpr int MT = D / 32, NWV = D / 64;
  __shared__ double dm[D], red[2][NWV];
  const int k = blockIdx.x, j = threadIdx.x;
  if (k >= K) return;
  const float* rec = packed + (size_t)k * S;
  const float* centre = wbias + (size_t)k_max * (D + 4);
  dm[j] = (double)rec[4 + j] - (double)centre[j];
  __syncthreads();
  const float* w = rec + 4 + D + j * (j + 1) / 2;
  double b = 0.0, wn = 0.0;
  for (int i = 0; i <= j; ++i) {
    const double wji = (double)w[i];
    b = fma(wji, dm[i], b);
    wn = fma(wji, wji, wn);
  }
  const int mt = j >> 5, jj = j & 31;
  const int hh = (jj >> 2) & 1, r = ((jj >> 3) << 2) | (jj & 3);
  wbias[((size_t)k * MT + mt) * 32 + hh * 16 + r] = (float)(-b);
  double m2 = dm[j] * dm[j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    wn += __shfl_xor(wn, o);
    m2 += __shfl_xor(m2, o);
  }
  if ((j & 63) == 0) {
    red[0][j >> 6] = wn;
    red[1][j >> 6] = m2;
  }
  __syncthreads();
  if (j == 0) {
    double wf = 0.0, mm = 0.0;
    for (int v = 0; v < NWV; ++v) {
      wf += red[0][v];
      mm += red[1][v];
    }
    const double f = sqrt(wf) * (1.0 + 1e-6);
    float4 c;
    c.x = rec[0];
    c.y = (float)(((double)UC_GAMMA + (double)UC_GAMMA2) * f);
    c.z = (float)((double)UC_GAMMA2 * f * sqrt(mm) * (1.0 + 1e-6));
    c.w = 0.0f;
    reinterpret_cast<float4*>(wbias + (size_t)k_max * D)[k] = c;
  }
}

}  // namespace

size_t wbias_floats(int d, int k_max) { return (d == 64 || d == 128) ? (size_t)k_max * (d + 4) + d : 0; }

size_t sub_labels_x3_lds(int d) {
  const int nt = d == 128 ? 20 : 6;
  return (size_t)4 * nt * 64 * 16 + (size_t)(3 * d + 4) * sizeof(float) + 16;
}

hipError_t launch_sub_labels_x3(int d, const float* x, long long n, const int* perm, const int* z, const int* zrow,
                                unsigned char* zsub, const float* packed, int K, int k_max, uint32_t t, uint64_t seed,
                                const SubX3& b, hipStream_t s) {
  if (n == 0) return hipSuccess;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_sub_labels_x3<128>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)sub_labels_x3_lds(128));
    if (e != hipSuccess) return e;
    attr = true;
  }
  // one workgroup per CU (eight waves of 64 rows), each on a contiguous range of whole waves' rows
  const long long cap = SUBX_GROUPS;
  long long per = (n + cap - 1) / cap;
  per = ((per + 63) / 64) * 64;
  const unsigned G = (unsigned)((n + per - 1) / per);
  const size_t lds = sub_labels_x3_lds(d);
  const bf16x8* hi = (const bf16x8*)b.hi;
  const bf16x8* lo = (const bf16x8*)b.lo;
  if (d == 128)
    hipLaunchKernelGGL(k_sub_labels_x3<128>, dim3(G), dim3(SUBX_BLOCK), lds, s, x, n, per, perm, z, zrow, zsub, packed,
                       hi, lo, K, k_max, t, seed, b.flag, b.cnt);
  else if (d == 64)
    hipLaunchKernelGGL(k_sub_labels_x3<64>, dim3(G), dim3(SUBX_BLOCK), lds, s, x, n, per, perm, z, zrow, zsub, packed,
                       hi, lo, K, k_max, t, seed, b.flag, b.cnt);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_subx_scan, dim3(1), dim3(1024), 0, s, b.cnt, (int)G, b.offs);
  hipLaunchKernelGGL(k_subx_scatter, dim3(G), dim3(256), 0, s, n, per, b.flag, perm, z, zrow, b.offs, b.perm_c,
                     b.zrow_c);
  return hipGetLastError();
}

bool mfma_supported(int d) { return d == 32 || d == 64 || d == 128; }

hipError_t launch_pack_wfrag(int K, int d, int k_max, const float* packed, void* whi, void* wlo, float* wbias,
                             void* shi, void* slo, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_wfrag, dim3(K), dim3(256), 0, s, K, d, 0, packed, (__bf16*)whi, (__bf16*)wlo);
  // the sub-clusters' records follow the clusters' (slot k_max + 2 k + h)
  if (shi) hipLaunchKernelGGL(k_pack_wfrag, dim3(2 * K), dim3(256), 0, s, 2 * K, d, k_max, packed, (__bf16*)shi, (__bf16*)slo);
  if (wbias && (d == 64 || d == 128)) {
    hipLaunchKernelGGL(k_pack_centre, dim3(1), dim3(128), 0, s, K, d, packed, wbias + (size_t)k_max * (d + 4));
    if (d == 128)
      hipLaunchKernelGGL(k_pack_bias<128>, dim3(K), dim3(128), 0, s, K, k_max, packed, wbias);
    else
      hipLaunchKernelGGL(k_pack_bias<64>, dim3(K), dim3(64), 0, s, K, k_max, packed, wbias);
  }
  return hipGetLastError();
}

hipError_t launch_label_gauss_mfma(int d, bool x3, const float* x, long long n, int G, long long per_block,
                                   const float* packed, const void* whi, const void* wlo, const float* wbias, int K,
                                   int k_max, uint32_t t, uint64_t seed, int* z, int* hist, int* tot, int* flagged,
                                   int* cand, int* n_flagged, hipStream_t s, hipEvent_t ev_main0,
                                   hipEvent_t ev_main1, float* cst) {
  if (n == 0) return hipSuccess;
  hipError_t e = launch_zero64(tot, (size_t)(K + 1) / 2 + 1, s);
  if (e != hipSuccess) return e;
  const size_t lh = (size_t)K * sizeof(int);
  const bf16x8* hi = (const bf16x8*)whi;
  const bf16x8* lo = (const bf16x8*)wlo;
  e = launch_zero64(n_flagged, 1, s);
  if (e != hipSuccess) return e;
  static bool attr_set = false;
  if (!attr_set) {  // d = 32 and the uncentred kernels: more than 64 KB of dynamic LDS (160 KB per CU)
    const void* fns[8] = {(const void*)k_label_gauss_mfma32<true, false>, (const void*)k_label_gauss_mfma32<false, false>,
                          (const void*)k_label_gauss_mfma32<true, true>,
                          (const void*)k_label_gauss_mfma_uc<64, 256, 4>, (const void*)k_label_gauss_mfma_uc<128, 512, 8>,
                          (const void*)k_label_gauss_mfma_uc<64, 512, 8>, (const void*)k_label_gauss_mfma_uc<128, 256, 8>,
                          (const void*)k_label_gauss_mfma_uc<64, 256, 8>};
    for (const void* f : fns) {
      e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      if (e != hipSuccess) return e;
    }
    attr_set = true;
  }
  // the main pass, then the candidate pass over the points it deferred (grid-strided,
  // about 2048 waves: usually it finds none)
  for (int pass = 0; pass < 2; ++pass) {
    const bool cands = pass == 1;
    const int Gp = cands ? (d == 32 ? (G < 256 ? G : 256) : (G < 512 ? G : 512)) : G;
    // optional events taken by the main pass's own dispatch (its start and end
    // time stamps, for timing it alone without extra queue packets)
    hipEvent_t e0 = cands ? nullptr : ev_main0, e1 = cands ? nullptr : ev_main1;
    if ((d == 64 || d == 128) && !cands && !x3 && wbias) {
      // BF16 main pass, uncentred: the rows centred once on the common centre.  At
      // d = 64, two workgroups of four waves per CU (256 rows per step each) while
      // both fit in LDS, so that one copies its rows while the other runs its
      // matrix-core work; at d = 128 (and for larger K at d = 64) one workgroup of
      // eight waves, 512 rows per step while they and the counters fit in LDS
      // (fewer fragment fetches and merges per point), else 256
      const size_t l256 = label_uc_lds(d, K, 256), l512 = label_uc_lds(d, K, 512);
      const bool two = d == 64 && 2 * l256 <= (size_t)160 * 1024;
      const bool big = !two && l512 <= (size_t)160 * 1024;
      const size_t luc = big ? l512 : l256;
#define DPMM_UC(DD, PP, NWV)                                                                                     \
  hipExtLaunchKernelGGL((k_label_gauss_mfma_uc<DD, PP, NWV>), dim3(Gp), dim3(64 * NWV), luc, s, e0, e1, 0, x, n, \
                        per_block, hi, wbias, K, k_max, z, hist, tot, flagged, n_flagged)
      if (d == 128) {
        if (big)
          DPMM_UC(128, 512, 8);
        else
          DPMM_UC(128, 256, 8);
      } else {
        if (two)
          DPMM_UC(64, 256, 4);
        else if (big)
          DPMM_UC(64, 512, 8);
        else
          DPMM_UC(64, 256, 8);
      }
#undef DPMM_UC
    } else if (d == 64 || d == 128) {
      // static staging buffers; only the histogram is dynamic
#define DPMM_MFMA_W32(DD, XX, CC)                                                                            \
  hipExtLaunchKernelGGL((k_label_gauss_mfma_w32<DD, XX, CC>), dim3(Gp), dim3(BLOCK_W32), lh, s, e0, e1, 0, x, n, \
                        per_block, packed, hi, lo, K, t, seed, z, hist, tot, flagged, cand, n_flagged, 1,        \
                        (CC) && cst ? CAND_SPLIT_CAP : 0, nullptr)
      // the candidate pass scores in bf16x3 whatever the main pass's form; while
      // few points are deferred its clusters are split over CAND_SPLIT_NG
      // workgroups per point chunk and the lists merged (the single form below
      // then returns at once)
      if (cands && cst) {
        const unsigned gx = (unsigned)((CAND_SPLIT_CAP + BLOCK_W32 / 2 - 1) / (BLOCK_W32 / 2) < Gp
                                           ? (CAND_SPLIT_CAP + BLOCK_W32 / 2 - 1) / (BLOCK_W32 / 2)
                                           : Gp);
        if (d == 128)
          hipLaunchKernelGGL((k_label_gauss_mfma_w32<128, true, true>), dim3(gx, CAND_SPLIT_NG), dim3(BLOCK_W32), lh, s,
                             x, n, per_block, packed, hi, lo, K, t, seed, z, hist, tot, flagged, cand, n_flagged,
                             CAND_SPLIT_NG, CAND_SPLIT_CAP, cst);
        else
          hipLaunchKernelGGL((k_label_gauss_mfma_w32<64, true, true>), dim3(gx, CAND_SPLIT_NG), dim3(BLOCK_W32), lh, s,
                             x, n, per_block, packed, hi, lo, K, t, seed, z, hist, tot, flagged, cand, n_flagged,
                             CAND_SPLIT_NG, CAND_SPLIT_CAP, cst);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_cands_merge, dim3(CAND_SPLIT_CAP / 256), dim3(256), 0, s, n_flagged, CAND_SPLIT_NG,
                           CAND_SPLIT_CAP, cst, BF16X3_TOL_REL, K, per_block, t, seed, flagged, z, hist, tot, cand);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
      if (d == 128) {
        if (cands)
          DPMM_MFMA_W32(128, true, true);
        else if (x3)
          DPMM_MFMA_W32(128, true, false);
        else
          DPMM_MFMA_W32(128, false, false);
      } else {
        if (cands)
          DPMM_MFMA_W32(64, true, true);
        else if (x3)
          DPMM_MFMA_W32(64, true, false);
        else
          DPMM_MFMA_W32(64, false, false);
      }
#undef DPMM_MFMA_W32
    } else if (d == 32) {
      // [CG][NB][NF] fragments (64 KB), [CG][d + 4] means and constants, the histogram;
      // the candidate pass scores in bf16x3
      const size_t lds = (size_t)65536 + (size_t)(x3 || cands ? 16 : 32) * (d + 4) * sizeof(float) + lh;
#define DPMM_MFMA32(XX, CC)                                                                                  \
  hipExtLaunchKernelGGL((k_label_gauss_mfma32<XX, CC>), dim3(Gp), dim3(BLOCK32), lds, s, e0, e1, 0, x, n, per_block, \
                        packed, hi, lo, K, t, seed, z, hist, tot, flagged, cand, n_flagged)
      if (cands)
        DPMM_MFMA32(true, true);
      else if (x3)
        DPMM_MFMA32(true, false);
      else
        DPMM_MFMA32(false, false);
#undef DPMM_MFMA32
    } else {
      return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // the deferred points in FP32 (grid-strided; the count stays on the device)
#define DPMM_RESCORE(DD)                                                                                 \
  hipLaunchKernelGGL(k_rescore_flagged<DD>, dim3(512), dim3(RS_BLOCK), 0, s, x, flagged, cand, n_flagged, \
                     per_block, packed, K, t, seed, z, hist, tot)
  if (d == 32)
    DPMM_RESCORE(32);
  else if (d == 64)
    DPMM_RESCORE(64);
  else
    DPMM_RESCORE(128);
#undef DPMM_RESCORE
  return hipGetLastError();
}

}  // namespace dpmm
