// Cluster-sorted second half of the Gaussian label step, for d >= 5:
// Sec. 4.1 step (f) (sub-labels) and the statistics update of Sec. 4.4.
//
// After the cluster draw, points are counting-sorted by z:
//   k_hist_z     per-block histogram of z over contiguous point ranges (only
//                when the label kernel did not produce it);
//   k_scan_hist  per-(block, cluster) output offsets;
//   k_scatter_z  perm[offset] = i, zsort[offset] = z_i (the cluster of each
//                sorted row, read coalesced by the kernels below).
// Then k_sub_stats walks the sorted order in tiles of TR rows.  A tile holds
// one or a few clusters, so sub-cluster scoring reads the two sub-cluster
// records of a cluster with wave-uniform (scalar) loads instead of per-lane
// gathers.  The tile's rows are then placed in LDS grouped by segment
// s = 2 z + zsub, and every lane accumulates a 2x2 block of sum x x^T (or two
// entries of sum x) in float64 registers over each segment's rows, with one
// global atomic per entry, segment and tile.
#include <utility>

#include "kernels.hpp"
#include "score.hpp"

namespace dpmm {

namespace {

using score::BLOCK;
using score::score_rec;
using score::score_rec_dyn;
constexpr int IPT_MAX = 9;  // 2x2 work items per lane for d <= 128
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;

// Inclusive scan over a workgroup of `NT` threads (integer: exact in any
// order), left in buf (NT ints) as well: shuffles within each wave, then the
// preceding waves' totals (staged in buf's first entries); three barriers.
template <int NT>
__device__ __forceinline__ int block_inclusive_scan_n(int v, int* buf) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  if (lane == 63) buf[w] = v;
  __syncthreads();
  int add = 0;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) add += q < w ? buf[q] : 0;
  v += add;
  __syncthreads();  // every wave has read the totals
  buf[tid] = v;
  __syncthreads();
  return v;
}

__device__ __forceinline__ int block_inclusive_scan(int v, int* buf) { return block_inclusive_scan_n<BLOCK>(v, buf); }

}  // namespace

__global__ __launch_bounds__(BLOCK) void k_hist_z(const int* __restrict__ z, long long n, long long per_block, int K,
                                                  int* __restrict__ hist, int* __restrict__ tot) {
  extern __shared__ int h[];
  for (int k = threadIdx.x; k < K; k += BLOCK) h[k] = 0;
  __syncthreads();
  const long long begin = (long long)blockIdx.x * per_block;
  const long long end = begin + per_block < n ? begin + per_block : n;
  for (long long i = begin + threadIdx.x; i < end; i += BLOCK) {
    const int zi = z[i];
    if ((unsigned)zi < (unsigned)K) atomicAdd(&h[zi], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += BLOCK) {
    hist[(size_t)blockIdx.x * K + k] = h[k];
    if (h[k]) atomicAdd(&tot[k], h[k]);
  }
}

// One workgroup per cluster k: offs[b][k] = sum_{k' < k} tot[k'] + sum_{b' < b} hist[b'][k].
__global__ __launch_bounds__(BLOCK) void k_scan_hist(const int* __restrict__ hist, int G, int K,
                                                     const int* __restrict__ tot, int* __restrict__ offs) {
  __shared__ int buf[BLOCK];
  __shared__ long long base_sh;
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  long long b0 = 0;
  for (int q = tid; q < k; q += BLOCK) b0 += tot[q];
  // reduce b0 over the block
  buf[tid] = (int)b0;  // cluster totals are below 2^31 (n < 2^31 for this path)
  __syncthreads();
  if (tid == 0) {
    long long s = 0;
    for (int q = 0; q < BLOCK; ++q) s += buf[q];
    base_sh = s;
  }
  __syncthreads();
  const int per = (G + BLOCK - 1) / BLOCK;
  const int g0 = tid * per;
  int local = 0;
  for (int g = g0; g < g0 + per && g < G; ++g) local += hist[(size_t)g * K + k];
  const int incl = block_inclusive_scan(local, buf);
  int run = (int)base_sh + incl - local;
  for (int g = g0; g < g0 + per && g < G; ++g) {
    offs[(size_t)g * K + k] = run;
    run += hist[(size_t)g * K + k];
  }
}

// Stable scatter: within block b the rows of a cluster keep their index
// order, so the sorted order (and every float64 sum taken over it) does not
// depend on timing.  Wave w owns the contiguous quarter [begin + w q, begin +
// (w + 1) q) of the block's range (q = per_block / 4, a multiple of 64): it
// counts its rows per cluster (LDS integer atomics, exact), its cursor for
// cluster k is the block's offset plus the counts of the waves before it, and
// it then walks its quarter 64 rows at a time.  The lanes holding the same
// cluster are found with one ballot per bit of the cluster index (the lanes
// that agree with this lane on every bit); a lane's rank among them is the
// count of those below it, and the highest of them moves the cursor.
__global__ __launch_bounds__(BLOCK) void k_scatter_z(const int* __restrict__ z, long long n, long long per_block,
                                                     int K, const int* __restrict__ offs, int* __restrict__ perm,
                                                     int* __restrict__ zsort) {
  extern __shared__ int cur[];  // [4][K]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int q = threadIdx.x; q < 4 * K; q += BLOCK) cur[q] = 0;
  __syncthreads();
  const long long begin = (long long)blockIdx.x * per_block;
  const long long end = begin + per_block < n ? begin + per_block : n;
  const long long quarter = per_block / 4;
  const long long wb = begin + w * quarter;
  const long long we = wb + quarter < end ? wb + quarter : end;
  int* mine = cur + w * K;
  for (long long i = wb + lane; i < we; i += 64) {
    const int zi = z[i];
    if ((unsigned)zi < (unsigned)K) atomicAdd(&mine[zi], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += BLOCK) {
    int run = offs[(size_t)blockIdx.x * K + k];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = cur[u * K + k];
      cur[u * K + k] = run;
      run += c;
    }
  }
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
  int nbits = 1;
  while ((1 << nbits) < K) ++nbits;
  for (long long c0 = wb; c0 < we; c0 += 64) {
    const long long i = c0 + lane;
    const int zi = i < we ? z[i] : -1;
    const bool v = (unsigned)zi < (unsigned)K;
    unsigned long long m = __ballot(v);
    for (int b = 0; b < nbits; ++b) {
      const unsigned long long on = __ballot(v && ((zi >> b) & 1));
      m &= ((zi >> b) & 1) ? on : ~on;
    }
    int base = 0;
    if (v) base = mine[zi];
    // every lane has read its cursor before any moves (wave order)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (v) {
      const int pos = base + __popcll(m & below);
      perm[pos] = (int)i;
      zsort[pos] = zi;
      if ((m >> lane) == 1ull) mine[zi] = base + __popcll(m);  // the highest lane of its cluster
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// 2x2 work items of one lane for dimension D (0: the generic bound, d <= 128)
__host__ __device__ constexpr int items_per_lane(int D) {
  return D == 0 ? IPT_MAX : ((((D + 1) / 2) * ((D + 1) / 2 + 1) / 2 + (D + 1) / 2) + 255) / 256;
}

// D > 0: a lane's row stays in registers for sub-cluster scoring and is then
// stored straight to its segment-sorted LDS position; D == 0 (generic d): rows
// are staged in LDS and reached through an index list.  SAMPLE: draw zsub
// (else read it).  Workgroup g walks the tiles [g tpw, (g + 1) tpw) of TR
// sorted rows each (TR <= BLOCK: one row per lane).  Clusters are contiguous
// in sorted order, so the lanes keep float64 accumulators of the current
// cluster's two segments across tiles; each segment keeps the rows' sorted
// order.  Slot mode (part != nullptr, cstart / ctot indexed by cluster -
// kbase): a cluster inside the workgroup's rows is written to its final
// place, the first and last clusters that reach beyond them to partial slots
// 2 g, 2 g + 1 that k_sub_stats_fix adds in a fixed order.  Otherwise the
// sums are added with global atomics when the cluster changes.
template <int D, bool SAMPLE>
__global__ __launch_bounds__(BLOCK) void k_sub_stats(const float* __restrict__ x, int d, int TR, int tpw,
                                                     long long n_sorted, const int* __restrict__ perm,
                                                     const int* __restrict__ z, unsigned char* __restrict__ zsub,
                                                     const float* __restrict__ packed, int K, int k_max, uint32_t t,
                                                     uint64_t seed, long long* __restrict__ counts,
                                                     double* __restrict__ moments, const int* __restrict__ cstart,
                                                     const int* __restrict__ ctot, int kbase,
                                                     double* __restrict__ part) {
  constexpr int IPT = items_per_lane(D);
  extern __shared__ float lds[];
  const int tid = threadIdx.x;
  const int dp = (d + 1) & ~1;  // even, padded with a zero column
  const int ld = dp + 1;        // odd row stride: lanes touching their own rows hit distinct banks
  float* xs = lds;                                         // [TR][ld]
  int* rk = reinterpret_cast<int*>(xs + (size_t)TR * ld);  // [TR] cluster of the row
  int* order = rk + TR;                                    // [TR] (generic d) row of each sorted slot
  int* lcount = order + TR;                                // [2 TR]
  int* lstart = lcount + 2 * TR;                           // [2 TR]
  int* rinfo = lstart + 2 * TR;                            // [2 TR]: run start row, right rows before it
  int* buf = rinfo + 2 * TR;                               // [BLOCK]
  int* rcl = buf + BLOCK;                                  // [TR] cluster of each run
  float* dxc = reinterpret_cast<float*>(rcl + TR);         // [d][BLOCK] (generic d, SAMPLE only)
  const int S = gauss_rec_stride(d);
  const int E = d + d * (d + 1) / 2;
  // this lane's 2x2 work items: blocks (I, J), I <= J, of sum x x^T over the
  // even-padded dimension, then pairs I of sum x (J = -2)
  const int hb = dp / 2;
  const int n_tri = hb * (hb + 1) / 2;
  const int n_items = n_tri + hb;
  short iI[IPT], iJ[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int it = tid + j * BLOCK;
    iI[j] = -1;
    iJ[j] = -1;
    if (it < n_tri) {
      int u = it, a = 0;
      while (u >= hb - a) {
        u -= hb - a;
        ++a;
      }
      iI[j] = (short)a;
      iJ[j] = (short)(a + u);
    } else if (it < n_items) {
      iI[j] = (short)(it - n_tri);
      iJ[j] = -2;
    }
  }
  const long long tiles = (n_sorted + TR - 1) / TR;
  const long long tile_beg = (long long)blockIdx.x * tpw;
  const long long tile_end = tile_beg + tpw < tiles ? tile_beg + tpw : tiles;
  const long long r_begin = tile_beg * TR;
  const long long r_end = tile_end * TR < n_sorted ? tile_end * TR : n_sorted;
  // running sums of the current cluster's left (accL) and right (accR)
  // segments; indexed statically so they stay in registers
  double accL[IPT][4], accR[IPT][4];
  long long cntL = 0, cntR = 0;
  int cur_k = -1, k_first = -1;
  auto zero_acc = [&]() {
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      accL[j][0] = accL[j][1] = accL[j][2] = accL[j][3] = 0.0;
      accR[j][0] = accR[j][1] = accR[j][2] = accR[j][3] = 0.0;
    }
    cntL = cntR = 0;
  };
  // atomic: added to M / C; else stored to M and C (or the slot's count Cd)
  auto flush_one = [&](double (&acc)[IPT][4], long long cnt, double* M, long long* C, double* Cd, bool atomic) {
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int I = iI[j], J = iJ[j];
      if (I < 0) continue;
      if (J == -2) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
          if (2 * I + u < d) {
            if (atomic)
              atomicAdd(&M[2 * I + u], acc[j][u]);
            else
              M[2 * I + u] = acc[j][u];
          }
      } else {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            const int a = 2 * I + u, b = 2 * J + v;
            if (a < d && b < d && a <= b) {
              double* dst = &M[d + a * d - (a * (a - 1)) / 2 + (b - a)];
              if (atomic)
                atomicAdd(dst, acc[j][2 * u + v]);
              else
                *dst = acc[j][2 * u + v];
            }
          }
      }
    }
    if (tid == 0) {
      if (atomic)
        atomicAdd((unsigned long long*)C, (unsigned long long)cnt);
      else if (C)
        *C = cnt;
      else
        *Cd = (double)cnt;
    }
  };
  auto flush = [&]() {
    if (cur_k < 0) return;
    const int sL = 2 * cur_k, sR = sL + 1;
    if (!part) {
      if (cntL) flush_one(accL, cntL, moments + (size_t)sL * E, counts + sL, nullptr, true);
      if (cntR) flush_one(accR, cntR, moments + (size_t)sR * E, counts + sR, nullptr, true);
      return;
    }
    const long long cs = cstart[cur_k - kbase], ce = cs + ctot[cur_k - kbase];
    if (cs >= r_begin && ce <= r_end) {
      flush_one(accL, cntL, moments + (size_t)sL * E, counts + sL, nullptr, false);
      flush_one(accR, cntR, moments + (size_t)sR * E, counts + sR, nullptr, false);
    } else {
      double* P = part + (size_t)(2 * blockIdx.x + (cur_k == k_first ? 0 : 1)) * 2 * (E + 1);
      flush_one(accL, cntL, P + 1, nullptr, P, false);
      flush_one(accR, cntR, P + (E + 1) + 1, nullptr, P + (E + 1), false);
    }
  };
  auto accumulate = [&](double (&acc)[IPT][4], int st, int cnt) {
#pragma unroll 4
    for (int p = st; p < st + cnt; ++p) {
      const float* xr = xs + (size_t)(D > 0 ? p : order[p]) * ld;
#pragma unroll
      for (int j = 0; j < IPT; ++j) {
        const int I = iI[j], J = iJ[j];
        if (I < 0) continue;
        const double a0 = xr[2 * I], a1 = xr[2 * I + 1];
        if (J == -2) {
          acc[j][0] += a0;
          acc[j][1] += a1;
        } else {
          const double b0 = xr[2 * J], b1 = xr[2 * J + 1];
          acc[j][0] = fma(a0, b0, acc[j][0]);
          acc[j][1] = fma(a0, b1, acc[j][1]);
          acc[j][2] = fma(a1, b0, acc[j][2]);
          acc[j][3] = fma(a1, b1, acc[j][3]);
        }
      }
    }
  };
  zero_acc();
  for (long long tile = tile_beg; tile < tile_end; ++tile) {
    const long long tile0 = tile * TR;
    const int rows = (int)((n_sorted - tile0) < TR ? (n_sorted - tile0) : TR);
    const int r = tid;
    const bool valid = r < rows;
    // ---- phase A: load the row, draw or read its sub-label
    long long i = 0;
    int k = -1;
    float xv[D > 0 ? D : 1];
    if (valid) {
      i = perm[tile0 + r];
      k = z[i];
      rk[r] = k;
      if constexpr (D > 0) {
#pragma unroll
        for (int j = 0; j < D; ++j) xv[j] = x[i * D + j];
      } else {
        // eight loads in flight at a time (d is not known at compile time)
        float* xr = xs + (size_t)r * ld;
        for (int j0 = 0; j0 < d; j0 += 8) {
          float tv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) tv[u] = j0 + u < d ? x[i * d + j0 + u] : 0.0f;
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (j0 + u < d) xr[j0 + u] = tv[u];
        }
        for (int j = d; j < dp; ++j) xr[j] = 0.0f;
      }
    }
    for (int q = tid; q < 2 * TR; q += BLOCK) lcount[q] = 0;
    int zs = 0;
    if (SAMPLE) {
      float delta = 0.0f;
      unsigned long long pending = __ballot(valid);
      while (pending) {
        const int lane0 = __ffsll((long long)pending) - 1;
        const int kk = __shfl(k, lane0);
        const bool mine = valid && k == kk;
        if (mine) {
          const float* ps = packed + (size_t)(k_max + 2 * kk) * S;
          if constexpr (D > 0) {
            delta = score_rec<D>(ps, xv) - score_rec<D>(ps + S, xv);
          } else {
            const float* xr = xs + (size_t)r * ld;
            delta = score_rec_dyn(ps, xr, dxc + tid, d) - score_rec_dyn(ps + S, xr, dxc + tid, d);
          }
        }
        pending &= ~__ballot(mine);
      }
      if (valid) {
        zs = sub_label_draw(delta, seed, t, (uint32_t)i, K);
        zsub[i] = (unsigned char)zs;
      }
    } else if (valid) {
      zs = zsub[i] ? 1 : 0;
    }
    __syncthreads();
    // ---- group rows by segment: run of the cluster (rows are sorted by z),
    // then the sub-label; one scan gives the run of each row (high half) and
    // the right rows up to it (low half)
    const int flag = (valid && (r == 0 || rk[r] != rk[r - 1])) ? 1 : 0;
    const int sc = block_inclusive_scan((flag << 16) | zs, buf);
    const int run = (sc >> 16) - 1, ones_ex = (sc & 0xFFFF) - zs;
    const int nruns = buf[BLOCK - 1] >> 16;
    const int lid = 2 * run + zs;
    if (flag) {
      rinfo[2 * run] = r;
      rinfo[2 * run + 1] = ones_ex;
      rcl[run] = k;
    }
    if (valid) atomicAdd(&lcount[lid], 1);  // integer counts: exact in any order
    __syncthreads();
    if (tid == 0) {
      int a = 0;
      for (int q = 0; q < 2 * nruns; ++q) {
        lstart[q] = a;
        a += lcount[q];
      }
    }
    __syncthreads();
    // slot within the segment: the row's rank among the run's rows of the same
    // sub-label, so each segment keeps the sorted order
    if (valid) {
      const int ones_run = ones_ex - rinfo[2 * run + 1];
      const int pos = lstart[lid] + (zs ? ones_run : (r - rinfo[2 * run]) - ones_run);
      if constexpr (D > 0) {
        float* xr = xs + (size_t)pos * ld;
#pragma unroll
        for (int j = 0; j < D; ++j) xr[j] = xv[j];
        if (D & 1) xr[D] = 0.0f;
      } else {
        order[pos] = r;
      }
    }
    __syncthreads();
    // ---- phase B: every run in order into the running sums
    for (int j = 0; j < nruns; ++j) {
      const int kq = rcl[j];
      if (kq != cur_k) {
        flush();
        zero_acc();
        if (cur_k < 0) k_first = kq;
        cur_k = kq;
      }
      const int cl = lcount[2 * j], cr = lcount[2 * j + 1];
      cntL += cl;
      cntR += cr;
      accumulate(accL, lstart[2 * j], cl);
      accumulate(accR, lstart[2 * j + 1], cr);
    }
    __syncthreads();
  }
  flush();
}

// Wave-independent kernel for D in {8, 16, 32}: each wave walks its own
// contiguous range of sorted rows in chunks of 64 (one row per lane), with no
// workgroup barriers.  Per chunk:
//   (1) sub-cluster scores: for each run of lanes with the same cluster (rows
//       are sorted by z, so a cluster is a run of lanes) every lane scores the
//       run's two sub-cluster records; control flow stays wave-uniform, so the
//       records are read with scalar loads, and each lane keeps the result of
//       its own run;
//   (2) each row is stored to LDS at its segment-sorted slot: within a run the
//       left rows first, then the right rows;
//   (3) per segment, four rows at a time, v_mfma_f64_16x16x4_f64 adds the
//       16x16 blocks (I <= J) of sum x x^T (dimensions padded to a multiple
//       of 16 with zeros); the same operands give sum x.
// The current cluster's two segments are carried across chunks and flushed
// with global atomics when the cluster changes or the range ends.
template <int D, bool SAMPLE>
__global__ __launch_bounds__(BLOCK) void k_sub_stats_w(const float* __restrict__ x, long long npts, long long n_sorted,
                                                       long long rows_per_wave, const int* __restrict__ perm,
                                                       const int* __restrict__ z, const int* __restrict__ zrow,
                                                       unsigned char* __restrict__ zsub,
                                                       const float* __restrict__ packed, int K, int k_max, uint32_t t,
                                                       uint64_t seed, long long* __restrict__ counts,
                                                       double* __restrict__ moments, const int* __restrict__ cstart,
                                                       const int* __restrict__ ctot, int kbase,
                                                       double* __restrict__ part) {
  constexpr int NB = (D + 15) / 16;  // 16-wide blocks of dimensions
  constexpr int NBLK = NB * (NB + 1) / 2;
  constexpr int LDW = D + 1;  // odd row stride
  constexpr int S = (4 + D + D * (D + 1) / 2 + 3) & ~3;
  constexpr int E = D + D * (D + 1) / 2;
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* xs = lds + wave * 64 * LDW;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int col = lane & 15;
  f64x4 cL[NBLK], cR[NBLK];
  double sL[NB], sR[NB];
  long long nL = 0, nR = 0;
  int cur_k = -1;
  auto zero_acc = [&]() {
#pragma unroll
    for (int b = 0; b < NBLK; ++b) cL[b] = cR[b] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < NB; ++b) sL[b] = sR[b] = 0.0;
    nL = nR = 0;
  };
  const long long gw = (long long)blockIdx.x * (BLOCK / 64) + wave;
  const long long w_begin = gw * rows_per_wave;
  const long long w_end = w_begin + rows_per_wave < n_sorted ? w_begin + rows_per_wave : n_sorted;
  int k_first = -1;  // cluster of the wave's first row (partial-slot mode)
  // lane l holds element j of block (I, J) at row 16 I + l / 16 + 4 j, column 16 J + l % 16.
  // Atomic mode (part == nullptr): added to counts[seg], moments[seg].  Slot mode:
  // stored to M (moments layout) and *cnt_out, either the final arrays (the
  // cluster lies in this wave's rows) or a partial slot that k_sub_stats_fix sums.
  auto flush_one = [&](f64x4 (&c)[NBLK], double (&sx)[NB], long long cnt, double* M, long long* cnt_out,
                       double* cnt_d, bool atomic) {
    int blk = 0;
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = I; J < NB; ++J, ++blk)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int a = 16 * I + (lane >> 4) + 4 * j, b = 16 * J + col;
          if (a <= b && b < D) {
            double* dst = &M[D + a * D - (a * (a - 1)) / 2 + (b - a)];
            if (atomic)
              atomicAdd(dst, c[blk][j]);
            else
              *dst = c[blk][j];
          }
        }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      double v = sx[b];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (lane < 16 && 16 * b + lane < D) {
        if (atomic)
          atomicAdd(&M[16 * b + lane], v);
        else
          M[16 * b + lane] = v;
      }
    }
    if (lane == 0) {
      if (atomic)
        atomicAdd((unsigned long long*)cnt_out, (unsigned long long)cnt);
      else if (cnt_out)
        *cnt_out = cnt;
      else
        *cnt_d = (double)cnt;
    }
  };
  auto flush = [&]() {
    if (cur_k < 0) return;
    if (!part) {
      if (nL) flush_one(cL, sL, nL, moments + (size_t)(2 * cur_k) * E, &counts[2 * cur_k], nullptr, true);
      if (nR) flush_one(cR, sR, nR, moments + (size_t)(2 * cur_k + 1) * E, &counts[2 * cur_k + 1], nullptr, true);
      return;
    }
    const long long cs = cstart[cur_k - kbase], ce = cs + ctot[cur_k - kbase];
    if (cs >= w_begin && ce <= w_end) {
      // the whole cluster is this wave's: final values, both segments
      flush_one(cL, sL, nL, moments + (size_t)(2 * cur_k) * E, &counts[2 * cur_k], nullptr, false);
      flush_one(cR, sR, nR, moments + (size_t)(2 * cur_k + 1) * E, &counts[2 * cur_k + 1], nullptr, false);
    } else {
      // slot 2 gw: the wave's first cluster; 2 gw + 1: its last (when different); each [2][1 + E]
      double* P = part + (size_t)(2 * gw + (cur_k == k_first ? 0 : 1)) * 2 * (E + 1);
      flush_one(cL, sL, nL, P + 1, nullptr, P, false);
      flush_one(cR, sR, nR, P + (E + 1) + 1, nullptr, P + (E + 1), false);
    }
  };
  // rows [s0, e0) of the wave's LDS tile, four at a time: A = B = the rows' block of dimensions
  auto mfma_rows = [&](f64x4 (&c)[NBLK], double (&sx)[NB], int s0, int e0) {
    for (int g = s0; g < e0; g += 4) {
      // unconditional LDS reads of an element inside the tile (row s0, column 0 for a
      // lane past the rows or the dimensions), then zeroed: no branches, so the reads
      // of the next step can overlap the matrix-core work of this one
      const int rr = g + (lane >> 4);
      const bool ok = rr < e0;
      const int rs = ok ? rr : s0;
      double a[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int cc = 16 * b + col;
        const float v = xs[rs * LDW + (cc < D ? cc : 0)];
        a[b] = (ok && cc < D) ? (double)v : 0.0;
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) sx[b] += a[b];
      int blk = 0;
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = I; J < NB; ++J, ++blk) c[blk] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[I], a[J], c[blk], 0, 0, 0);
    }
  };
  zero_acc();
  for (long long c0 = w_begin; c0 < w_end; c0 += 64) {
    const long long r = c0 + lane;
    bool valid = r < w_end;
    long long i = 0;
    int k = -1;
    float xv[D];
    if (valid) {
      i = perm[r];
      // a label outside [0, K) leaves its row out (and never reaches memory)
      valid = (unsigned long long)i < (unsigned long long)npts;
      if (valid) k = zrow ? zrow[r] : z[i];
      valid = valid && (unsigned)k < (unsigned)K;
    }
    if (valid) {
#pragma unroll
      for (int j = 0; j < D; ++j) xv[j] = x[i * D + j];
    } else {
      i = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) xv[j] = 0.0f;
    }
    // ---- (1) sub-labels
    int zs = 0;
    if (SAMPLE) {
      float delta = 0.0f;
      unsigned long long pend = __ballot(valid);
      while (pend) {
        const int lane0 = __ffsll((long long)pend) - 1;
        const int kk = __builtin_amdgcn_readlane(k, lane0);
        const bool mine = valid && k == kk;
        const float* ps = packed + (size_t)(k_max + 2 * kk) * S;
        const float dl = score_rec<D>(ps, xv) - score_rec<D>(ps + S, xv);
        if (mine) delta = dl;
        pend &= ~__ballot(mine);
      }
      if (valid) {
        zs = sub_label_draw(delta, seed, t, (uint32_t)i, K);
        zsub[i] = (unsigned char)zs;
      }
    } else if (valid) {
      zs = zsub[i] ? 1 : 0;
    }
    // ---- (2) segment-sorted slot of each row
    const unsigned long long right = __ballot(valid && zs == 1);
    int pos = 0;
    unsigned long long rem = __ballot(valid);
    while (rem) {
      const int lane0 = __ffsll((long long)rem) - 1;
      const int kk = __builtin_amdgcn_readlane(k, lane0);
      const bool mine = valid && k == kk;
      const unsigned long long mk = __ballot(mine);
      const unsigned long long mR = mk & right, mL = mk & ~right;
      if (mine) pos = lane0 + (zs ? __popcll(mL) + __popcll(mR & below) : __popcll(mL & below));
      rem &= ~mk;
    }
    // the previous chunk's reads of xs are done: same wave, in order
    __builtin_amdgcn_wave_barrier();
    if (valid) {
#pragma unroll
      for (int j = 0; j < D; ++j) xs[pos * LDW + j] = xv[j];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // ---- (3) each run's two segments into the running sums
    rem = __ballot(valid);
    while (rem) {
      const int lane0 = __ffsll((long long)rem) - 1;
      const int kk = __builtin_amdgcn_readlane(k, lane0);
      const unsigned long long mk = __ballot(valid && k == kk);
      if (kk != cur_k) {
        flush();
        zero_acc();
        if (cur_k < 0) k_first = kk;
        cur_k = kk;
      }
      const int cl = __popcll(mk & ~right), cr = __popcll(mk & right);
      nL += cl;
      nR += cr;
      mfma_rows(cL, sL, lane0, lane0 + cl);
      mfma_rows(cR, sR, lane0 + cl, lane0 + cl + cr);
      rem &= ~mk;
    }
  }
  flush();
}

// Slot mode of the sorted-order statistics kernels: the counts and moments of
// every cluster whose rows span several row ranges (rpw rows each: a wave of
// k_sub_stats_w, a workgroup of the other kernels) are the sums of those
// ranges' partial slots (2 g for the range's first cluster, 2 g + 1 for its
// last); empty clusters get zeros; a cluster inside one range was written by
// it.  Grid (entries / FIX_EN, clusters): cluster kbase + blockIdx.y, whose
// start and size are cstart / ctot[blockIdx.y].  FIX_PH phases of threads take
// every FIX_PH-th slot of FIX_EN entries, and their sums are added in a fixed
// order (the result does not depend on timing).
constexpr int FIX_PH = 16, FIX_EN = 16;
__global__ __launch_bounds__(FIX_PH * FIX_EN) void k_sub_stats_fix(int E, long long rpw, const int* __restrict__ cstart,
                                                                 const int* __restrict__ ctot,
                                                                 const double* __restrict__ part,
                                                                 long long* __restrict__ counts,
                                                                 double* __restrict__ moments, int kbase) {
  __shared__ double red[FIX_PH][FIX_EN];
  const int k = blockIdx.y;
  const int W = 2 * (E + 1);
  const int el = threadIdx.x % FIX_EN, ph = threadIdx.x / FIX_EN;
  const int e = blockIdx.x * FIX_EN + el;
  const long long cs = cstart[k], cnt = ctot[k];
  const long long ga = cnt > 0 ? cs / rpw : 0, gb = cnt > 0 ? (cs + cnt - 1) / rpw : -1;
  if (cnt > 0 && ga == gb) return;  // written by the range that holds it (uniform over the block)
  double v = 0.0;
  if (e < W) {
#pragma unroll 4
    for (long long g = ga + ph; g <= gb; g += FIX_PH)
      v += part[(size_t)(2 * g + (g == ga && cs != g * rpw ? 1 : 0)) * W + e];
  }
  red[ph][el] = v;
  __syncthreads();
  if (ph != 0 || e >= W) return;
  double sum = 0.0;
  for (int q = 0; q < FIX_PH; ++q) sum += red[q][el];
  const int h = e / (E + 1), f = e - h * (E + 1);
  const size_t seg = 2 * ((size_t)k + kbase) + h;
  if (f == 0)
    counts[seg] = (long long)sum;  // a sum of integer counts below 2^53: exact
  else
    moments[seg * E + (f - 1)] = sum;
}

namespace {

struct SortedPlan {
  int G;
  long long per_block;
};

SortedPlan plan_blocks(long long n, int K, long long hist_cap) {
  long long G = (n + 511) / 512;
  if (G > 2048) G = 2048;
  while (G > 1 && G * K > hist_cap) G = (G + 1) / 2;
  if (G < 1) G = 1;
  long long per = (n + G - 1) / G;
  per = ((per + BLOCK - 1) / BLOCK) * BLOCK;
  G = (n + per - 1) / per;
  if (G < 1) G = 1;
  return SortedPlan{(int)G, per};
}

int tile_rows(int d) {
  if (d <= 32) return 256;
  if (d <= 64) return 128;
  return 32;  // generic d up to 128: the per-lane centred columns take d x 1 KB of LDS
}

size_t sub_stats_lds(int d, int TR, bool generic) {
  const int dp = (d + 1) & ~1;
  size_t b = (size_t)TR * (dp + 1) * sizeof(float) + (size_t)(9 * TR + BLOCK) * sizeof(int);
  if (generic) b += (size_t)d * BLOCK * sizeof(float);
  return b;
}


constexpr int BIG_THREADS = 512;  // 8 waves: 0-3 own the left segment, 4-7 the right
// sorted rows per tile: 64 KB of FP32 rows, so that two tiles fit in LDS
constexpr int big_rows_of(int d) { return 16384 / d; }
typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ int block_inclusive_scan_big(int v, int* buf) { return block_inclusive_scan_n<BIG_THREADS>(v, buf); }

// Sub-label draw of sorted rows on the FP32 matrix cores (d = 32, 64, 128), Sec. 4.1
// step (f): the scores of the two sub-clusters of the row's cluster, from
// Y = W_h (x - mu_h) with v_mfma_f32_32x32x2_f32 (A = W_h, B = the centred
// rows).  A workgroup walks a contiguous range of sorted rows; the two records
// of the current cluster are staged in LDS whenever the cluster changes.  A
// wave scores 64 rows (two 32-row tiles): a lane holds half the coordinates of
// one row, k = 2s + h at MFMA step s (h = lane / 32).  The rows are centred
// once on mu_0; sub-cluster 1 starts its accumulators at W_1 (mu_0 - mu_1), so
// that both products read the same centred rows.  Row blocks of W above the
// diagonal are skipped (k <= 32 mt + 31 for output rows 32 mt ... 32 mt + 31)
// and the entries above the diagonal inside a block are read as zero.  With
// n_dev the rows are the list of n_dev[0] rows that the bf16x3 pass left
// undecided (n_sorted then only bounds the grid).
constexpr int SUBL_BLOCK = 256;

template <int D>
__global__ __launch_bounds__(SUBL_BLOCK) __attribute__((amdgpu_waves_per_eu(2, D <= 32 ? 3 : 2))) void k_sub_labels_mfma(
    const float* __restrict__ x, long long n_sorted, long long per_block, const int* __restrict__ perm,
    const int* __restrict__ z, const int* __restrict__ zrow, unsigned char* __restrict__ zsub,
    const float* __restrict__ packed, int K, int k_max, uint32_t t, uint64_t seed, const int* __restrict__ n_dev) {
  constexpr int S = (4 + D + D * (D + 1) / 2 + 3) & ~3;
  constexpr int MT = D / 32, HALF = D / 2, QTR = D / 4;
  if (n_dev) {  // a row list whose length is on the device: split it evenly over the grid
    n_sorted = *n_dev;
    per_block = ((n_sorted + gridDim.x - 1) / gridDim.x + 63) / 64 * 64;
  }
  static_assert(D % 32 == 0 && D <= SUBL_BLOCK, "layout");
  typedef float f32x16 __attribute__((ext_vector_type(16)));
  extern __shared__ __align__(16) float s_rec[];  // records of sub-clusters 0 and 1, then W_1 (mu_0 - mu_1), mu_0 - mu_1
  float* s_corr = s_rec + 2 * S;
  float* s_dmu = s_corr + D;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, col = lane & 31;
  const long long begin = (long long)blockIdx.x * per_block;
  const long long end = begin + per_block < n_sorted ? begin + per_block : n_sorted;
  auto kof = [&](long long g) { return __builtin_amdgcn_readfirstlane(zrow ? zrow[g] : z[perm[g]]); };
  int staged = -1;
  for (long long chunk = begin; chunk < end; chunk += SUBL_BLOCK) {
    const long long cend = chunk + SUBL_BLOCK < end ? chunk + SUBL_BLOCK : end;
    const long long base = chunk + wave * 64;
    const long long rA = base + col, rB = base + 32 + col;
    const bool vA = rA < cend, vB = rB < cend;
    const long long iA = vA ? perm[rA] : 0, iB = vB ? perm[rB] : 0;
    const int kA = vA ? (zrow ? zrow[rA] : z[iA]) : -1, kB = vB ? (zrow ? zrow[rB] : z[iB]) : -1;
    const int kmine = h ? kB : kA;
    float delta = 0.0f;
    int cur = kof(chunk);
    const int last = kof(cend - 1);
    for (;;) {
      if (cur != staged) {
        __syncthreads();  // every wave is done with the previous records
        const float4* src = reinterpret_cast<const float4*>(packed + (size_t)(k_max + 2 * cur) * S);
        float4* dst = reinterpret_cast<float4*>(s_rec);
        for (int j = threadIdx.x; j < 2 * S / 4; j += SUBL_BLOCK) dst[j] = src[j];
        __syncthreads();
        if (threadIdx.x < D) s_dmu[threadIdx.x] = s_rec[4 + threadIdx.x] - s_rec[S + 4 + threadIdx.x];
        __syncthreads();
        if (threadIdx.x < D) {
          const int i = threadIdx.x;
          const float* w1 = s_rec + S + 4 + D + i * (i + 1) / 2;
          float c = 0.0f;
          for (int k = 0; k <= i; ++k) c = fmaf(w1[k], s_dmu[k], c);
          s_corr[i] = c;
        }
        __syncthreads();
        staged = cur;
      }
      if (__ballot(kA == cur || kB == cur)) {
        // rows of the two tiles: lane h loads coordinates [HALF h, HALF h + HALF) and the two halves
        // trade so that ra[2j] = x[2j + h], ra[2j + 1] = x[HALF + 2j + h], centred on mu_0
        float ra[HALF], rb[HALF];
        const float4* pa = reinterpret_cast<const float4*>(x + (size_t)iA * D + HALF * h);
        const float4* pb = reinterpret_cast<const float4*>(x + (size_t)iB * D + HALF * h);
#pragma unroll
        for (int q = 0; q < HALF / 4; ++q) {
          const float4 va = vA ? pa[q] : make_float4(0.f, 0.f, 0.f, 0.f);
          const float4 vb = vB ? pb[q] : make_float4(0.f, 0.f, 0.f, 0.f);
          ra[4 * q] = va.x, ra[4 * q + 1] = va.y, ra[4 * q + 2] = va.z, ra[4 * q + 3] = va.w;
          rb[4 * q] = vb.x, rb[4 * q + 1] = vb.y, rb[4 * q + 2] = vb.z, rb[4 * q + 3] = vb.w;
        }
#pragma unroll
        for (int j = 0; j < QTR; ++j) {
          const float sa = __shfl_xor(h ? ra[2 * j] : ra[2 * j + 1], 32);
          const float sb = __shfl_xor(h ? rb[2 * j] : rb[2 * j + 1], 32);
          if (h) {
            ra[2 * j] = sa;
            rb[2 * j] = sb;
          } else {
            ra[2 * j + 1] = sa;
            rb[2 * j + 1] = sb;
          }
          const float m0 = s_rec[4 + 2 * j + h], m1 = s_rec[4 + HALF + 2 * j + h];
          ra[2 * j] -= m0;
          rb[2 * j] -= m0;
          ra[2 * j + 1] -= m1;
          rb[2 * j + 1] -= m1;
        }
        float sc[2];
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
          const float* rec = s_rec + sub * S;
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
            const int i = 32 * mt + col;
            const float* wr = rec + 4 + D + i * (i + 1) / 2 + h;
#pragma unroll
            for (int st = 0; st < 16 * (mt + 1); ++st) {
              float a = wr[2 * st];
              if (st >= 16 * mt && 2 * st + h > i) a = 0.0f;  // above the diagonal
              const int reg = st < QTR ? 2 * st : 2 * (st - QTR) + 1;
              acca = __builtin_amdgcn_mfma_f32_32x32x2f32(a, ra[reg], acca, 0, 0, 0);
              accb = __builtin_amdgcn_mfma_f32_32x32x2f32(a, rb[reg], accb, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              qa = fmaf(acca[r], acca[r], qa);
              qb = fmaf(accb[r], accb[r], qb);
            }
          }
          qa += __shfl_xor(qa, 32);
          qb += __shfl_xor(qb, 32);
          sc[sub] = fmaf(-0.5f, h ? qb : qa, rec[0]);
        }
        if (kmine == cur) delta = sc[0] - sc[1];
      }
      if (cur == last) break;
      // the next cluster: the first row of the chunk above cur (rows are sorted by cluster)
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
      zsub[i] = (unsigned char)sub_label_draw(delta, seed, t, (uint32_t)i, K);
    }
  }
}

size_t sub_labels_mfma_lds(int d) {
  const int S = (4 + d + d * (d + 1) / 2 + 3) & ~3;
  return (size_t)(2 * S + 2 * d) * sizeof(float);
}

// Upper 16 x 16 block u (row-major over I <= J) of an NB x NB block grid.
constexpr int blk_i(int u, int nb) {
  int a = 0;
  while (a < nb && u >= nb - a) {
    u -= nb - a;
    ++a;
  }
  return a;
}
constexpr int blk_j(int u, int nb) { return u - (blk_i(u, nb) * nb - blk_i(u, nb) * (blk_i(u, nb) - 1) / 2) + blk_i(u, nb); }

// The accumulator updates of one four-row step for wave quarter WQ: block
// u = WQ + 4 j of accumulator j, its (I, J) fixed at compile time so that the
// operands are plain registers.
template <int U, int NB>
constexpr int BLK_I = blk_i(U, NB) < NB ? blk_i(U, NB) : NB - 1;
template <int U, int NB>
constexpr int BLK_J = blk_i(U, NB) < NB ? blk_j(U, NB) : NB - 1;

template <int NB, int WQ, int TPW, int... J>
__device__ __forceinline__ void big_mfmas(f64x4 (&acc)[TPW], const double (&xv)[NB], std::integer_sequence<int, J...>) {
  constexpr int NT = NB * (NB + 1) / 2;
  ((WQ + 4 * J < NT
        ? (void)(acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[BLK_I<WQ + 4 * J, NB>], xv[BLK_J<WQ + 4 * J, NB>],
                                                               acc[J], 0, 0, 0))
        : (void)0),
   ...);
}

// Column held by lane i (of 16) for column block I in the statistics tile:
// lane i reads its D / 16 columns as one contiguous piece of the row (one or
// two 16-byte LDS reads), so block I is the column set {col(I, i)}.  At
// d = 128 the two halves of a lane's piece are read in an order that depends
// on bits 2 and 3 of i, so that any 8 or 16 consecutive lanes reading one row
// hit distinct LDS banks.
template <int D>
__device__ __forceinline__ int big_col(int blk, int i) {
  if constexpr (D == 128) {
    const int s = ((i >> 2) ^ (i >> 3)) & 1;
    return 8 * i + (blk ^ (4 * s));
  } else {
    return 4 * i + blk;
  }
}

// Rows [st, st + cnt) of a tile's order list, four at a time, into the
// accumulators of wave quarter WQ (upper blocks WQ, WQ + 4, ...): each step
// reads the lane's piece of its row once and feeds every block from it (a
// lane past the segment reads the zero row R).  rd0 / rd1: the lane's two
// 16-byte offsets in a row (rd1 unused at d = 64).
template <int D, int WQ, int R, int TPW>
__device__ __forceinline__ void big_rows(f64x4 (&acc)[TPW], double (&sx)[D / 64], const float* __restrict__ xs,
                                         const int* __restrict__ order, int st, int cnt, int lane, int rd0, int rd1) {
  constexpr int NB = D / 16;
  const int p = lane >> 4;
  // (a two-step software pipeline of these reads measured the same: the other
  // wave of the SIMD covers their latency, and while an LDS DMA is in flight
  // the compiler waits for every LDS read before its first use anyway)
  for (int g = 0; g < cnt; g += 4) {
    const int q = g + p;
    const float* rp = xs + (q < cnt ? order[st + q] : R) * D;
    const float4 a = *reinterpret_cast<const float4*>(rp + rd0);
    double xv[NB];
    xv[0] = (double)a.x;
    xv[1] = (double)a.y;
    xv[2] = (double)a.z;
    xv[3] = (double)a.w;
    if constexpr (NB == 8) {
      const float4 b = *reinterpret_cast<const float4*>(rp + rd1);
      xv[4] = (double)b.x;
      xv[5] = (double)b.y;
      xv[6] = (double)b.z;
      xv[7] = (double)b.w;
    }
    big_mfmas<NB, WQ>(acc, xv, std::make_integer_sequence<int, TPW>{});
    // sum x over the quarter's column blocks WQ, WQ + 4, ...: lane l adds
    // column col(block, l % 16) of its row
#pragma unroll
    for (int j = 0; j < D / 64; ++j) sx[j] += xv[WQ + 4 * j];
  }
}

// Statistics for d in {64, 128} over the cluster-sorted order (the sub-labels
// are drawn before, by the sub-label kernels), with sum x x^T on the FP64
// matrix cores.  A workgroup of 8 waves walks a contiguous range of tiles of
// big_rows_of(D) sorted rows (64 KB of rows each), two tiles' rows in LDS:
//   (1) the next tile's rows are copied into the other LDS buffer by LDS DMA
//       (global_load_lds, 16 bytes per lane, no registers) while this tile's
//       matrix-core work runs; its point indices, clusters and sub-labels are
//       loaded into registers at the same time;
//   (2) rows are grouped by segment (run of a cluster, sub-label), each
//       segment keeping the rows' sorted order (ranks from one block scan);
//   (3) per segment, four rows at a time, v_mfma_f64_16x16x4_f64 adds
//       X_I^T X_J to the upper 16 x 16 blocks (I, J) of sum x x^T (column
//       blocks as big_col gives them): the left segment belongs to waves 0-3,
//       the right to waves 4-7, and a wave owns blocks w, w + 4, ... (FP32
//       inputs are exact in FP64); from the same registers it also sums x over
//       its column blocks in FP64.
// The only barriers are those of the grouping, whose wait for all memory
// operations also lands the next tile's DMA issued one tile earlier.  Each
// wave carries its segment of the current cluster across tiles.  Slot mode
// (part != nullptr): a cluster that lies inside the workgroup's rows is
// written to its final place, the workgroup's first and last clusters that
// reach beyond them to partial slots 2 g and 2 g + 1 ([2][1 + E] each) that
// k_sub_stats_fix adds in a fixed order: no float atomics, so the sums do not
// depend on timing.  cstart / ctot are indexed by cluster - kbase.  Otherwise
// the segments are added to counts / moments with atomics.
template <int D>
__global__ __launch_bounds__(BIG_THREADS) void k_sub_stats_big(const float* __restrict__ x, long long n_sorted,
                                                               int tpb, const int* __restrict__ perm,
                                                               const int* __restrict__ z,
                                                               const int* __restrict__ zrow,
                                                               const unsigned char* __restrict__ zsub,
                                                               long long* __restrict__ counts,
                                                               double* __restrict__ moments,
                                                               const int* __restrict__ cstart,
                                                               const int* __restrict__ ctot, int kbase,
                                                               double* __restrict__ part) {
  constexpr int R = big_rows_of(D);
  constexpr int NB = D / 16, NT = NB * (NB + 1) / 2, TPW = (NT + 3) / 4;
  constexpr int E = D + D * (D + 1) / 2;
  constexpr int SB = D / 64;       // column blocks of sum x per wave
  constexpr int C4 = D / 4;        // 16-byte pieces per row
  constexpr int RPI = 64 / C4;     // rows per wave DMA instruction
  constexpr int NI = R / RPI / 8;  // DMA instructions per wave and tile
  static_assert(NI * RPI * 8 == R, "tile rows split evenly over the waves' DMA");
  // rows of two tiles, each followed by a zero row (read by lanes past a
  // segment).  Two arrays, and each tile's array fixed at compile time: the
  // compiler then knows that the rows a tile reads are not the ones its DMA
  // writes, and does not wait for the DMA before those reads.
  __shared__ float xa[(R + 1) * D], xb[(R + 1) * D];
  __shared__ int order[R], rk[R], buf[BIG_THREADS];
  __shared__ int lcount[2 * R], lstart[2 * R];
  __shared__ int rstart[R], ostart[R], rcl[R];
  __shared__ int nperm[2][R];  // point indices of the tiles whose rows are in flight
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int side = wave >> 2, wq = wave & 3;  // segment (0 left, 1 right), quarter
  int rd0, rd1;
  {
    const int i = lane & 15;
    if constexpr (D == 128) {
      const int s = ((i >> 2) ^ (i >> 3)) & 1;
      rd0 = 8 * i + 4 * s;
      rd1 = 8 * i + 4 * (1 - s);
    } else {
      rd0 = 4 * i;
      rd1 = rd0;
    }
  }
  const long long tiles = (n_sorted + R - 1) / R;
  const long long tb = (long long)blockIdx.x * tpb;
  const long long te = tb + tpb < tiles ? tb + tpb : tiles;
  const int nt = (int)(te - tb);
  const long long r_begin = tb * R;
  const long long r_end = te * R < n_sorted ? te * R : n_sorted;
  auto tile_rows = [&](int lt) __attribute__((always_inline)) -> int {
    const long long b = (tb + lt) * R;
    return (int)(n_sorted - b < R ? n_sorted - b : R);
  };
  f64x4 acc[TPW];
  double sx[SB];
  long long cnt_seg = 0;
  int cur_k = -1, k_first = -1;
  auto zero_acc = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < TPW; ++j) acc[j] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < SB; ++j) sx[j] = 0.0;
    cnt_seg = 0;
  };
  auto flush = [&]() __attribute__((always_inline)) {
    if (cur_k < 0) return;
    const int seg = 2 * cur_k + side;
    bool atomic = part == nullptr;
    double* M = moments + (size_t)seg * E;
    long long* C = counts + seg;
    double* Cd = nullptr;
    if (atomic) {
      if (cnt_seg == 0) return;
    } else {
      const long long cs = cstart[cur_k - kbase], ce = cs + ctot[cur_k - kbase];
      if (!(cs >= r_begin && ce <= r_end)) {
        double* P = part + ((size_t)(2 * blockIdx.x + (cur_k == k_first ? 0 : 1)) * 2 + side) * (E + 1);
        Cd = P;
        M = P + 1;
        C = nullptr;
      }
    }
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      // block (bI, bJ) of accumulator j: upper block wq + 4 j, row-major over I <= J
      int u = wq + 4 * j, bI = 0;
      if (u >= NT) continue;
      while (u >= NB - bI) {
        u -= NB - bI;
        ++bI;
      }
      const int bJ = bI + u;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // accumulator element e of lane l is row l / 16 + 4 e, column l % 16
        // of block (I, J): the pair of columns col(I, row), col(J, column)
        const int ra = (lane >> 4) + 4 * e, rb = lane & 15;
        if (bI == bJ && ra > rb) continue;  // a diagonal block holds both orders
        const int c1 = big_col<D>(bI, ra), c2 = big_col<D>(bJ, rb);
        const int a = c1 < c2 ? c1 : c2, b = c1 < c2 ? c2 : c1;
        double* dst = &M[D + a * D - (a * (a - 1)) / 2 + (b - a)];
        if (atomic)
          atomicAdd(dst, acc[j][e]);
        else
          *dst = acc[j][e];
      }
    }
#pragma unroll
    for (int j = 0; j < SB; ++j) {
      // the four row groups (lanes l, l + 16, l + 32, l + 48) combined
      double v = sx[j];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (lane < 16) {
        double* dst = &M[big_col<D>(wq + 4 * j, lane)];
        if (atomic)
          atomicAdd(dst, v);
        else
          *dst = v;
      }
    }
    if (wq == 0 && lane == 0) {
      if (atomic)
        atomicAdd((unsigned long long*)C, (unsigned long long)cnt_seg);
      else if (C)
        *C = cnt_seg;
      else
        *Cd = (double)cnt_seg;
    }
  };
  // LDS DMA of tile lt's rows into dst, the point indices from nperm[lt % 2]
  auto issue_rows = [&](int lt, float* dst) __attribute__((always_inline)) {
    const int rows = tile_rows(lt);
    const int* np = nperm[lt & 1];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      // rows past the tile's end copy its first row (never read): no branches,
      // so the compiler's count of loads in flight stays exact
      const int r0 = (wave * NI + i) * RPI;
      const int r = r0 + lane / C4;
      __builtin_amdgcn_global_load_lds((const void*)(x + (size_t)np[r < rows ? r : 0] * D + 4 * (lane % C4)),
                                       (lds_void*)(dst + r0 * D), 16, 0, 0);
    }
  };
  zero_acc();
  // (k, zb: cluster and sub-label of row tid of the tile being grouped, loaded a
  // tile ahead and first used after the barrier that lands them)
  int k = -1;
  unsigned char zb = 0;
  if (nt > 0) {
    if (tid < tile_rows(0)) nperm[0][tid] = perm[r_begin + tid];
    for (int c = tid; c < D; c += BIG_THREADS) {
      xa[R * D + c] = 0.0f;
      xb[R * D + c] = 0.0f;
    }
    __syncthreads();
    const int r = tid < tile_rows(0) ? tid : 0;
    const int mi = nperm[0][r];
    k = zrow ? zrow[r_begin + r] : z[mi];
    zb = zsub[mi];
    issue_rows(0, xa);
    if (nt > 1 && tid < tile_rows(1)) nperm[1][tid] = perm[r_begin + R + tid];
  }
  // one tile; its rows in xa (B = 0) or xb (B = 1), the next tile's DMA into the other
  auto tile_step = [&](auto bsel, auto wqc, int lt) __attribute__((always_inline)) {
    constexpr int B = decltype(bsel)::value;
    constexpr int WQ = decltype(wqc)::value;
    const float* tx = B ? xb : xa;
    float* nx = B ? xa : xb;
    const int rows = tile_rows(lt);
    const bool valid = tid < rows;
    // tile lt's rows and metadata have landed (the barrier waits for every memory
    // operation), the previous tile's LDS reads are done, nperm[(lt + 1) % 2] is visible
    __syncthreads();
    const int zs = zb ? 1 : 0;
    if (valid) rk[tid] = k;
    for (int q = tid; q < 2 * R; q += BIG_THREADS) lcount[q] = 0;
    __syncthreads();
    // ---- (2) group rows by segment: run of the cluster (rows are sorted by
    // z), then sub-label.  One scan gives the run of each row (high half) and
    // the right rows up to it (low half; both counts are <= R)
    const int zsv = valid ? zs : 0;
    const int flag = (valid && (tid == 0 || rk[tid] != rk[tid - 1])) ? 1 : 0;
    const int sc = block_inclusive_scan_big((flag << 16) | zsv, buf);
    const int run = (sc >> 16) - 1, ones_ex = (sc & 0xFFFF) - zsv;
    const int nruns = __builtin_amdgcn_readfirstlane(buf[BIG_THREADS - 1] >> 16);
    if (flag) {
      rstart[run] = tid;
      ostart[run] = ones_ex;
      rcl[run] = k;
    }
    const int lid = 2 * run + zsv;
    if (valid) atomicAdd(&lcount[lid], 1);  // integer counts: exact in any order
    __syncthreads();
    if (tid == 0) {
      int a = 0;
      for (int q = 0; q < 2 * nruns; ++q) {
        lstart[q] = a;
        a += lcount[q];
      }
    }
    __syncthreads();
    if (valid) {
      // rank among the run's rows of the same sub-label, in sorted order
      const int ones_run = ones_ex - ostart[run];
      const int rank = zsv ? ones_run : (tid - rstart[run]) - ones_run;
      order[lstart[lid] + rank] = tid;
    }
    __syncthreads();
    // ---- (1) the next tile: metadata into registers, the indices of the tile
    // after it, and its rows by DMA (the registers' first use is after the next
    // barrier, so nothing here waits for the DMA)
    int pn = -1;
    if (lt + 1 < nt) {
      const int r = tid < tile_rows(lt + 1) ? tid : 0;
      const int mi = nperm[(lt + 1) & 1][r];
      k = zrow ? zrow[(tb + lt + 1) * R + r] : z[mi];
      zb = zsub[mi];
      if (lt + 2 < nt) pn = perm[(tb + lt + 2) * R + (tid < tile_rows(lt + 2) ? tid : 0)];
      issue_rows(lt + 1, nx);
    }
    // ---- (3) every run, in order; this wave's side of it
    for (int j = 0; j < nruns; ++j) {
      const int kq = __builtin_amdgcn_readfirstlane(rcl[j]);
      if (kq != cur_k) {
        flush();
        zero_acc();
        if (cur_k < 0) k_first = kq;
        cur_k = kq;
      }
      const int q = 2 * j + side;
      const int cnt = __builtin_amdgcn_readfirstlane(lcount[q]);
      if (cnt == 0) continue;
      cnt_seg += cnt;
      const int st = __builtin_amdgcn_readfirstlane(lstart[q]);
      big_rows<D, WQ, R>(acc, sx, tx, order, st, cnt, lane, rd0, rd1);
    }
    // nperm[lt % 2] was last read before this tile's first barrier
    if (pn >= 0 && tid < R) nperm[lt & 1][tid] = pn;
  };
  // the tile loop once per quarter (a compile-time constant, so that its
  // blocks' operands are plain registers and the accumulators stay in place)
  auto run = [&](auto wqc) __attribute__((always_inline)) {
    for (int lt = 0; lt < nt; lt += 2) {
      tile_step(std::integral_constant<int, 0>{}, wqc, lt);
      if (lt + 1 < nt) tile_step(std::integral_constant<int, 1>{}, wqc, lt + 1);
    }
  };
  switch (wq) {
    case 0:
      run(std::integral_constant<int, 0>{});
      break;
    case 1:
      run(std::integral_constant<int, 1>{});
      break;
    case 2:
      run(std::integral_constant<int, 2>{});
      break;
    default:
      run(std::integral_constant<int, 3>{});
  }
  flush();
}

// workgroups of the generic statistics kernel: about four per CU, fewer
// above d = 64 (each range's partial slots hold 2 (1 + E) doubles per side)
long long generic_groups(int d, long long n) {
  const int TR = tile_rows(d);
  const long long tiles = (n + TR - 1) / TR;
  const long long cap = d <= 64 ? 1024 : 256;
  const long long g = tiles < cap ? tiles : cap;
  const long long tpw = g > 0 ? (tiles + g - 1) / g : 1;
  return tiles > 0 ? (tiles + tpw - 1) / tpw : 0;
}

template <bool SAMPLE>
hipError_t launch_sub_stats_t(int d, const float* x, long long n, const int* perm, const int* z, unsigned char* zsub,
                              const float* packed, int K, int k_max, uint32_t t, uint64_t seed, long long* counts,
                              double* moments, const int* cstart, const int* ctot, int kbase, int ncl, double* part,
                              hipStream_t s) {
  const int TR = tile_rows(d);
  static bool attr_set = false;
  if (!attr_set) {  // above d = 64 the per-lane centred columns take more than 64 KB
    hipError_t e = hipFuncSetAttribute((const void*)k_sub_stats<0, SAMPLE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  // contiguous tile ranges
  const long long tiles = (n + TR - 1) / TR;
  const long long g = generic_groups(d, n);
  const int tpw = (int)((tiles + g - 1) / g);
  const unsigned grid = (unsigned)((tiles + tpw - 1) / tpw);
#define DPMM_SUB_CASE(DD)                                                                                 \
  case DD:                                                                                                \
    hipLaunchKernelGGL((k_sub_stats<DD, SAMPLE>), dim3(grid), dim3(BLOCK), sub_stats_lds(d, TR, false), s, x, d, \
                       TR, tpw, n, perm, z, zsub, packed, K, k_max, t, seed, counts, moments, cstart, ctot, kbase,\
                       part);                                                                             \
    break;
  switch (d) {
    DPMM_SUB_CASE(8)
    DPMM_SUB_CASE(16)
    DPMM_SUB_CASE(32)
    DPMM_SUB_CASE(64)
    default:
      hipLaunchKernelGGL((k_sub_stats<0, SAMPLE>), dim3(grid), dim3(BLOCK), sub_stats_lds(d, TR, SAMPLE), s, x, d,
                         TR, tpw, n, perm, z, zsub, packed, K, k_max, t, seed, counts, moments, cstart, ctot, kbase,
                         part);
  }
#undef DPMM_SUB_CASE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !part) return e;
  const int E = d + d * (d + 1) / 2;
  hipLaunchKernelGGL(k_sub_stats_fix, dim3((2 * (E + 1) + FIX_EN - 1) / FIX_EN, ncl), dim3(FIX_PH * FIX_EN),
                     0, s, E, (long long)tpw * TR, cstart, ctot, part, counts, moments, kbase);
  return hipGetLastError();
}

}  // namespace

hipError_t sorted_plan(long long n, int K, long long hist_cap, int* G, long long* per_block) {
  const SortedPlan p = plan_blocks(n, K, hist_cap);
  *G = p.G;
  *per_block = p.per_block;
  return hipSuccess;
}

hipError_t launch_sort_by_z(const int* z, long long n, int K, int G, long long per_block, bool have_hist, int* hist,
                            int* tot, int* offs, int* perm, int* zsort, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipError_t e;
  if (!have_hist) {
    e = launch_zero64(tot, (size_t)(K + 1) / 2 + 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hist_z, dim3(G), dim3(BLOCK), (size_t)K * sizeof(int), s, z, n, per_block, K, hist, tot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_scan_hist, dim3(K), dim3(BLOCK), 0, s, hist, G, K, tot, offs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // per_block is a multiple of BLOCK: each wave's quarter is whole 64-row chunks
  if (per_block % BLOCK != 0 || 4 * (size_t)K * sizeof(int) > 64 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scatter_z, dim3(G), dim3(BLOCK), 4 * (size_t)K * sizeof(int), s, z, n, per_block, K, offs, perm,
                     zsort);
  return hipGetLastError();
}

namespace {

// rows per wave of k_sub_stats_w (whole 64-row chunks, at most SUBW_WAVES waves)
long long subw_rpw(long long n) {
  long long rpw = (n + SUBW_WAVES - 1) / SUBW_WAVES;
  return ((rpw + 63) / 64) * 64;
}

// tiles per workgroup of k_sub_stats_big (at most 512 workgroups at d = 64, 256 at d = 128)
int big_tpb(int d, long long n) {
  const long long tiles = (n + big_rows_of(d) - 1) / big_rows_of(d);
  const long long gmax = d == 128 ? 256 : 512;
  const long long g = tiles < gmax ? tiles : gmax;
  return g > 0 ? (int)((tiles + g - 1) / g) : 1;
}

// The statistics kernels over rows perm[0, n) (point indices below npts).
// Slot mode (part != nullptr): cstart / ctot give the sorted start and size
// of clusters kbase ... kbase + ncl - 1 (indexed from 0), every one of their
// entries is written and nothing is added with atomics; otherwise the kernels
// add into counts / moments (which the caller has zeroed).
hipError_t sub_stats_kernels(int d, bool sample, const float* x, long long npts, long long n, const int* perm,
                             const int* z, const int* zrow, unsigned char* zsub, const float* packed, int K, int k_max,
                             uint32_t t, uint64_t seed, long long* counts, double* moments, const int* cstart,
                             const int* ctot, int kbase, int ncl, double* part, hipStream_t s,
                             const SubX3* x3 = nullptr) {
  hipError_t e;
  if (n == 0) return hipSuccess;
  const int E = d + d * (d + 1) / 2;
  const dim3 fix_grid((2 * (E + 1) + FIX_EN - 1) / FIX_EN, ncl);
  if (sample && (d == 32 || d == 64 || d == 128)) {
    // the sub-labels in their own pass on the FP32 matrix cores, then the statistics; at
    // d = 128 two workgroups per CU (the staged records take 66 KB), each on a contiguous
    // range of rows
    {
      static bool lattr = false;
      const size_t llds = sub_labels_mfma_lds(d);
      if (!lattr) {
        e = hipFuncSetAttribute((const void*)k_sub_labels_mfma<128>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sub_labels_mfma_lds(128));
        if (e != hipSuccess) return e;
        lattr = true;
      }
      // d = 32: three waves per SIMD, all workgroups resident at once; each workgroup takes
      // a range of whole waves' rows (64), so that the ranges differ by at most one wave
      const long long cap = d == 128 ? 512 : (d == 64 ? 1024 : 768);
      long long lper = (n + cap - 1) / cap;
      lper = ((lper + 63) / 64) * 64;
      const unsigned lg = (unsigned)((n + lper - 1) / lper);
      // with BF16 tables (d = 64, 128) a bf16x3 pass draws most rows first and this
      // kernel only the list it leaves
      const int* lperm = perm;
      const int* lz = z;
      const int* lzrow = zrow;
      const int* ndev = nullptr;
      if (x3 && (d == 64 || d == 128)) {
        e = launch_sub_labels_x3(d, x, n, perm, z, zrow, zsub, packed, K, k_max, t, seed, *x3, s);
        if (e != hipSuccess) return e;
        lperm = x3->perm_c;
        lz = nullptr;
        lzrow = x3->zrow_c;
        ndev = x3->offs + SUBX_GROUPS;
      }
      if (d == 128)
        hipLaunchKernelGGL(k_sub_labels_mfma<128>, dim3(lg), dim3(SUBL_BLOCK), llds, s, x, n, lper, lperm, lz, lzrow,
                           zsub, packed, K, k_max, t, seed, ndev);
      else if (d == 64)
        hipLaunchKernelGGL(k_sub_labels_mfma<64>, dim3(lg), dim3(SUBL_BLOCK), llds, s, x, n, lper, lperm, lz, lzrow,
                           zsub, packed, K, k_max, t, seed, ndev);
      else
        hipLaunchKernelGGL(k_sub_labels_mfma<32>, dim3(lg), dim3(SUBL_BLOCK), llds, s, x, n, lper, lperm, lz, lzrow,
                           zsub, packed, K, k_max, t, seed, ndev);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    sample = false;
  }
  if (d == 64 || d == 128) {
    const int R = big_rows_of(d);
    const long long tiles = (n + R - 1) / R;
    const int tpb = big_tpb(d, n);
    const unsigned grid = (unsigned)((tiles + tpb - 1) / tpb);
    const size_t lds = 0;  // all of its LDS is static (two tiles' rows, 129 KB)
    if (d == 64)
      hipLaunchKernelGGL(k_sub_stats_big<64>, dim3(grid), dim3(BIG_THREADS), lds, s, x, n, tpb, perm, z, zrow, zsub,
                         counts, moments, cstart, ctot, kbase, part);
    else
      hipLaunchKernelGGL(k_sub_stats_big<128>, dim3(grid), dim3(BIG_THREADS), lds, s, x, n, tpb, perm, z, zrow, zsub,
                         counts, moments, cstart, ctot, kbase, part);
    if ((e = hipGetLastError()) != hipSuccess || !part) return e;
    hipLaunchKernelGGL(k_sub_stats_fix, fix_grid, dim3(FIX_PH * FIX_EN), 0, s, E, (long long)tpb * R, cstart,
                       ctot, part, counts, moments, kbase);
    return hipGetLastError();
  }
  if (d == 8 || d == 16 || d == 32) {
    // about eight waves per CU, each on a contiguous range of whole 64-row chunks
    const long long rpw = subw_rpw(n);
    const long long nw = (n + rpw - 1) / rpw;
    const unsigned grid = (unsigned)((nw + 3) / 4);
    const size_t lds = (size_t)4 * 64 * (d + 1) * sizeof(float);
#define DPMM_SUBW_CASE(DD)                                                                                      \
  case DD:                                                                                                      \
    if (sample)                                                                                                 \
      hipLaunchKernelGGL((k_sub_stats_w<DD, true>), dim3(grid), dim3(BLOCK), lds, s, x, npts, n, rpw, perm, z,  \
                         zrow, zsub, packed, K, k_max, t, seed, counts, moments, cstart, ctot, kbase, part);    \
    else                                                                                                        \
      hipLaunchKernelGGL((k_sub_stats_w<DD, false>), dim3(grid), dim3(BLOCK), lds, s, x, npts, n, rpw, perm, z, \
                         zrow, zsub, packed, K, k_max, t, seed, counts, moments, cstart, ctot, kbase, part);    \
    break;
    switch (d) {
      DPMM_SUBW_CASE(8)
      DPMM_SUBW_CASE(16)
      DPMM_SUBW_CASE(32)
    }
#undef DPMM_SUBW_CASE
    if ((e = hipGetLastError()) != hipSuccess || !part) return e;
    hipLaunchKernelGGL(k_sub_stats_fix, fix_grid, dim3(FIX_PH * FIX_EN), 0, s, E, rpw, cstart, ctot, part, counts,
                       moments, kbase);
    return hipGetLastError();
  }
  return sample ? launch_sub_stats_t<true>(d, x, n, perm, z, zsub, packed, K, k_max, t, seed, counts, moments,
                                           cstart, ctot, kbase, ncl, part, s)
                : launch_sub_stats_t<false>(d, x, n, perm, z, zsub, packed, K, k_max, t, seed, counts, moments,
                                            cstart, ctot, kbase, ncl, part, s);
}

}  // namespace

size_t sub_stats_part_doubles(int d, long long n) {
  const int E = d + d * (d + 1) / 2;
  long long ranges;
  if (n <= 0) return 0;
  if (d == 8 || d == 16 || d == 32) {
    const long long rpw = subw_rpw(n);
    ranges = (n + rpw - 1) / rpw;
  } else if (d == 64 || d == 128) {
    const long long tiles = (n + big_rows_of(d) - 1) / big_rows_of(d);
    const int tpb = big_tpb(d, n);
    ranges = (tiles + tpb - 1) / tpb;
  } else {
    ranges = generic_groups(d, n);
  }
  return (size_t)2 * ranges * 2 * (E + 1);
}

size_t sub_stats_part_doubles_max(int d) {
  const int E = d + d * (d + 1) / 2;
  long long ranges;
  if (d == 8 || d == 16 || d == 32)
    ranges = SUBW_WAVES;
  else if (d == 64 || d == 128)
    ranges = d == 128 ? 256 : 512;
  else
    ranges = d <= 64 ? 1024 : 256;
  return (size_t)2 * ranges * 2 * (E + 1);
}

hipError_t launch_sub_stats(int d, bool sample, const float* x, long long n, const int* perm, const int* z,
                            const int* zrow, unsigned char* zsub, const float* packed, int K, int k_max, uint32_t t,
                            uint64_t seed, long long* counts, double* moments, const int* cstart, const int* ctot,
                            double* part, hipStream_t s, const SubX3* x3) {
  const int E = d + d * (d + 1) / 2;
  if (n > 0 && part)  // slot mode: every cluster's entries are written, no zeroing
    return sub_stats_kernels(d, sample, x, n, n, perm, z, zrow, zsub, packed, K, k_max, t, seed, counts, moments,
                             cstart, ctot, 0, K, part, s, x3);
  hipError_t e = launch_zero64(counts, (size_t)2 * K, s);
  if (e != hipSuccess) return e;
  e = launch_zero64(moments, (size_t)2 * K * E, s);
  if (e != hipSuccess) return e;
  return sub_stats_kernels(d, sample, x, n, n, perm, z, zrow, zsub, packed, K, k_max, t, seed, counts, moments,
                           nullptr, nullptr, 0, K, nullptr, s, x3);
}

bool partition_stats_supported(int d) { return d == 8 || d == 16 || d == 32 || d == 64 || d == 128; }

// The listed points idx[0, nsel) all belong to cluster k1; side[i] in {0, 1}
// plays the sub-label, so the sorted-order kernels leave the statistics of
// side h in segment 2 k1 + h of the arrays they are given.  Shifting the base
// pointers by slot - 2 k1 segments puts them in counts[slot + h] and
// moments[(slot + h) E] and touches nothing else.  cspan: device int[2] =
// {0, nsel} (the one cluster's sorted start and size); part: partial slots
// (sub_stats_part_doubles(d, nsel) doubles), summed in a fixed order.
hipError_t launch_partition_stats(int d, const float* x, long long npts, const int* idx, long long nsel,
                                  const int* z, int k1, int K, const unsigned char* side, int slot,
                                  long long* counts, double* moments, const int* cspan, double* part, hipStream_t s) {
  if (!partition_stats_supported(d) || k1 < 0 || k1 >= K || slot < 2 * k1 || !cspan || !part)
    return hipErrorInvalidValue;
  const int E = d + d * (d + 1) / 2;
  const long long shift = (long long)slot - 2 * k1;
  if (nsel == 0) {
    hipError_t e = launch_zero64(counts + slot, 2, s);
    if (e != hipSuccess) return e;
    return launch_zero64(moments + (size_t)slot * E, (size_t)2 * E, s);
  }
  return sub_stats_kernels(d, false, x, npts, nsel, idx, z, nullptr, const_cast<unsigned char*>(side), nullptr, K, 0,
                           0, 0, counts + shift, moments + shift * E, cspan, cspan + 1, k1, 1, part, s);
}

}  // namespace dpmm
