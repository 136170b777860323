// Selection of the k lowest K2 (paper: the solution is the combination with
// the lowest K2, end of the Problem Formulation section; GPU approaches
// section: each thread keeps its best, the host picks the final one).
//
// Here, for k >= 1 and exactly:
//   1. radix select over the FP32 score plane finds the k-th smallest FP32
//      value T32 (3 passes of 2048 bins over a window that starts at the
//      plane's key range); after the first pass, every score up to the end
//      of the bin holding the k-th value plus 2 e(N) is compacted into a
//      short list, and the later passes and the candidate collection read
//      that list instead of the plane (the plane again if the list
//      overflows its capacity).  For large planes the first bound comes
//      instead from the same radix select run on a sample (every 32nd block
//      of 1024 scores): the sample's k-th smallest value is at least T32
//      (its k smallest are k scores of the plane), so compacting every score
//      up to it plus 2 e(N) takes one pass over the plane instead of two;
//   2. every triplet with K2_fp32 <= T32 + 2 e(N) is a candidate, where e(N)
//      bounds |K2_fp32 - K2_fp64| for any table of N samples, so the candidate
//      set contains every member of the FP64 top-k;
//   3. each candidate's table is recounted and K2 re-evaluated in FP64 with
//      Eq. 1's bracketing, rows summed in row order;
//   4. each candidate's position under (K2_fp64, i, j, k) is counted against
//      all others and the first k are written out.
#include <algorithm>

#include "epi3_internal.h"

namespace epi3 {

// ---------------------------------------------------------------- init ----
__global__ void init_select_kernel(SelJob *sj, int n) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  SelState *st = sj[x].st;
  st->kmin = 0xffffffffu;
  st->kmax = 0u;
  st->lo = 0u;
  st->shift = 0;
  st->krem = 0;
  st->done = 0u;
  st->kth = 0u;
  st->thr = 0.f;
  st->overflow = 0u;
  st->ncand = 0ull;
  st->whi = 0u;
  st->ub = 0.f;
  st->cmode = 0u;
  st->cn = 0ull;
  st->T = sj[x].T;
  st->k = sj[x].k;
  st->keff = sj[x].k < sj[x].T ? sj[x].k : sj[x].T;
  for (int b = 0; b < kHistBins; ++b) sj[x].hist[b] = 0u;
}

// After the count kernel: first window = [kmin, kmax].
__global__ void window_kernel(SelJob *sj, int n) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  SelState *st = sj[x].st;
  if (st->keff <= 0) {
    st->done = 2u;  // nothing to select
    return;
  }
  if (!sj[x].score && !(st->cmode == 1u && st->cn <= (unsigned long long)sj[x].ccap)) {
    // no plane to fall back on: the bounded list overflowed (reported as a
    // capacity error; every later kernel skips the job)
    st->done = 3u;
    return;
  }
  const uint32_t range = st->kmax - st->kmin;
  st->lo = st->kmin;
  st->krem = (uint64_t)st->keff;
  if (range == 0u) {
    st->done = 1u;
    st->kth = st->kmin;
    return;
  }
  const int bl = 32 - __builtin_clz(range);  // bits of range
  st->shift = bl > 11 ? bl - 11 : 0;
}

// True when the compacted list holds every key the remaining passes need.
__device__ __forceinline__ bool use_compact(const SelState *st, const SelJob &J) {
  return st->cmode == 1u && st->cn <= (unsigned long long)J.ccap;
}

// Plane index of element e of the sample (every kSampleStride-th block).
__device__ __forceinline__ int64_t sample_at(int64_t e) {
  return (e / kSampleBlock) * kSampleBlock * kSampleStride + e % kSampleBlock;
}
// Elements of the sample of a plane of T scores (the last block may be short).
__host__ __device__ __forceinline__ int64_t sample_len(int64_t T) {
  const int64_t nb = (T + kSampleBlock - 1) / kSampleBlock;          // blocks of the plane
  const int64_t ns = (nb + kSampleStride - 1) / kSampleStride;      // sampled blocks
  const int64_t last = (ns - 1) * kSampleStride;                    // index of the last one
  return ns <= 0 ? 0 : (ns - 1) * kSampleBlock + (T - last * kSampleBlock < kSampleBlock
                                                       ? T - last * kSampleBlock
                                                       : kSampleBlock);
}

// sampled: histogram of the sample of sampling jobs (other jobs skip).
__global__ void __launch_bounds__(256) hist_kernel(const SelJob *__restrict__ sj, int sampled) {
  const SelJob &J = sj[blockIdx.y];
  const SelState *st = J.st;
  if (st->done || (sampled && !J.sample)) return;
  const uint32_t lo = st->lo;
  const int shift = st->shift;
  __shared__ uint32_t h[kHistBins];
  for (int b = threadIdx.x; b < kHistBins; b += blockDim.x) h[b] = 0u;
  __syncthreads();
  const bool compact = !sampled && use_compact(st, J);
  const float *score = J.score;
  const int64_t n = sampled ? sample_len(J.T) : compact ? (int64_t)st->cn : J.T;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t key = compact ? J.ckey[x] : f2key(score[sampled ? sample_at(x) : x]);
    if (key >= lo) {
      const uint32_t d = (key - lo) >> shift;
      if (d < (uint32_t)kHistBins) atomicAdd(&h[d], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kHistBins; b += blockDim.x)
    if (h[b]) atomicAdd(&J.hist[b], h[b]);
}

// One block per job: find the bin holding the krem-th key, narrow the window.
// sampled: only the sampling jobs (their sample's krem-th key).
__global__ void __launch_bounds__(1024) find_kernel(SelJob *sj, int sampled) {
  SelJob &J = sj[blockIdx.x];
  SelState *st = J.st;
  if (st->done || (sampled && !J.sample)) return;
  __shared__ unsigned long long cum[kHistBins];
  const int t = threadIdx.x;
  // every thread reads the state before any thread updates it (barriers below)
  const uint64_t krem = st->krem;
  const int shift = st->shift;
  const uint32_t lo0 = st->lo;
  for (int b = t; b < kHistBins; b += blockDim.x) cum[b] = J.hist[b];
  __syncthreads();
  for (int off = 1; off < kHistBins; off <<= 1) {
    unsigned long long v0 = 0, v1 = 0;
    const int b0 = t, b1 = t + 1024;
    if (b0 >= off) v0 = cum[b0 - off];
    if (b1 >= off) v1 = cum[b1 - off];
    __syncthreads();
    cum[b0] += v0;
    cum[b1] += v1;
    __syncthreads();
  }
  for (int b = t; b < kHistBins; b += blockDim.x) {
    const unsigned long long before = b ? cum[b - 1] : 0ull;
    if (before < krem && cum[b] >= krem) {  // exactly one bin satisfies this
      const uint32_t lo = lo0 + ((uint32_t)b << shift);
      const uint32_t w = (1u << shift) - 1u;
      st->lo = lo;
      st->whi = lo > 0xffffffffu - w ? 0xffffffffu : lo + w;
      st->krem = krem - before;
      if (shift == 0) {
        st->done = 1u;
        st->kth = lo;
      } else {
        st->shift = shift > 11 ? shift - 11 : 0;
      }
    }
  }
  __syncthreads();
  for (int b = t; b < kHistBins; b += blockDim.x) J.hist[b] = 0u;
}

// Threshold T32 + 2 e(N), rounded up to the next float.
__global__ void threshold_kernel(SelJob *sj, int n) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  SelState *st = sj[x].st;
  if (st->done != 1u) return;
  const double thr = (double)key2f(st->kth) + sj[x].err2;
  float f = (float)thr;
  if ((double)f < thr) f = __uint_as_float(__float_as_uint(f) + 1u);  // f >= 0: next float up
  st->thr = f;
}

// After the sample's select (sampling jobs: whi = the sample's k-th key):
// the plane's window restarts at its key range with the exact rank k.
__global__ void bound_kernel(SelJob *sj, int n) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n || !sj[x].sample) return;
  SelState *st = sj[x].st;
  if (st->done != 1u) return;  // nothing to select
  const uint32_t ub = st->kth;
  st->lo = st->kmin;
  st->whi = ub;
  st->krem = (uint64_t)st->keff;
  const uint32_t range = ub - st->kmin;
  if (range == 0u) {  // at least k scores equal the minimum
    st->kth = st->kmin;
    return;
  }
  st->done = 0u;
  const int bl = 32 - __builtin_clz(range);
  st->shift = bl > 11 ? bl - 11 : 0;
}

// Every score <= (last key of the window) + 2 e(N) goes to the compacted list
// (key, rank): after the first pass (post), or right after the sample's
// bound (pre, sampling jobs).  That bound is at least the final threshold, so
// the list holds every key the later passes and the candidate collection
// look at.
__global__ void __launch_bounds__(256) compact_kernel(const SelJob *__restrict__ sj, int pre) {
  const SelJob &J = sj[blockIdx.y];
  SelState *st = J.st;
  if (st->done || (pre ? !J.sample : J.sample)) return;
  const double ubd = (double)key2f(st->whi) + J.err2;
  float ub = (float)ubd;
  if ((double)ub < ubd) ub = __uint_as_float(__float_as_uint(ub) + 1u);  // ub >= 0: next float up
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->ub = ub;
    st->cmode = 1u;
  }
  const float *score = J.score;
  const int64_t T = J.T, ccap = J.ccap;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // appends the wave's scores with pred set (wave-uniform call)
  auto emit = [&](bool pred, float v, int64_t x) {
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return;
    unsigned long long pos0 = 0;
    if (lane == 0) pos0 = atomicAdd(&st->cn, (unsigned long long)__popcll(m));
    pos0 = __shfl(pos0, 0);
    const unsigned long long pos = pos0 + __popcll(m & ((1ull << lane) - 1ull));
    if (pred && (int64_t)pos < ccap) {
      J.ckey[pos] = f2key(v);
      J.crank[pos] = x;
    }
  };
  int64_t done = 0;
  if ((reinterpret_cast<uintptr_t>(score) & 15u) == 0) {
    // 16-byte loads: four scores per lane and step; nearly every step holds
    // no candidate, so one ballot decides
    const int64_t T4 = T >> 2;
    const float4 *s4 = reinterpret_cast<const float4 *>(score);
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63); base < T4;
         base += stride) {
      const int64_t x4 = base + lane;
      const bool in = x4 < T4;
      const float4 v = in ? s4[x4] : make_float4(0.f, 0.f, 0.f, 0.f);
      const bool any = in && (v.x <= ub || v.y <= ub || v.z <= ub || v.w <= ub);
      if (__ballot(any) == 0ull) continue;
      emit(in && v.x <= ub, v.x, 4 * x4);
      emit(in && v.y <= ub, v.y, 4 * x4 + 1);
      emit(in && v.z <= ub, v.z, 4 * x4 + 2);
      emit(in && v.w <= ub, v.w, 4 * x4 + 3);
    }
    done = T4 << 2;
  }
  for (int64_t base = done + blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63); base < T;
       base += stride) {
    const int64_t x = base + lane;
    const float v = x < T ? score[x] : 0.f;
    emit(x < T && v <= ub, v, x);
  }
}

__global__ void __launch_bounds__(256) collect_kernel(const SelJob *__restrict__ sj) {
  const SelJob &J = sj[blockIdx.y];
  SelState *st = J.st;
  if (st->done != 1u) return;
  const float thr = st->thr;
  const bool compact = use_compact(st, J);
  const float *score = J.score;
  const int64_t n = compact ? (int64_t)st->cn : J.T, cap = J.cap;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63); base < n;
       base += stride) {
    const int64_t x = base + lane;
    const bool pred = x < n && (compact ? key2f(J.ckey[x]) : score[x]) <= thr;
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) continue;
    unsigned long long pos0 = 0;
    if (lane == 0) pos0 = atomicAdd(&st->ncand, (unsigned long long)__popcll(m));
    pos0 = __shfl(pos0, 0);
    const unsigned long long pos = pos0 + __popcll(m & ((1ull << lane) - 1ull));
    if (pred && (int64_t)pos < cap) {
      J.cand[pos] = compact ? J.crank[x] : x;
      J.candkey[pos] = compact ? J.ckey[x] : f2key(score[x]);
    }
  }
}

// ----------------------------------------------------- FP64 re-score ----
__device__ __forceinline__ unsigned wave_sum(unsigned v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Corner cells n[4a + 2b + c] over words [w0, w1) by the lanes of one wave,
// optionally restricted to mask bits.
__device__ __forceinline__ void corners(const uint32_t *planes, int64_t Mp, int w0, int w1, int i,
                                        int j, int k, const uint32_t *mask, uint32_t n[8]) {
  const int lane = threadIdx.x & 63;
  uint32_t a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int w = w0 + lane; w < w1; w += 64) {
    const uint2 *row = reinterpret_cast<const uint2 *>(planes) + (int64_t)w * Mp;
    const uint2 xi = row[i], xj = row[j], xk = row[k];
    const uint32_t mk = mask ? mask[w] : 0xffffffffu;
    const uint32_t xiv[2] = {xi.x & mk, xi.y & mk}, xjv[2] = {xj.x, xj.y}, xkv[2] = {xk.x, xk.y};
#pragma unroll
    for (int p = 0; p < 8; ++p)
      a[p] += __builtin_popcount(xiv[p >> 2] & xjv[(p >> 1) & 1] & xkv[p & 1]);
  }
#pragma unroll
  for (int p = 0; p < 8; ++p) n[p] = wave_sum(a[p]);
}

__device__ __forceinline__ void pair_args(const int32_t *pairs, int64_t Mp, int i, int j, int k,
                                          int aij[4], int aik[4], int ajk[4], int mi[2], int mj[2],
                                          int mk[2], int64_t st = 1) {
  const int4 *pr = reinterpret_cast<const int4 *>(pairs);
  const int4 pij = pr[((int64_t)i * Mp + j) * st], pik = pr[((int64_t)i * Mp + k) * st],
             pjk = pr[((int64_t)j * Mp + k) * st];
  const int4 ii = pr[((int64_t)i * Mp + i) * st], jj = pr[((int64_t)j * Mp + j) * st],
             kk = pr[((int64_t)k * Mp + k) * st];
  aij[0] = pij.x; aij[1] = pij.y; aij[2] = pij.z; aij[3] = pij.w;
  aik[0] = pik.x; aik[1] = pik.y; aik[2] = pik.z; aik[3] = pik.w;
  ajk[0] = pjk.x; ajk[1] = pjk.y; ajk[2] = pjk.z; ajk[3] = pjk.w;
  mi[0] = ii.x; mi[1] = ii.w; mj[0] = jj.x; mj[1] = jj.w; mk[0] = kk.x; mk[1] = kk.w;
}

// Full table [2][27] of one triplet, computed by the lanes of one wave.
// SPLIT: class words [0, W0) and [W0, W0 + W1), pairs [2][Mp][Mp].
// MASKED: totals from all words and pairs[0]; cases with the mask and
// case_pairs; controls = totals - cases.
__device__ void triplet_table(const uint32_t *planes, const int32_t *pairs,
                              const int32_t *case_pairs, int64_t case_stride,
                              const uint32_t *mask, int layout, int64_t Mp, int W0, int W1,
                              int N0, int N1, int i, int j, int k, int tab[2][27]) {
  int aij[4], aik[4], ajk[4], mi[2], mj[2], mk[2];
  uint32_t n[8];
  if (layout == EPI3_LAYOUT_SPLIT) {
    for (int c = 0; c < 2; ++c) {
      corners(planes, Mp, c ? W0 : 0, c ? W0 + W1 : W0, i, j, k, nullptr, n);
      pair_args(pairs + (int64_t)c * Mp * Mp * 4, Mp, i, j, k, aij, aik, ajk, mi, mj, mk);
      complete_table(n, aij, aik, ajk, mi, mj, mk, c ? N1 : N0, tab[c]);
    }
  } else {
    int tot[27];
    corners(planes, Mp, 0, W0, i, j, k, nullptr, n);
    pair_args(pairs, Mp, i, j, k, aij, aik, ajk, mi, mj, mk);
    complete_table(n, aij, aik, ajk, mi, mj, mk, N0 + N1, tot);
    corners(planes, Mp, 0, W0, i, j, k, mask, n);
    // case pair tables: two 16-bit counts per word
    {
      const uint2 *cp = reinterpret_cast<const uint2 *>(case_pairs);
      auto unpack = [&](int x, int y, int v[4]) {
        const uint2 w = cp[((int64_t)x * Mp + y) * case_stride];
        v[0] = (int)(w.x & 0xffffu); v[1] = (int)(w.x >> 16);
        v[2] = (int)(w.y & 0xffffu); v[3] = (int)(w.y >> 16);
      };
      int d[4];
      unpack(i, j, aij); unpack(i, k, aik); unpack(j, k, ajk);
      unpack(i, i, d); mi[0] = d[0]; mi[1] = d[3];
      unpack(j, j, d); mj[0] = d[0]; mj[1] = d[3];
      unpack(k, k, d); mk[0] = d[0]; mk[1] = d[3];
    }
    complete_table(n, aij, aik, ajk, mi, mj, mk, N1, tab[1]);
    for (int x = 0; x < 27; ++x) tab[0][x] = tot[x] - tab[1][x];
  }
}

// Pair (i, j) of lexicographic rank `rank` among the pairs of M SNPs.
__device__ __forceinline__ void decode_pair_rank(int64_t M, int64_t rank, int &i, int &j) {
  int lo = 0, hi = (int)M - 2;  // last i whose first rank <= rank
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pair_rank(M, mid, mid + 1) <= rank) lo = mid; else hi = mid - 1;
  }
  i = lo;
  j = (int)(rank - pair_rank(M, i, i + 1)) + i + 1;
}

// Both 9-row tables of the pair (i, j) of a SPLIT data set, recounted from
// the planes by the lanes of one wave: the four cells with genotypes in
// {0, 1} and the per-SNP counts, then the rest by pair_cells.
__device__ void pair_table(const uint32_t *planes, int64_t Mp, int W0, int W1, int N0, int N1,
                           int i, int j, int tab[2][27]) {
  const int lane = threadIdx.x & 63;
  for (int c = 0; c < 2; ++c) {
    const int w0 = c ? W0 : 0, w1 = c ? W0 + W1 : W0;
    uint32_t a[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // n[2a + b] (4), mi[a] (2), mj[b] (2)
    for (int w = w0 + lane; w < w1; w += 64) {
      const uint2 *row = reinterpret_cast<const uint2 *>(planes) + (int64_t)w * Mp;
      const uint2 xi = row[i], xj = row[j];
      a[0] += __builtin_popcount(xi.x & xj.x);
      a[1] += __builtin_popcount(xi.x & xj.y);
      a[2] += __builtin_popcount(xi.y & xj.x);
      a[3] += __builtin_popcount(xi.y & xj.y);
      a[4] += __builtin_popcount(xi.x);
      a[5] += __builtin_popcount(xi.y);
      a[6] += __builtin_popcount(xj.x);
      a[7] += __builtin_popcount(xj.y);
    }
    int v[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) v[p] = (int)wave_sum(a[p]);
    const int n[4] = {v[0], v[1], v[2], v[3]}, mi[2] = {v[4], v[5]}, mj[2] = {v[6], v[7]};
    pair_cells(n, mi, mj, c ? N1 : N0, tab[c]);
  }
}

// Eq. 1 in FP64: rows in order, each row L[r + 1] - (L[r_0] + L[r_1]).
__device__ __forceinline__ double k2_fp64_rows(const int tab[2][27], int rows, const double *L) {
  double k2 = 0.0;
  for (int x = 0; x < rows; ++x) {
    const int r0 = tab[0][x], r1 = tab[1][x];
    k2 += L[r0 + r1 + 1] - (L[r0] + L[r1]);
  }
  return k2;
}

// Eq. 1 in FP64: rows in order, each row L[r + 1] - (L[r_0] + L[r_1]).
__device__ __forceinline__ double k2_fp64(const int tab[2][27], const double *L) {
  double k2 = 0.0;
  for (int x = 0; x < 27; ++x) {
    const int r0 = tab[0][x], r1 = tab[1][x];
    k2 += L[r0 + r1 + 1] - (L[r0] + L[r1]);
  }
  return k2;
}

__global__ void __launch_bounds__(256) rescore_kernel(const SelJob *__restrict__ sj) {
  const SelJob &J = sj[blockIdx.y];
  SelState *st = J.st;
  if (st->done != 1u) return;
  const int64_t n = (int64_t)st->ncand < J.cap ? (int64_t)st->ncand : J.cap;
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t c = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); c < n;
       c += waves) {
    const int64_t rank = J.cand[c];
    int tab[2][27];
    if (J.order == 4) {
      int i, j, k, l;
      decode_quad_rank(J.M, rank, i, j, k, l);
      int q[2][81];
      const int64_t MpMp4 = (int64_t)J.Mp * J.Mp * 4;
      for (int cl = 0; cl < 2; ++cl) {
        uint32_t cnt[48];
        const int w0 = cl ? J.W0 : 0, w1 = cl ? J.W0 + J.W1 : J.W0;
        quad_counts(J.planes, J.Mp, w0 + lane, w1, 64, i, j, k, l, cnt);
        for (int x = 0; x < 48; ++x) cnt[x] = wave_sum(cnt[x]);
        quad_cells(cnt, J.pairs + cl * MpMp4, J.Mp, i, j, k, l, cl ? J.N1 : J.N0, q[cl]);
      }
      if (lane == 0) {
        CandRec &R = J.rec[c];
        double k2 = 0.0;  // Eq. 1 in FP64: rows in order
        for (int x = 0; x < 81; ++x) {
          const int r0 = q[0][x], r1 = q[1][x];
          k2 += J.lf64[r0 + r1 + 1] - (J.lf64[r0] + J.lf64[r1]);
        }
        R.key = (uint64_t)__double_as_longlong(k2);
        R.rank = rank;
        R.i = i; R.j = j; R.k = k; R.l = l;
        R.k2f = key2f(J.candkey[c]);
        R.k2 = k2;
        for (int x = 0; x < 81; ++x) {
          R.counts[x] = (uint32_t)q[0][x];
          R.counts[81 + x] = (uint32_t)q[1][x];
        }
      }
      continue;
    }
    if (J.order == 2) {
      int i, j;
      decode_pair_rank(J.M, rank, i, j);
      pair_table(J.planes, J.Mp, J.W0, J.W1, J.N0, J.N1, i, j, tab);
      if (lane == 0) {
        CandRec &R = J.rec[c];
        const double k2 = k2_fp64_rows(tab, 9, J.lf64);
        R.key = (uint64_t)__double_as_longlong(k2);
        R.rank = rank;
        R.i = i; R.j = j; R.k = 0;
        R.k2f = key2f(J.candkey[c]);
        R.k2 = k2;
        for (int x = 0; x < 9; ++x) {
          R.counts[x] = (uint32_t)tab[0][x];
          R.counts[27 + x] = (uint32_t)tab[1][x];
        }
      }
      continue;
    }
    int i, j, k;
    decode_rank(J.M, rank, i, j, k);
    int N0 = J.N0, N1 = J.N1;
    if (J.n1_dev) {
      N1 = *J.n1_dev;
      N0 = J.N0 + J.N1 - N1;
    }
    triplet_table(J.planes, J.pairs, J.case_pairs, J.case_stride, J.case_mask, J.layout, J.Mp,
                  J.W0, J.W1, N0, N1, i, j, k, tab);
    if (lane == 0) {
      CandRec &R = J.rec[c];
      const double k2 = k2_fp64(tab, J.lf64);
      R.key = (uint64_t)__double_as_longlong(k2);
      R.rank = rank;
      R.i = i; R.j = j; R.k = k;
      R.k2f = key2f(J.candkey[c]);
      R.k2 = k2;
      for (int x = 0; x < 27; ++x) {
        R.counts[x] = (uint32_t)tab[0][x];
        R.counts[27 + x] = (uint32_t)tab[1][x];
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (int64_t)st->ncand > J.cap) st->overflow = 1u;
}

// Position of each candidate under (key, rank); the first keff go out.
// Hit `pos` of the job's list from candidate record x.
__device__ __forceinline__ void emit_hit(const SelJob &J, int64_t x, int64_t pos) {
  const CandRec &R = J.rec[x];
  if (J.order == 4) {
    epi3_quad_hit &H = J.quad_hits[pos];
    H.i = R.i; H.j = R.j; H.k = R.k; H.l = R.l;
    H.k2_f32 = R.k2f;
    H.reserved = 0u;
    H.k2 = R.k2;
    for (int q = 0; q < 81; ++q) {
      H.counts[0][q] = R.counts[q];
      H.counts[1][q] = R.counts[81 + q];
    }
  } else if (J.order == 2) {
    epi3_pair_hit &H = J.pair_hits[pos];
    H.i = R.i; H.j = R.j;
    H.k2_f32 = R.k2f;
    H.reserved = 0u;
    H.k2 = R.k2;
    for (int q = 0; q < 9; ++q) {
      H.counts[0][q] = R.counts[q];
      H.counts[1][q] = R.counts[27 + q];
    }
  } else {
    epi3_hit &H = J.hits[pos];
    H.i = R.i; H.j = R.j; H.k = R.k;
    H.k2_f32 = R.k2f;
    H.k2 = R.k2;
    for (int q = 0; q < 27; ++q) {
      H.counts[0][q] = R.counts[q];
      H.counts[1][q] = R.counts[27 + q];
    }
  }
}

// Rank of every candidate = number of candidates before it under
// (K2_fp64, rank); each workgroup takes 64 candidates (one per lane) and its
// 16 waves split the comparisons, so chains stay short for a few thousand
// candidates.  Jobs with sort buffers (sortP > 0) are ordered by the sort
// kernels below instead.
constexpr int kRankThreads = 1024;
__global__ void __launch_bounds__(kRankThreads) rank_kernel(const SelJob *__restrict__ sj) {
  const SelJob &J = sj[blockIdx.y];
  SelState *st = J.st;
  if (st->done != 1u || J.sortP > 0) return;
  const int64_t n = (int64_t)st->ncand < J.cap ? (int64_t)st->ncand : J.cap;
  const int64_t keff = st->keff;
  __shared__ uint64_t skey[kRankThreads];
  __shared__ int64_t srank[kRankThreads];
  __shared__ int64_t spos[kRankThreads / 64][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t xb = blockIdx.x; xb * 64 < n; xb += gridDim.x) {
    const int64_t x = xb * 64 + lane;
    uint64_t mykey = ~0ull;
    int64_t myrank = 0;
    if (x < n) {
      mykey = J.rec[x].key;
      myrank = J.rec[x].rank;
    }
    int64_t part = 0;
    for (int64_t yb = 0; yb < n; yb += kRankThreads) {
      const int64_t y = yb + threadIdx.x;
      __syncthreads();
      skey[threadIdx.x] = y < n ? J.rec[y].key : ~0ull;
      srank[threadIdx.x] = y < n ? J.rec[y].rank : INT64_MAX;
      __syncthreads();
      // wave w compares with entries [64 w, 64 w + 64) of the chunk
      const int64_t left = n - yb - 64 * wave;
      const int lim = left < 0 ? 0 : (left < 64 ? (int)left : 64);
      for (int z = 64 * wave; z < 64 * wave + lim; ++z) {
        const uint64_t kz = skey[z];
        part += (kz < mykey) || (kz == mykey && srank[z] < myrank);
      }
    }
    spos[wave][lane] = part;
    __syncthreads();
    if (wave != 0) continue;
    int64_t pos = 0;
    for (int w = 0; w < kRankThreads / 64; ++w) pos += spos[w][lane];
    if (x < n && pos < keff) emit_hit(J, x, pos);
  }
}

// ---- ordering of large candidate sets: bitonic sort of (key, index) ----
// Entries past the candidate count carry key ~0 (above every FP64 key, which
// is the bit pattern of a non-negative double); equal keys of candidates are
// ordered by their lexicographic rank, equal padding keys by index.
__device__ __forceinline__ bool sort_before(const SelJob &J, uint64_t ka, uint32_t ia, uint64_t kb,
                                            uint32_t ib) {
  if (ka != kb) return ka < kb;
  if (ka == ~0ull) return ia < ib;
  return J.rec[ia].rank < J.rec[ib].rank;
}

__global__ void __launch_bounds__(256) sort_init_kernel(const SelJob *__restrict__ sj) {
  const SelJob &J = sj[blockIdx.y];
  const SelState *st = J.st;
  if (J.sortP == 0 || st->done != 1u) return;
  const int64_t n = (int64_t)st->ncand < J.cap ? (int64_t)st->ncand : J.cap;
  for (int64_t x = blockIdx.x * 256 + threadIdx.x; x < J.sortP; x += (int64_t)gridDim.x * 256) {
    J.skey[x] = x < n ? J.rec[x].key : ~0ull;
    J.sidx[x] = (uint32_t)x;
  }
}

// One compare-exchange stage (block size k, distance j >= kSortLocal) over
// global memory: thread t handles the pair (lo, lo + j).
__global__ void __launch_bounds__(256) sort_global_kernel(const SelJob *__restrict__ sj, int64_t k,
                                                          int64_t j) {
  const SelJob &J = sj[blockIdx.y];
  if (J.sortP == 0 || J.st->done != 1u) return;
  for (int64_t t = blockIdx.x * 256 + threadIdx.x; t < J.sortP / 2; t += (int64_t)gridDim.x * 256) {
    const int64_t lo = ((t & ~(j - 1)) << 1) | (t & (j - 1)), hi = lo + j;
    const bool asc = (lo & k) == 0;
    const uint64_t ka = J.skey[lo], kb = J.skey[hi];
    const uint32_t ia = J.sidx[lo], ib = J.sidx[hi];
    if (asc ? sort_before(J, kb, ib, ka, ia) : sort_before(J, ka, ia, kb, ib)) {
      J.skey[lo] = kb; J.skey[hi] = ka;
      J.sidx[lo] = ib; J.sidx[hi] = ia;
    }
  }
}

// The stages of distance j < kSortLocal inside blocks of kSortLocal entries
// in LDS: every block size from 2 up (full = 1), or only block size k.
constexpr int kSortLocal = 2048;
__global__ void __launch_bounds__(1024) sort_local_kernel(const SelJob *__restrict__ sj, int64_t k,
                                                          int full) {
  const SelJob &J = sj[blockIdx.y];
  if (J.sortP == 0 || J.st->done != 1u) return;
  __shared__ uint64_t lk[kSortLocal];
  __shared__ uint32_t li[kSortLocal];
  for (int64_t base = (int64_t)blockIdx.x * kSortLocal; base < J.sortP;
       base += (int64_t)gridDim.x * kSortLocal) {
    __syncthreads();
    for (int x = threadIdx.x; x < kSortLocal; x += 1024) {
      lk[x] = J.skey[base + x];
      li[x] = J.sidx[base + x];
    }
    __syncthreads();
    for (int64_t kk = full ? 2 : k; kk <= (full ? (int64_t)kSortLocal : k); kk <<= 1) {
      for (int jj = (int)((kk < kSortLocal ? kk : kSortLocal) >> 1); jj > 0; jj >>= 1) {
        const int t = threadIdx.x;  // pair t of the block
        const int lo = ((t & ~(jj - 1)) << 1) | (t & (jj - 1)), hi = lo + jj;
        const bool asc = ((base + lo) & kk) == 0;
        const uint64_t ka = lk[lo], kb = lk[hi];
        const uint32_t ia = li[lo], ib = li[hi];
        if (asc ? sort_before(J, kb, ib, ka, ia) : sort_before(J, ka, ia, kb, ib)) {
          lk[lo] = kb; lk[hi] = ka;
          li[lo] = ib; li[hi] = ia;
        }
        __syncthreads();
      }
    }
    for (int x = threadIdx.x; x < kSortLocal; x += 1024) {
      J.skey[base + x] = lk[x];
      J.sidx[base + x] = li[x];
    }
  }
}

__global__ void __launch_bounds__(256) sort_emit_kernel(const SelJob *__restrict__ sj) {
  const SelJob &J = sj[blockIdx.y];
  const SelState *st = J.st;
  if (J.sortP == 0 || st->done != 1u) return;
  const int64_t keff = st->keff;
  for (int64_t pos = blockIdx.x * 256 + threadIdx.x; pos < keff; pos += (int64_t)gridDim.x * 256)
    emit_hit(J, J.sidx[pos], pos);
}

__global__ void write_seljob_kernel(SelJob j0, SelJob *dst) { if (threadIdx.x == 0) *dst = j0; }

hipError_t launch_write_seljobs(const SelJob *h, int32_t n, SelJob *dst_dev, hipStream_t s) {
  for (int x = 0; x < n; ++x)
    hipLaunchKernelGGL(write_seljob_kernel, dim3(1), dim3(64), 0, s, h[x], dst_dev + x);
  return hipGetLastError();
}

hipError_t launch_init_select(SelJob *sel_dev, int32_t n_jobs, hipStream_t s) {
  hipLaunchKernelGGL(init_select_kernel, dim3((n_jobs + 63) / 64), dim3(64), 0, s, sel_dev,
                     n_jobs);
  return hipGetLastError();
}

// After a batch's sample pass (see launch_sample_bound in the header).
__global__ void sample_bound_kernel(SelJob *main, const SelJob *smp, int n) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  SelState *st = main[x].st;
  const SelState *ss = smp[x].st;
  float ub = __builtin_inff();
  uint32_t whi = 0xffffffffu;
  if (ss->done == 1u) {
    // the sample's k smallest are k scores of the whole set, so its k-th
    // smallest is at least the whole set's: every member of the FP64 top-k
    // has an FP32 score <= that + 2 e(N)
    const double u = (double)key2f(ss->kth) + main[x].err2;
    ub = (float)u;
    if ((double)ub < u) ub = __uint_as_float(__float_as_uint(ub) + 1u);  // ub >= 0: next float up
    whi = ss->kth;
  }
  st->ub = ub;
  st->whi = whi;
  st->cmode = 1u;
  st->cn = 0ull;
}

hipError_t launch_sample_bound(SelJob *main_dev, const SelJob *sample_dev, int32_t n_jobs,
                               hipStream_t s) {
  hipLaunchKernelGGL(sample_bound_kernel, dim3((n_jobs + 63) / 64), dim3(64), 0, s, main_dev,
                     sample_dev, n_jobs);
  return hipGetLastError();
}

hipError_t launch_select_kth(SelJob *sel_dev, int32_t n_jobs, int64_t max_T, hipStream_t s) {
  const unsigned nj = (unsigned)n_jobs;
  hipLaunchKernelGGL(window_kernel, dim3((n_jobs + 63) / 64), dim3(64), 0, s, sel_dev, n_jobs);
  int64_t hb = (max_T + 256 * 16 - 1) / (256 * 16);
  if (hb > 2048) hb = 2048;
  if (hb < 1) hb = 1;
  for (int p = 0; p < kHistPasses; ++p) {
    hipLaunchKernelGGL(hist_kernel, dim3((unsigned)hb, nj), dim3(256), 0, s, sel_dev, 0);
    hipLaunchKernelGGL(find_kernel, dim3(nj), dim3(1024), 0, s, sel_dev, 0);
  }
  return hipGetLastError();
}

hipError_t launch_select(SelJob *sel_dev, int32_t n_jobs, int64_t max_T, int64_t max_cap,
                         int32_t max_k, bool sampled, hipStream_t s) {
  const unsigned nj = (unsigned)n_jobs;
  hipLaunchKernelGGL(window_kernel, dim3((n_jobs + 63) / 64), dim3(64), 0, s, sel_dev, n_jobs);
  int64_t hb = (max_T + 256 * 16 - 1) / (256 * 16);
  if (hb > 2048) hb = 2048;
  if (hb < 1) hb = 1;
  if (sampled) {
    int64_t hs = (sample_len(max_T) + 256 * 16 - 1) / (256 * 16);
    if (hs > 2048) hs = 2048;
    if (hs < 1) hs = 1;
    for (int p = 0; p < kHistPasses; ++p) {
      hipLaunchKernelGGL(hist_kernel, dim3((unsigned)hs, nj), dim3(256), 0, s, sel_dev, 1);
      hipLaunchKernelGGL(find_kernel, dim3(nj), dim3(1024), 0, s, sel_dev, 1);
    }
    hipLaunchKernelGGL(bound_kernel, dim3((n_jobs + 63) / 64), dim3(64), 0, s, sel_dev, n_jobs);
    hipLaunchKernelGGL(compact_kernel, dim3((unsigned)hb, nj), dim3(256), 0, s, sel_dev, 1);
  }
  for (int p = 0; p < kHistPasses; ++p) {
    hipLaunchKernelGGL(hist_kernel, dim3((unsigned)hb, nj), dim3(256), 0, s, sel_dev, 0);
    hipLaunchKernelGGL(find_kernel, dim3(nj), dim3(1024), 0, s, sel_dev, 0);
    if (p == 0)
      hipLaunchKernelGGL(compact_kernel, dim3((unsigned)hb, nj), dim3(256), 0, s, sel_dev, 0);
  }
  hipLaunchKernelGGL(threshold_kernel, dim3((n_jobs + 63) / 64), dim3(64), 0, s, sel_dev, n_jobs);
  hipLaunchKernelGGL(collect_kernel, dim3((unsigned)hb, nj), dim3(256), 0, s, sel_dev);
  int64_t rb = (max_cap + 3) / 4;
  if (rb > 4096) rb = 4096;
  if (rb < 1) rb = 1;
  hipLaunchKernelGGL(rescore_kernel, dim3((unsigned)rb, nj), dim3(256), 0, s, sel_dev);
  int64_t kb = (max_cap + 63) / 64;
  if (kb > 1024) kb = 1024;
  if (kb < 1) kb = 1;
  hipLaunchKernelGGL(rank_kernel, dim3((unsigned)kb, nj), dim3(kRankThreads), 0, s, sel_dev);
  const int64_t P = sort_len(max_cap);  // jobs with sort buffers (each skips the other path)
  if (P > 0) {
    const unsigned gb = (unsigned)std::min<int64_t>(P / 512, 4096);
    const unsigned lb = (unsigned)std::min<int64_t>(P / kSortLocal, 1024);
    hipLaunchKernelGGL(sort_init_kernel, dim3(gb, nj), dim3(256), 0, s, sel_dev);
    hipLaunchKernelGGL(sort_local_kernel, dim3(lb, nj), dim3(1024), 0, s, sel_dev, (int64_t)0, 1);
    for (int64_t k2 = 2 * kSortLocal; k2 <= P; k2 <<= 1) {
      for (int64_t j = k2 >> 1; j >= kSortLocal; j >>= 1)
        hipLaunchKernelGGL(sort_global_kernel, dim3(gb, nj), dim3(256), 0, s, sel_dev, k2, j);
      hipLaunchKernelGGL(sort_local_kernel, dim3(lb, nj), dim3(1024), 0, s, sel_dev, k2, 0);
    }
    const unsigned eb = (unsigned)std::min<int64_t>((max_k + 255) / 256, 1024);
    hipLaunchKernelGGL(sort_emit_kernel, dim3(eb > 0 ? eb : 1, nj), dim3(256), 0, s, sel_dev);
  }
  return hipGetLastError();
}

// ------------------------------------------------------- test hook ----
__global__ void __launch_bounds__(256) score_triplets_kernel(
    const uint32_t *__restrict__ planes, const int32_t *__restrict__ pairs,
    const double *__restrict__ lf64, const float *__restrict__ lf32, int M, int64_t Mp, int W0,
    int W1, int N0, int N1, const uint32_t *__restrict__ ijk, int64_t n,
    uint32_t *__restrict__ counts, float *__restrict__ k2f, double *__restrict__ k2d) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t c = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); c < n;
       c += waves) {
    const uint32_t i = ijk[3 * c], j = ijk[3 * c + 1], k = ijk[3 * c + 2];
    if (!(i < j && j < k && k < (uint32_t)M)) {  // not a triplet of this data set
      if (lane == 0) {
        if (k2f) k2f[c] = __builtin_nanf("");
        if (k2d) k2d[c] = __builtin_nan("");
        if (counts)
          for (int x = 0; x < 54; ++x) counts[c * 54 + x] = 0xffffffffu;
      }
      continue;
    }
    int tab[2][27];
    triplet_table(planes, pairs, nullptr, 1, nullptr, EPI3_LAYOUT_SPLIT, Mp, W0, W1, N0, N1, i, j,
                  k, tab);
    if (lane == 0) {
      float f = 0.f;
      for (int x = 0; x < 27; ++x) {
        const int r0 = tab[0][x], r1 = tab[1][x];
        f += lf32[r0 + r1 + 1] - (lf32[r0] + lf32[r1]);
      }
      if (k2f) k2f[c] = f;
      if (k2d) k2d[c] = k2_fp64(tab, lf64);
      if (counts)
        for (int x = 0; x < 27; ++x) {
          counts[c * 54 + x] = (uint32_t)tab[0][x];
          counts[c * 54 + 27 + x] = (uint32_t)tab[1][x];
        }
    }
  }
}

hipError_t launch_score_triplets(const epi3_dataset &d, const uint32_t *ijk, int64_t n,
                                 uint32_t *counts, float *k2f, double *k2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 3) / 4;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(score_triplets_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     (const uint32_t *)d.planes, d.pairs, d.lf64, d.lf32, d.n_snps,
                     (int64_t)d.snp_stride,
                     d.words[0], d.words[1], d.n_controls, d.n_cases, ijk, n, counts, k2f, k2);
  return hipGetLastError();
}

}  // namespace epi3
