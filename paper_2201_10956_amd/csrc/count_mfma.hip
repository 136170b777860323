// Count stage for many phenotypes at once on the int8 matrix cores.
//
// With all samples kept in one set of planes (no class split), the cases of
// phenotype q among the samples of genotype cell (a, b, c) of triplet
// (i, j, k) are
//     n_q(a, b, c) = sum_s X_i[a][s] X_j[b][s] X_k[c][s] PH_q[s],
// a dense contraction over samples s of 0/1 values: rows (triplet, corner
// cell) x columns (phenotype q) with K = samples, exact in int32.  The paper
// fills its table with 27 AND + POPCNT per 32 samples and class (Alg. 2);
// here the 8 corner cells of the cases of 32 phenotypes come from one
// v_mfma_i32_32x32x32_i8 per 32 samples and 4 triplets, and the other 19
// cells follow from pairwise tables as in the vector-ALU kernel.  Totals
// (cases + controls) come from byte popcounts of the same operand, so
// controls = totals - cases.
//
// Fragment layout of v_mfma_i32_32x32x32_i8 (gfx950, checked on hardware):
// lane l supplies A row l % 32 and B column l % 32 with 16 consecutive K
// values starting at 16 (l / 32); the result of row r, column c is in lane
// c + 32 ((r / 4) % 2), register 4 (r / 8) + r % 4.
#include "epi3_internal.h"

namespace epi3 {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kPermKB = 16;  // k values per wave tile (4 row tiles x 4 triplets)
constexpr int kPermT = 4;    // row tiles per wave tile

__host__ __device__ __forceinline__ int64_t perm_tiles_of_j(int64_t M, int64_t j) {
  if (j < 1 || j > M - 2) return 0;
  return ((j + 3) / 4) * ((M - 1 - j + kPermKB - 1) / kPermKB);
}

__device__ __forceinline__ int64_t rfl64p(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t popc4(v4i x) {
  return __builtin_popcount((uint32_t)x.x) + __builtin_popcount((uint32_t)x.y) +
         __builtin_popcount((uint32_t)x.z) + __builtin_popcount((uint32_t)x.w);
}

// jprefix for the permutation tiles (one block).
__global__ void __launch_bounds__(1024) perm_prefix_kernel(PermJob *pj) {
  const int64_t M = pj->M;
  int64_t *pre = const_cast<int64_t *>(pj->jprefix);
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (M + 1023) / 1024;
  const int64_t a = t * chunk, b = (a + chunk < M) ? a + chunk : M;
  int64_t sum = 0;
  for (int64_t j = a; j < b; ++j) sum += perm_tiles_of_j(M, j);
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - sum;
  for (int64_t j = a; j < b; ++j) {
    pre[j] = run;
    run += perm_tiles_of_j(M, j);
  }
  if (t == 1023) pre[M] = part[1023];
}

// PH[q][s] = 1 if sample s is a case of phenotype q (0 for q >= Q or s >= N);
// n1[q] = number of cases.  One block per q.
__global__ void __launch_bounds__(256) mask_bytes_kernel(const uint32_t *const *masks, int32_t Q,
                                                         int32_t N, int32_t S, uint8_t *ph,
                                                         int32_t *n1) {
  const int q = blockIdx.x;
  __shared__ int red[256];
  int cnt = 0;
  uint32_t *row = reinterpret_cast<uint32_t *>(ph + (int64_t)q * S);
  for (int d = threadIdx.x; d < S / 4; d += blockDim.x) {
    uint32_t v = 0;
    if (q < Q) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int s = 4 * d + b;
        if (s < N) {
          const uint32_t bit = (masks[q][s >> 5] >> (s & 31)) & 1u;
          v |= bit << (8 * b);
          cnt += (int)bit;
        }
      }
    }
    row[d] = v;
  }
  red[threadIdx.x] = cnt;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) n1[q] = red[0];
}

// Case pairs of every phenotype: out[x][y][q] = (n(0,0), n(0,1), n(1,0), n(1,1))
// over the samples whose bit is set in mask q.  One wave per (x, 64 y); the
// block's z index selects a group of 16 phenotypes.
__global__ void __launch_bounds__(256) case_pairs_kernel(const uint32_t *__restrict__ planes,
                                                         int32_t Mp, int32_t W,
                                                         const uint32_t *const *masks, int32_t Q,
                                                         int32_t Qp, int32_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int x = __builtin_amdgcn_readfirstlane(blockIdx.y * 4 + (threadIdx.x >> 6));
  const int y = blockIdx.x * 64 + lane;
  const int q0 = blockIdx.z * 16;
  if (x >= Mp) return;
  uint32_t acc[16][4];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t][0] = acc[t][1] = acc[t][2] = acc[t][3] = 0u;
  cptr<uint32_t> pc = as_const(planes);
  const uint2 *pv = reinterpret_cast<const uint2 *>(planes);
  for (int w = 0; w < W; ++w) {
    const uint32_t x0 = pc[((int64_t)w * Mp + x) * 2], x1 = pc[((int64_t)w * Mp + x) * 2 + 1];
    const uint2 yv = (y < Mp) ? pv[(int64_t)w * Mp + y] : make_uint2(0u, 0u);
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int q = q0 + t;
      const uint32_t mk = q < Q ? masks[q][w] : 0u;
      const uint32_t a0 = x0 & mk, a1 = x1 & mk;
      acc[t][0] += __builtin_popcount(a0 & yv.x);
      acc[t][1] += __builtin_popcount(a0 & yv.y);
      acc[t][2] += __builtin_popcount(a1 & yv.x);
      acc[t][3] += __builtin_popcount(a1 & yv.y);
    }
  }
  if (y >= Mp) return;
  int4 *o = reinterpret_cast<int4 *>(out) + ((int64_t)x * Mp + y) * Qp;
#pragma unroll
  for (int t = 0; t < 16; ++t)
    if (q0 + t < Qp)
      o[q0 + t] = make_int4((int)acc[t][0], (int)acc[t][1], (int)acc[t][2], (int)acc[t][3]);
}

__device__ __forceinline__ void load_pair(const int32_t *p, int64_t idx, int v[4]) {
  const int4 x = reinterpret_cast<const int4 *>(p)[idx];
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}

// Staging geometry: samples are processed in chunks of kKC staged in LDS,
// each row padded to an odd number of 16-byte units against bank conflicts.
constexpr int kKC = 128;
constexpr int kRow = kKC + 16;
constexpr int kRowsPH = 64;                  // phenotype rows (B operand)
constexpr int kRowsXK = 2 * kPermKB;         // (k, c) rows shared by the 4 waves
constexpr int kRowsP = 16;                   // pair rows X_i[a] & X_j[b]: 4 waves x 4 (a, b)
constexpr int kRowsAll = kRowsPH + kRowsXK + kRowsP;
constexpr int kStageBytes = kRowsAll * kRow; // one buffer
constexpr int kChunks16 = kRowsAll * (kKC / 16);
// epilogue data placed in the staging buffers (bytes)
constexpr int kEpiBytes = 16 * 4 * 64 + 8 * 4 * 64 + 8 * 64 + 4 * 64 + 16 * (4 * 16 + 16 + 16 + 4 + 4 + 4) +
                          16 * 4 * 4 * 64 + 16 * 4 * 64 + 8 * 4 * 64;
static_assert(kEpiBytes <= 2 * kStageBytes, "epilogue data must fit the staging buffers");

template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

// Workgroup tile: pivot j, four pivots i = 4 ib + wave (one per wave), 16
// consecutive k > j, 64 phenotypes.  Phenotype bytes, the k planes and the
// pair words are staged per chunk of kKC samples in double-buffered LDS; each
// wave then runs 8 MFMAs per 32 samples (4 row tiles of 4 triplets x 8
// corner cells, 2 column tiles of 32 phenotypes).
__global__ void __launch_bounds__(256) count_mfma_perm_kernel(const PermJob *__restrict__ pjp,
                                                              SelState *__restrict__ st,
                                                              unsigned long long *__restrict__ queue,
                                                              const float *__restrict__ lf32,
                                                              int lf_len) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  uint8_t *stage = smem;                                          // 2 buffers
  uint32_t *sTot = reinterpret_cast<uint32_t *>(smem + 2 * kStageBytes);
  int64_t *sTile = reinterpret_cast<int64_t *>(sTot + 4 * kPermT * 32);
  float *sL = reinterpret_cast<float *>(sTile + 2);
  for (int x = threadIdx.x; x < lf_len; x += blockDim.x) sL[x] = lf32[x];

  const PermJob pj = *pjp;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  uint32_t *myTot = sTot + wave * (kPermT * 32);
  const int r = lane & 31, g = lane >> 5;
  const int ta = r >> 3, ra = (r >> 2) & 1, rb = (r >> 1) & 1, rc = r & 1;
  const int M = pj.M, Mp = pj.Mp, S = pj.S, Q = pj.Q, Qp = pj.Qp;
  const int64_t T = pj.T;
  gptr<uint8_t> gb = (gptr<uint8_t>)pj.bytes;
  gptr<uint8_t> gph = (gptr<uint8_t>)pj.ph;
  cptr<int64_t> pre = as_const(pj.jprefix);
  const int nch = S / kKC;  // S is a multiple of 256
  int j = -1;
  int64_t jlo = 0, jhi = 0;

  for (;;) {
    __syncthreads();  // previous tile's readers of sTile / stage are done
    if (tid == 0) sTile[0] = (int64_t)atomicAdd(queue, 1ull);
    __syncthreads();
    const int64_t t = rfl64p(sTile[0]);
    if (t >= pj.n_tiles) break;
    if (j < 0 || t < jlo || t >= jhi) {
      int lo = 0, hi = M - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= t) lo = mid; else hi = mid - 1;
      }
      j = lo;
      jlo = pre[j];
      jhi = pre[j + 1];
    }
    const int nkb = (M - 1 - j + kPermKB - 1) / kPermKB;
    const int rr = (int)(t - jlo);
    const int ib = rr / nkb, kb = rr - ib * nkb;
    const int i = 4 * ib + wave;  // may be >= j (then the wave's results are dropped)
    const int kbase = j + 1 + kb * kPermKB;

    // ---- staging plan: this thread's 16-byte chunks of one LDS buffer ----
    // rows [0, 64): phenotype q; [64, 96): (k, c) = k planes; [96, 112): pair rows.
    auto chunk_src = [&](int c16, int ch, v4i &v) {
      const int row = c16 >> 3, col = (c16 & 7) * 16;
      const int64_t s0 = (int64_t)ch * kKC + col;
      if (row < kRowsPH) {
        v = *reinterpret_cast<gptr<v4i>>(gph + (int64_t)row * S + s0);
      } else if (row < kRowsPH + kRowsXK) {
        const int x = row - kRowsPH;
        v = *reinterpret_cast<gptr<v4i>>(gb + ((int64_t)(kbase + (x >> 1)) * 2 + (x & 1)) * S + s0);
      } else {
        const int x = row - kRowsPH - kRowsXK;  // wave w = x >> 2, (a, b) = x & 3
        const int ii = 4 * ib + (x >> 2);
        const v4i va =
            *reinterpret_cast<gptr<v4i>>(gb + ((int64_t)ii * 2 + ((x >> 1) & 1)) * S + s0);
        const v4i vb = *reinterpret_cast<gptr<v4i>>(gb + ((int64_t)j * 2 + (x & 1)) * S + s0);
        v = va & vb;
      }
    };
    constexpr int kPer = (kChunks16 + 255) / 256;  // chunks per thread (4)
    v4i pf[kPer];
    auto fetch = [&](int ch) {
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int c16 = tid + 256 * u;
        if (c16 < kChunks16) chunk_src(c16, ch, pf[u]);
      }
    };
    auto store = [&](int buf) {
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int c16 = tid + 256 * u;
        if (c16 < kChunks16) {
          const int row = c16 >> 3, col = (c16 & 7) * 16;
          *reinterpret_cast<v4i *>(stage + buf * kStageBytes + row * kRow + col) = pf[u];
        }
      }
    };

    v16i acc[kPermT][2];
    uint32_t tot[kPermT];
#pragma unroll
    for (int tt = 0; tt < kPermT; ++tt) {
      tot[tt] = 0u;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[tt][0][v] = acc[tt][1][v] = 0;
    }
    fetch(0);
    store(0);
    __syncthreads();
    const int prow = kRowsPH + kRowsXK + wave * 4 + (ra * 2 + rb);
    for (int ch = 0; ch < nch; ++ch) {
      if (ch + 1 < nch) fetch(ch + 1);
      const uint8_t *buf = stage + (ch & 1) * kStageBytes;
#pragma unroll
      for (int stp = 0; stp < kKC / 32; ++stp) {
        const int off = stp * 32 + 16 * g;
        const v4i p = *reinterpret_cast<const v4i *>(buf + prow * kRow + off);
        const v4i b0 = *reinterpret_cast<const v4i *>(buf + r * kRow + off);
        const v4i b1 = *reinterpret_cast<const v4i *>(buf + (32 + r) * kRow + off);
#pragma unroll
        for (int tt = 0; tt < kPermT; ++tt) {
          const int xrow = kRowsPH + (4 * tt + ta) * 2 + rc;
          const v4i a = p & *reinterpret_cast<const v4i *>(buf + xrow * kRow + off);
          tot[tt] += popc4(a);
          acc[tt][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b0, acc[tt][0], 0, 0, 0);
          acc[tt][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b1, acc[tt][1], 0, 0, 0);
        }
      }
      if (ch + 1 < nch) store((ch + 1) & 1);
      __syncthreads();
    }

    // totals of row r (both sample halves) to LDS
#pragma unroll
    for (int tt = 0; tt < kPermT; ++tt) {
      const uint32_t full = tot[tt] + __shfl_xor(tot[tt], 32);
      if (g == 0) myTot[tt * 32 + r] = full;
    }

    // ---- epilogue data staged in the (now idle) staging buffers ----
    // fixed per tile: case pairs (i, j), (i, i), (j, j) of every phenotype, the
    // phenotypes' case counts and the all-sample pairs of the tile; then per
    // row tile: case pairs (i, k), (j, k), (k, k).  One batched round of loads
    // per row tile instead of a dependent chain per triplet and phenotype.
    int4 *eFix = reinterpret_cast<int4 *>(stage);
    int4 *ePij = eFix;                      // [4 waves][64 q]
    int2 *ePii = reinterpret_cast<int2 *>(ePij + 4 * 64);   // [4][64]
    int2 *ePjj = ePii + 4 * 64;             // [64]
    int *eN1 = reinterpret_cast<int *>(ePjj + 64);          // [64]
    int4 *eTik = reinterpret_cast<int4 *>(eN1 + 64);         // [4 waves][16 k]
    int4 *eTjk = eTik + 4 * kPermKB;        // [16]
    int4 *eTkk = eTjk + kPermKB;            // [16]
    int4 *eTij = eTkk + kPermKB;            // [4]
    int4 *eTii = eTij + 4;                  // [4]
    int4 *eTjj = eTii + 4;                  // [1]
    int4 *ePik = eTjj + 4;                  // per row tile: [4 waves][4 tg][64 q]
    int4 *ePjk = ePik + 4 * 4 * 64;         // [4 tg][64 q]
    int2 *ePkk = reinterpret_cast<int2 *>(ePjk + 4 * 64);   // [4 tg][64 q]
    const int ib4 = 4 * ib;
    {
      const int4 *cp = reinterpret_cast<const int4 *>(pj.case_pairs);
      const int4 *tp = reinterpret_cast<const int4 *>(pj.tot_pairs);
      // case pairs (i, j) and (i, i): 256 each; (j, j), n1: 64 each
      const int w = tid >> 6, q = tid & 63;
      const int qq = q < Qp ? q : Qp - 1;
      const int ii = ib4 + w;
      const int4 a = cp[((int64_t)ii * Mp + j) * Qp + qq];
      const int4 b = cp[((int64_t)ii * Mp + ii) * Qp + qq];
      int4 c = make_int4(0, 0, 0, 0);
      int n1v = 0;
      if (w == 0) c = cp[((int64_t)j * Mp + j) * Qp + qq];
      if (w == 1) n1v = pj.n1[qq];
      int4 d = make_int4(0, 0, 0, 0);
      // all-sample pairs: tik [4][16] (threads 0..63), tjk, tkk (64..95), tij, tii, tjj
      if (tid < 64) d = tp[(int64_t)(ib4 + (tid >> 4)) * Mp + kbase + (tid & 15)];
      else if (tid < 80) d = tp[(int64_t)j * Mp + kbase + (tid - 64)];
      else if (tid < 96) d = tp[(int64_t)(kbase + tid - 80) * Mp + kbase + (tid - 80)];
      else if (tid < 100) d = tp[(int64_t)(ib4 + tid - 96) * Mp + j];
      else if (tid < 104) d = tp[(int64_t)(ib4 + tid - 100) * Mp + (ib4 + tid - 100)];
      else if (tid < 105) d = tp[(int64_t)j * Mp + j];
      ePij[tid] = a;
      ePii[tid] = make_int2(b.x, b.w);
      if (w == 0) ePjj[q] = make_int2(c.x, c.w);
      if (w == 1) eN1[q] = n1v;
      if (tid < 64) eTik[tid] = d;
      else if (tid < 80) eTjk[tid - 64] = d;
      else if (tid < 96) eTkk[tid - 80] = d;
      else if (tid < 100) eTij[tid - 96] = d;
      else if (tid < 104) eTii[tid - 100] = d;
      else if (tid < 105) eTjj[0] = d;
    }
    const int h = g;
    const int iw = wave;  // this wave's pivot i = ib4 + iw
    const bool wave_valid = i < j;
    uint32_t kmin[2] = {0xffffffffu, 0xffffffffu}, kmax[2] = {0u, 0u};
    const int64_t base_ij = wave_valid ? lex_base(M, i, j) : 0;
#pragma unroll
    for (int tt = 0; tt < kPermT; ++tt) {
      __syncthreads();  // previous row tile's readers are done
      {
        const int4 *cp = reinterpret_cast<const int4 *>(pj.case_pairs);
        const int q = tid & 63;
        const int qq = q < Qp ? q : Qp - 1;
        int4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // (i, k): [4 waves][4 tg] x 64 q = 1024
          const int x = (tid >> 6) + 4 * u;  // 0..15 = w * 4 + tg
          const int ii = ib4 + (x >> 2), kk = kbase + 4 * tt + (x & 3);
          v[u] = cp[((int64_t)ii * Mp + kk) * Qp + qq];
        }
        const int tg = tid >> 6, kk = kbase + 4 * tt + tg;
        const int4 vjk = cp[((int64_t)j * Mp + kk) * Qp + qq];
        const int4 vkk = cp[((int64_t)kk * Mp + kk) * Qp + qq];
#pragma unroll
        for (int u = 0; u < 4; ++u) ePik[((tid >> 6) + 4 * u) * 64 + q] = v[u];
        ePjk[tg * 64 + q] = vjk;
        ePkk[tg * 64 + q] = make_int2(vkk.x, vkk.w);
      }
      __syncthreads();
      if (!wave_valid) continue;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int tg = 2 * h + u;  // triplet within the row tile
        const int kl = 4 * tt + tg;
        const int k = kbase + kl;
        // totals table of this triplet (the same for every phenotype)
        uint32_t tn[8];
#pragma unroll
        for (int x = 0; x < 8; ++x) tn[x] = myTot[tt * 32 + 8 * tg + x];
        int ttab[27];
        {
          const int4 a = eTij[iw], b = eTik[iw * kPermKB + kl], c = eTjk[kl];
          const int4 ii4 = eTii[iw], jj4 = eTjj[0], kk4 = eTkk[kl];
          const int tij[4] = {a.x, a.y, a.z, a.w}, tik[4] = {b.x, b.y, b.z, b.w};
          const int tjk[4] = {c.x, c.y, c.z, c.w};
          const int mi[2] = {ii4.x, ii4.w}, mj[2] = {jj4.x, jj4.w}, mk[2] = {kk4.x, kk4.w};
          complete_table(tn, tij, tik, tjk, mi, mj, mk, pj.N, ttab);
        }
        float tl[27];  // L[r + 1] of each row: Eq. 1's first inner sum, shared by all phenotypes
#pragma unroll
        for (int x = 0; x < 27; ++x) tl[x] = sL[ttab[x] + 1];
#pragma unroll
        for (int qb = 0; qb < 2; ++qb) {
          const int q = qb * 32 + r;
          int send[4], recv[4];
          // lane h holds corner cells a = h of triplets; partner holds a = 1 - h
#pragma unroll
          for (int x = 0; x < 4; ++x)
            send[x] = h ? acc[tt][qb][4 * u + x] : acc[tt][qb][8 + 4 * u + x];
#pragma unroll
          for (int x = 0; x < 4; ++x) recv[x] = __shfl_xor(send[x], 32);
          uint32_t cn[8];
#pragma unroll
          for (int bc = 0; bc < 4; ++bc) {
            const int own = h ? acc[tt][qb][8 + 4 * u + bc] : acc[tt][qb][4 * u + bc];
            cn[bc] = (uint32_t)(h ? recv[bc] : own);      // a = 0
            cn[4 + bc] = (uint32_t)(h ? own : recv[bc]);  // a = 1
          }
          int ctab[27];
          {
            const int4 a = ePij[iw * 64 + q], b = ePik[(iw * 4 + tg) * 64 + q], c = ePjk[tg * 64 + q];
            const int2 ii2 = ePii[iw * 64 + q], jj2 = ePjj[q], kk2 = ePkk[tg * 64 + q];
            const int cij[4] = {a.x, a.y, a.z, a.w}, cik[4] = {b.x, b.y, b.z, b.w};
            const int cjk[4] = {c.x, c.y, c.z, c.w};
            const int mi[2] = {ii2.x, ii2.y}, mj[2] = {jj2.x, jj2.y}, mk[2] = {kk2.x, kk2.y};
            complete_table(cn, cij, cik, cjk, mi, mj, mk, eN1[q], ctab);
          }
          float k2 = 0.f;  // rows in order, each L[r + 1] - (L[r_0] + L[r_1]) as in the plain kernel
#pragma unroll
          for (int x = 0; x < 27; ++x) k2 += tl[x] - (sL[ttab[x] - ctab[x]] + sL[ctab[x]]);
          if (q < Q && k < M) {
            pj.score[(int64_t)q * T + base_ij + k] = k2;
            const uint32_t key = f2key(k2);
            kmin[qb] = key < kmin[qb] ? key : kmin[qb];
            kmax[qb] = key > kmax[qb] ? key : kmax[qb];
          }
        }
      }
    }
    // per-phenotype key range: lanes q and q + 32 hold the same q
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
      const int q = qb * 32 + r;
      const uint32_t omin = __shfl_xor(kmin[qb], 32), omax = __shfl_xor(kmax[qb], 32);
      const uint32_t mn = omin < kmin[qb] ? omin : kmin[qb];
      const uint32_t mx = omax > kmax[qb] ? omax : kmax[qb];
      if (h == 0 && q < Q && mx != 0u) {
        atomicMin(&st[q].kmin, mn);
        atomicMax(&st[q].kmax, mx);
      }
    }
  }
}

hipError_t launch_perm_prefix(PermJob *pj_dev, hipStream_t s) {
  hipLaunchKernelGGL(perm_prefix_kernel, dim3(1), dim3(1024), 0, s, pj_dev);
  return hipGetLastError();
}

hipError_t launch_mask_bytes(const uint32_t *const *masks_dev, int32_t Q, int32_t Qp, int32_t N,
                             int32_t S, uint8_t *ph, int32_t *n1, hipStream_t s) {
  hipLaunchKernelGGL(mask_bytes_kernel, dim3(Qp), dim3(256), 0, s, masks_dev, Q, N, S, ph, n1);
  return hipGetLastError();
}

hipError_t launch_case_pairs(const uint32_t *planes, int32_t Mp, int32_t W,
                             const uint32_t *const *masks_dev, int32_t Q, int32_t Qp, int32_t *out,
                             hipStream_t s) {
  dim3 grid((Mp + 63) / 64, (Mp + 3) / 4, (Qp + 15) / 16);
  hipLaunchKernelGGL(case_pairs_kernel, grid, dim3(256), 0, s, planes, Mp, W, masks_dev, Q, Qp, out);
  return hipGetLastError();
}

__global__ void write_permjob_kernel(PermJob h, PermJob *dst) { if (threadIdx.x == 0) *dst = h; }

hipError_t launch_write_permjob(const PermJob &h, PermJob *dst_dev, hipStream_t s) {
  hipLaunchKernelGGL(write_permjob_kernel, dim3(1), dim3(64), 0, s, h, dst_dev);
  return hipGetLastError();
}

struct PtrPack {
  const uint32_t *p[32];
};
__global__ void write_ptrs_kernel(PtrPack h, int n, const uint32_t **dst) {
  if ((int)threadIdx.x < n) dst[threadIdx.x] = h.p[threadIdx.x];
}

hipError_t launch_write_ptrs(const uint32_t *const *h, int32_t n, const uint32_t **dst_dev,
                             hipStream_t s) {
  for (int32_t base = 0; base < n; base += 32) {
    PtrPack pk{};
    const int m = n - base < 32 ? n - base : 32;
    for (int x = 0; x < m; ++x) pk.p[x] = h[base + x];
    hipLaunchKernelGGL(write_ptrs_kernel, dim3(1), dim3(64), 0, s, pk, m, dst_dev + base);
  }
  return hipGetLastError();
}

int64_t host_perm_tiles(int64_t M) {
  int64_t n = 0;
  for (int64_t j = 0; j < M; ++j) n += perm_tiles_of_j(M, j);
  return n;
}

hipError_t launch_count_mfma_perm(const PermJob *pj_dev, int64_t n_tiles, SelState *st,
                                  unsigned long long *queue, const float *lf32, int32_t lf_len,
                                  hipStream_t s) {
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const size_t lds = 2 * (size_t)kStageBytes + 4 * kPermT * 32 * sizeof(uint32_t) +
                     2 * sizeof(int64_t) + (size_t)lf_len * sizeof(float);
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(&count_mfma_perm_kernel),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, count_mfma_perm_kernel, 256, lds);
  if (e != hipSuccess) return e;
  if (per_cu <= 0) per_cu = 1;
  int64_t blocks = (int64_t)n_cu * per_cu;
  if (blocks > n_tiles) blocks = n_tiles > 0 ? n_tiles : 1;
  hipLaunchKernelGGL(count_mfma_perm_kernel, dim3((unsigned)blocks), dim3(256), lds, s, pj_dev, st,
                     queue, lf32, lf_len);
  return hipGetLastError();
}

}  // namespace epi3
