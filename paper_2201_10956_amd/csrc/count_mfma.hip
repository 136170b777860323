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
  return j * ((M - 1 - j + kPermKB - 1) / kPermKB);
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

// One wave tile: pivot pair (i, j), 16 consecutive k > j, 64 phenotypes.
__global__ void __launch_bounds__(256) count_mfma_perm_kernel(const PermJob *__restrict__ pjp,
                                                              SelState *__restrict__ st,
                                                              unsigned long long *__restrict__ queue,
                                                              const float *__restrict__ lf32,
                                                              int lf_len) {
  extern __shared__ float smem[];
  float *sL = smem;
  uint32_t *sTot = reinterpret_cast<uint32_t *>(smem + ((lf_len + 3) & ~3));
  for (int x = threadIdx.x; x < lf_len; x += blockDim.x) sL[x] = lf32[x];
  __syncthreads();

  const PermJob pj = *pjp;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t *myTot = sTot + wave * (kPermT * 32);
  const int r = lane & 31, g = lane >> 5;
  const int ta = r >> 3, ra = (r >> 2) & 1, rb = (r >> 1) & 1, rc = r & 1;
  const int M = pj.M, Mp = pj.Mp, S = pj.S, Q = pj.Q, Qp = pj.Qp;
  const int64_t T = pj.T;
  cptr<int64_t> pre = as_const(pj.jprefix);
  int j = -1;
  int64_t jlo = 0, jhi = 0;

  for (;;) {
    unsigned long long got = 0;
    if (lane == 0) got = atomicAdd(queue, 1ull);
    const int64_t t = rfl64p((int64_t)got);
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
    const int i = rr / nkb, kb = rr - i * nkb;
    const int kbase = j + 1 + kb * kPermKB;

    // ---- main loop over samples: 32 per step ----
    v16i acc[kPermT][2];
    uint32_t tot[kPermT];
#pragma unroll
    for (int tt = 0; tt < kPermT; ++tt) {
      tot[tt] = 0u;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[tt][0][v] = acc[tt][1][v] = 0;
    }
    const uint8_t *xi = pj.bytes + ((int64_t)i * 2 + ra) * S + 16 * g;
    const uint8_t *xj = pj.bytes + ((int64_t)j * 2 + rb) * S + 16 * g;
    const uint8_t *ph0 = pj.ph + (int64_t)r * S + 16 * g;
    const uint8_t *ph1 = pj.ph + (int64_t)(32 + r) * S + 16 * g;
    const uint8_t *xk[kPermT];
#pragma unroll
    for (int tt = 0; tt < kPermT; ++tt)
      xk[tt] = pj.bytes + ((int64_t)(kbase + 4 * tt + ta) * 2 + rc) * S + 16 * g;
    for (int s0 = 0; s0 < S; s0 += 32) {
      const v4i vi = *reinterpret_cast<const v4i *>(xi + s0);
      const v4i vj = *reinterpret_cast<const v4i *>(xj + s0);
      const v4i b0 = *reinterpret_cast<const v4i *>(ph0 + s0);
      const v4i b1 = *reinterpret_cast<const v4i *>(ph1 + s0);
      const v4i p = vi & vj;
#pragma unroll
      for (int tt = 0; tt < kPermT; ++tt) {
        const v4i vk = *reinterpret_cast<const v4i *>(xk[tt] + s0);
        const v4i a = p & vk;
        tot[tt] += popc4(a);
        acc[tt][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b0, acc[tt][0], 0, 0, 0);
        acc[tt][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b1, acc[tt][1], 0, 0, 0);
      }
    }
    // totals of row r (both sample halves) to LDS
#pragma unroll
    for (int tt = 0; tt < kPermT; ++tt) {
      const uint32_t full = tot[tt] + __shfl_xor(tot[tt], 32);
      if (g == 0) myTot[tt * 32 + r] = full;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");

    // ---- epilogue: lane (q, h) finishes triplets 2h, 2h + 1 of every row tile ----
    const int h = g;
    const int64_t MpMp = (int64_t)Mp * Mp;
    int tij[4], tii[4], tjj[4];
    load_pair(pj.tot_pairs, (int64_t)i * Mp + j, tij);
    load_pair(pj.tot_pairs, (int64_t)i * Mp + i, tii);
    load_pair(pj.tot_pairs, (int64_t)j * Mp + j, tjj);
    (void)MpMp;
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
      const int q = qb * 32 + r;
      const bool qvalid = q < Q;
      const int qq = q < Qp ? q : Qp - 1;
      const int n1 = pj.n1[qq];
      int cij[4], cii[4], cjj[4];
      load_pair(pj.case_pairs, ((int64_t)i * Mp + j) * Qp + qq, cij);
      load_pair(pj.case_pairs, ((int64_t)i * Mp + i) * Qp + qq, cii);
      load_pair(pj.case_pairs, ((int64_t)j * Mp + j) * Qp + qq, cjj);
      uint32_t kmin = 0xffffffffu, kmax = 0u;
#pragma unroll
      for (int tt = 0; tt < kPermT; ++tt) {
        int send[8], recv[8];
#pragma unroll
        for (int x = 0; x < 8; ++x) send[x] = h ? acc[tt][qb][x] : acc[tt][qb][8 + x];
#pragma unroll
        for (int x = 0; x < 8; ++x) recv[x] = __shfl_xor(send[x], 32);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int tg = 2 * h + u;                 // triplet within the row tile
          const int k = kbase + 4 * tt + tg;
          uint32_t cn[8], tn[8];
#pragma unroll
          for (int bc = 0; bc < 4; ++bc) {
            const int own = h ? acc[tt][qb][8 + 4 * u + bc] : acc[tt][qb][4 * u + bc];
            const int oth = recv[4 * u + bc];
            cn[bc] = (uint32_t)(h ? oth : own);      // a = 0
            cn[4 + bc] = (uint32_t)(h ? own : oth);  // a = 1
          }
#pragma unroll
          for (int x = 0; x < 8; ++x) tn[x] = myTot[tt * 32 + 8 * tg + x];
          int tik[4], tjk[4], tkk[4], cik[4], cjk[4], ckk[4];
          load_pair(pj.tot_pairs, (int64_t)i * Mp + k, tik);
          load_pair(pj.tot_pairs, (int64_t)j * Mp + k, tjk);
          load_pair(pj.tot_pairs, (int64_t)k * Mp + k, tkk);
          load_pair(pj.case_pairs, ((int64_t)i * Mp + k) * Qp + qq, cik);
          load_pair(pj.case_pairs, ((int64_t)j * Mp + k) * Qp + qq, cjk);
          load_pair(pj.case_pairs, ((int64_t)k * Mp + k) * Qp + qq, ckk);
          int ttab[27], ctab[27];
          {
            const int mi[2] = {tii[0], tii[3]}, mj[2] = {tjj[0], tjj[3]}, mk[2] = {tkk[0], tkk[3]};
            complete_table(tn, tij, tik, tjk, mi, mj, mk, pj.N, ttab);
          }
          {
            const int mi[2] = {cii[0], cii[3]}, mj[2] = {cjj[0], cjj[3]}, mk[2] = {ckk[0], ckk[3]};
            complete_table(cn, cij, cik, cjk, mi, mj, mk, n1, ctab);
          }
          float k2 = 0.f;
#pragma unroll
          for (int x = 0; x < 27; ++x) {
            const int r1 = ctab[x], r0 = ttab[x] - ctab[x];
            k2 += sL[ttab[x] + 1] - (sL[r0] + sL[r1]);
          }
          if (qvalid && k < M) {
            pj.score[(int64_t)q * T + lex_base(M, i, j) + k] = k2;
            const uint32_t key = f2key(k2);
            kmin = key < kmin ? key : kmin;
            kmax = key > kmax ? key : kmax;
          }
        }
      }
      // per-phenotype key range: lanes q and q + 32 hold the same q
      const uint32_t omin = __shfl_xor(kmin, 32), omax = __shfl_xor(kmax, 32);
      kmin = omin < kmin ? omin : kmin;
      kmax = omax > kmax ? omax : kmax;
      if (h == 0 && qvalid && kmax != 0u) {
        atomicMin(&st[q].kmin, kmin);
        atomicMax(&st[q].kmax, kmax);
      }
    }
    __builtin_amdgcn_wave_barrier();
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
  const size_t lds = (size_t)((lf_len + 3) & ~3) * sizeof(float) + 4 * kPermT * 32 * sizeof(uint32_t);
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(&count_mfma_perm_kernel),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, count_mfma_perm_kernel, 256, lds);
  if (e != hipSuccess) return e;
  if (per_cu <= 0) per_cu = 1;
  int64_t blocks = (int64_t)n_cu * per_cu;
  const int64_t need = (n_tiles + 3) / 4;
  if (blocks > need) blocks = need > 0 ? need : 1;
  hipLaunchKernelGGL(count_mfma_perm_kernel, dim3((unsigned)blocks), dim3(256), lds, s, pj_dev, st,
                     queue, lf32, lf_len);
  return hipGetLastError();
}

}  // namespace epi3
