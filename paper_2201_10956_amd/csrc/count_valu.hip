// Count stage on the vector ALU: AND + popcount over bit-planes, fused with
// the FP32 K2 score.
//
// Paper, Alg. 2 and the GPU approaches section: every combination i < j < k
// gets a private frequency table in registers, filled over all samples of
// both classes, then scored.  Differences from the paper's kernel:
//   * a wave owns P pivot pairs (i, j) with j wave-uniform and 64 lanes own
//     64 consecutive k > j, so the pair words X_i[a] & X_j[b] are formed once
//     per 32 samples on the scalar unit and shared by all lanes;
//   * only the 8 cells with genotypes in {0,1}^3 are counted (8 AND + 8
//     v_bcnt per triplet and 32 samples); the other 19 cells of each class
//     follow exactly from the pairwise tables and the class size (every
//     sample falls in exactly one of the 27 rows), so the table is the same
//     integer table the paper fills with 27 AND/POPCNT per word;
//   * a persistent grid pulls tiles (job, j, i-block, k-block) from an atomic
//     queue, which also serves batches of data sets of different shape.
#include "epi3_internal.h"

namespace epi3 {

__device__ __forceinline__ int64_t rfl64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Tiles of pivot j: ceil(j / P) i-blocks x ceil((M - 1 - j) / 64) k-blocks.
__host__ __device__ __forceinline__ int64_t tiles_of_j(int64_t M, int64_t j, int P) {
  if (j < 1 || j > M - 2) return 0;
  return ((j + P - 1) / P) * ((M - 1 - j + 63) / 64);
}

// jprefix[j] = job-local tiles before pivot j, jprefix[M] = total; one block per job.
__global__ void __launch_bounds__(1024) tile_prefix_kernel(Job *jobs) {
  Job &J = jobs[blockIdx.x];
  const int64_t M = J.M;
  const int P = J.P;
  int64_t *pre = const_cast<int64_t *>(J.jprefix);
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (M + 1023) / 1024;
  const int64_t a = t * chunk, b = (a + chunk < M) ? a + chunk : M;
  int64_t sum = 0;
  for (int64_t j = a; j < b; ++j) sum += tiles_of_j(M, j, P);
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - sum;  // exclusive prefix of this chunk
  for (int64_t j = a; j < b; ++j) {
    pre[j] = run;
    run += tiles_of_j(M, j, P);
  }
  if (t == 1023) pre[M] = part[1023];
}

// acc + popcount(x) as one v_bcnt_u32_b32.  Written out because the compiler
// may otherwise reassociate the sums of an unrolled loop into v_bcnt(x, 0)
// plus v_add3, one more VALU op per two counts.
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
  return r;
}

// Accumulate the 8 corner cells of P pairs over words [w0, w1).
// acc[t][4a + 2b + c] += popcount(X_{i0+t}[a] & X_j[b] & X_k[c]).
template <int P>
__device__ __forceinline__ void accumulate(uint32_t (&acc)[P][8], const uint32_t *planes,
                                           int64_t Mp, int w0, int w1, int i0, int j, int k) {
  cptr<uint32_t> pc = as_const(planes);
  const uint2 *pv = reinterpret_cast<const uint2 *>(planes);
#pragma unroll 2
  for (int w = w0; w < w1; ++w) {
    const int64_t rowbase = (int64_t)w * Mp;
    const uint2 xk = pv[rowbase + k];
    const uint32_t xj0 = pc[(rowbase + j) * 2], xj1 = pc[(rowbase + j) * 2 + 1];
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const uint32_t xi0 = pc[(rowbase + i0 + t) * 2], xi1 = pc[(rowbase + i0 + t) * 2 + 1];
      const uint32_t p00 = xi0 & xj0, p01 = xi0 & xj1, p10 = xi1 & xj0, p11 = xi1 & xj1;
      acc[t][0] = bcnt_acc(p00 & xk.x, acc[t][0]);
      acc[t][1] = bcnt_acc(p00 & xk.y, acc[t][1]);
      acc[t][2] = bcnt_acc(p01 & xk.x, acc[t][2]);
      acc[t][3] = bcnt_acc(p01 & xk.y, acc[t][3]);
      acc[t][4] = bcnt_acc(p10 & xk.x, acc[t][4]);
      acc[t][5] = bcnt_acc(p10 & xk.y, acc[t][5]);
      acc[t][6] = bcnt_acc(p11 & xk.x, acc[t][6]);
      acc[t][7] = bcnt_acc(p11 & xk.y, acc[t][7]);
    }
  }
}

// One tile: P pivots i0 .. i0 + P - 1, pivot j, 64 lanes = 64 consecutive k.
template <int P, bool COUNTS>
__device__ __forceinline__ void valu_tile(cptr<Job> cj, int job, int j, int r, int lane,
                                          const float *sL) {
  const uint32_t *planes = cj[job].planes;
  const int32_t *pairs = cj[job].pairs;
  const int M = cj[job].M, Mp = cj[job].Mp;
  const int W0 = cj[job].W0, W1 = cj[job].W1;
  const int nkb = (M - 1 - j + 63) >> 6;
  const int ib = r / nkb, kb = r - ib * nkb;
  const int i0 = ib * P;
  const int k = j + 1 + kb * 64 + lane;

  uint32_t acc0[P][8], acc1[P][8];
#pragma unroll
  for (int x = 0; x < P; ++x)
#pragma unroll
    for (int y = 0; y < 8; ++y) acc0[x][y] = acc1[x][y] = 0u;
  accumulate<P>(acc0, planes, Mp, 0, W0, i0, j, k);
  accumulate<P>(acc1, planes, Mp, W0, W0 + W1, i0, j, k);

  // ---- epilogue: complete the tables, K2 in FP32, write ----
  const int N0 = cj[job].N0, N1 = cj[job].N1;
  float *score = cj[job].score;
  uint32_t *counts = cj[job].counts;
  const int64_t MpMp = (int64_t)Mp * Mp;
  const int4 *pr = reinterpret_cast<const int4 *>(pairs);
  const bool kvalid = k < M;
  uint32_t kmin = 0xffffffffu, kmax = 0u;
  int mk0[2], mk1[2];
  int4 pjk[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int4 kk = pr[c * MpMp + (int64_t)k * Mp + k];
    mk0[c] = kk.x;
    mk1[c] = kk.w;
    pjk[c] = pr[c * MpMp + (int64_t)j * Mp + k];
  }
  typedef int i4v __attribute__((ext_vector_type(4)));
  cptr<i4v> prc = as_const(reinterpret_cast<const i4v *>(pairs));
#pragma unroll
  for (int tt = 0; tt < P; ++tt) {
    const int i = i0 + tt;
    float k2 = 0.f;
    int tab[2][27];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const i4v pij = prc[c * MpMp + (int64_t)i * Mp + j];
      const i4v mii = prc[c * MpMp + (int64_t)i * Mp + i];
      const i4v mjj = prc[c * MpMp + (int64_t)j * Mp + j];
      const int4 pik = pr[c * MpMp + (int64_t)i * Mp + k];
      const int aij[4] = {pij.x, pij.y, pij.z, pij.w};
      const int aik[4] = {pik.x, pik.y, pik.z, pik.w};
      const int ajk[4] = {pjk[c].x, pjk[c].y, pjk[c].z, pjk[c].w};
      const int mi[2] = {mii.x, mii.w}, mj[2] = {mjj.x, mjj.w}, mk[2] = {mk0[c], mk1[c]};
      complete_table(c == 0 ? acc0[tt] : acc1[tt], aij, aik, ajk, mi, mj, mk, c == 0 ? N0 : N1,
                     tab[c]);
    }
#pragma unroll
    for (int x = 0; x < 27; ++x) {
      const int r0 = tab[0][x], r1 = tab[1][x];
      k2 += sL[r0 + r1 + 1] - (sL[r0] + sL[r1]);
    }
    if (i < j && kvalid) {
      const int64_t rank = lex_base(M, i, j) + k;
      score[rank] = k2;
      const uint32_t key = f2key(k2);
      kmin = key < kmin ? key : kmin;
      kmax = key > kmax ? key : kmax;
      if (COUNTS) {
        uint32_t *o = counts + rank * 54;
#pragma unroll
        for (int x = 0; x < 27; ++x) {
          o[x] = (uint32_t)tab[0][x];
          o[27 + x] = (uint32_t)tab[1][x];
        }
      }
    }
  }
  // wave-reduce the key range, one atomic per tile
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t a = __shfl_xor(kmin, off), b = __shfl_xor(kmax, off);
    kmin = a < kmin ? a : kmin;
    kmax = b > kmax ? b : kmax;
  }
  if (lane == 0 && kmax != 0u) {
    atomicMin(cj[job].keyrange, kmin);
    atomicMax(cj[job].keyrange + 1, kmax);
  }
}

// Persistent grid over the tiles of every job; a job's tiles use its own P
// (PA or PB: one kernel serves a batch whose data sets prefer different P).
template <int PA, int PB, bool COUNTS, bool LDS>
__global__ void __launch_bounds__(256) count_valu_kernel(const Job *__restrict__ jobs, int n_jobs,
                                                         int64_t total_tiles,
                                                         unsigned long long *__restrict__ queue,
                                                         const float *__restrict__ lf32,
                                                         int lf_len) {
  extern __shared__ float sLds[];
  const float *sL = lf32;
  if (LDS) {
    for (int x = threadIdx.x; x < lf_len; x += blockDim.x) sLds[x] = lf32[x];
    __syncthreads();
    sL = sLds;
  }

  const int lane = threadIdx.x & 63;
  cptr<Job> cj = as_const(jobs);
  int job = -1;
  int64_t jb_begin = 0, jb_end = 0;
  int j = -1;
  int64_t jlo = 0, jhi = 0;

  for (;;) {
    unsigned long long got = 0;
    if (lane == 0) got = atomicAdd(queue, 1ull);
    const int64_t t = rfl64((int64_t)got);
    if (t >= total_tiles) break;
    if (t < jb_begin || t >= jb_end) {
      int lo = 0, hi = n_jobs - 1;  // last job whose first tile is <= t
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cj[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
      }
      job = lo;
      jb_begin = cj[job].tile_begin;
      jb_end = jb_begin + cj[job].n_tiles;
      jlo = jhi = 0;
      j = -1;
    }
    const int M = cj[job].M;
    const int64_t local = t - jb_begin;
    if (j < 0 || local < jlo || local >= jhi) {
      cptr<int64_t> pre = as_const(cj[job].jprefix);
      int lo = 0, hi = M - 1;  // last pivot whose first tile is <= local
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= local) lo = mid; else hi = mid - 1;
      }
      j = lo;
      jlo = pre[j];
      jhi = pre[j + 1];
    }
    const int r = (int)(local - jlo);
    if (PA == PB || cj[job].P == PA)
      valu_tile<PA, COUNTS>(cj, job, j, r, lane, sL);
    else
      valu_tile<PB, COUNTS>(cj, job, j, r, lane, sL);
  }
}

hipError_t launch_tile_prefix(Job *jobs_dev, int32_t n_jobs, hipStream_t s) {
  hipLaunchKernelGGL(tile_prefix_kernel, dim3(n_jobs), dim3(1024), 0, s, jobs_dev);
  return hipGetLastError();
}

__global__ void write_jobs_kernel(Job j0, Job *dst) { if (threadIdx.x == 0) *dst = j0; }

hipError_t launch_write_jobs(const Job *jobs_host, int32_t n, Job *dst_dev, hipStream_t s) {
  for (int x = 0; x < n; ++x)
    hipLaunchKernelGGL(write_jobs_kernel, dim3(1), dim3(64), 0, s, jobs_host[x], dst_dev + x);
  return hipGetLastError();
}

template <int PA, int PB, bool C, bool LDS>
static hipError_t launch_valu_l(const Job *jobs_dev, int32_t n_jobs, int64_t total_tiles,
                                unsigned long long *queue, const float *lf32, int32_t lf_len,
                                hipStream_t s) {
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const size_t lds = LDS ? (size_t)lf_len * sizeof(float) : 0;
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(&count_valu_kernel<PA, PB, C, LDS>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, count_valu_kernel<PA, PB, C, LDS>, 256,
                                                   lds);
  if (e != hipSuccess) return e;
  if (per_cu <= 0) per_cu = 1;
  int64_t blocks = (int64_t)n_cu * per_cu;
  const int64_t need = (total_tiles + 3) / 4;
  if (blocks > need) blocks = need > 0 ? need : 1;
  hipLaunchKernelGGL((count_valu_kernel<PA, PB, C, LDS>), dim3((unsigned)blocks), dim3(256), lds, s,
                     jobs_dev, n_jobs, total_tiles, queue, lf32, lf_len);
  return hipGetLastError();
}

template <int PA, int PB, bool C>
static hipError_t launch_valu_t(const Job *jobs_dev, int32_t n_jobs, int64_t total_tiles,
                                unsigned long long *queue, const float *lf32, int32_t lf_len,
                                hipStream_t s) {
  return lf_in_lds(lf_len)
             ? launch_valu_l<PA, PB, C, true>(jobs_dev, n_jobs, total_tiles, queue, lf32, lf_len, s)
             : launch_valu_l<PA, PB, C, false>(jobs_dev, n_jobs, total_tiles, queue, lf32, lf_len, s);
}

hipError_t launch_count_valu(const Job *jobs_dev, int32_t n_jobs, int64_t total_tiles,
                             unsigned long long *queue, const float *lf32, int32_t lf_len,
                             int32_t P_lo, int32_t P_hi, bool counts, hipStream_t s) {
  if (P_lo != P_hi) {  // mixed batch (never with tables)
    if (counts) return hipErrorInvalidValue;
    return launch_valu_t<8, 4, false>(jobs_dev, n_jobs, total_tiles, queue, lf32, lf_len, s);
  }
  if (P_lo == 4)
    return counts ? launch_valu_t<4, 4, true>(jobs_dev, n_jobs, total_tiles, queue, lf32, lf_len, s)
                  : launch_valu_t<4, 4, false>(jobs_dev, n_jobs, total_tiles, queue, lf32, lf_len, s);
  return counts ? launch_valu_t<8, 8, true>(jobs_dev, n_jobs, total_tiles, queue, lf32, lf_len, s)
                : launch_valu_t<8, 8, false>(jobs_dev, n_jobs, total_tiles, queue, lf32, lf_len, s);
}

int64_t host_tiles(int64_t M, int P) {
  int64_t n = 0;
  for (int64_t j = 0; j < M; ++j) n += tiles_of_j(M, j, P);
  return n;
}

int tile_P_default(int32_t M, int32_t N) {
  (void)N;
  return M >= 256 ? 8 : 4;
}

}  // namespace epi3
