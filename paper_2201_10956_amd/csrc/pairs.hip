// Second-order scan: K2 of every pair of SNPs.
//
// Eq. 1 holds for any number of interacting SNPs (I = 3^k rows); for pairs
// the table has 9 rows per class.  Its four cells with both genotypes in
// {0, 1} are the pairwise tables that encoding counts for the triplet scan
// (AND + POPCNT of the two SNPs' planes over the class's words), and the
// other five follow from the per-SNP counts (the diagonal of the pairwise
// tables) and the class size.  So scoring a pair is table completion and 27
// lookups; the counting itself happened at encoding.
#include "epi3_internal.h"

namespace epi3 {
namespace {

// Persistent workgroups, rows i round robin, thread per j > i: FP32 K2 by
// lexicographic pair rank (rows in order, each L[r + 1] - (L[r_0] + L[r_1]))
// and the scores' key range.  LDS: the log-factorial table, loaded once per
// workgroup.
template <bool LDS>
__global__ void __launch_bounds__(256) pair_scores_kernel(const int32_t *__restrict__ pairs,
                                                          int32_t M, int32_t Mp, int32_t N0,
                                                          int32_t N1, const float *__restrict__ lf32,
                                                          int32_t lf_len, float *__restrict__ score,
                                                          uint32_t *__restrict__ keyrange) {
  extern __shared__ float tab[];
  const float *L = lf32;
  if (LDS) {
    for (int x = threadIdx.x; x < lf_len; x += blockDim.x) tab[x] = lf32[x];
    __syncthreads();
    L = tab;
  }
  const int4 *pr = reinterpret_cast<const int4 *>(pairs);
  const int64_t MpMp = (int64_t)Mp * Mp;
  uint32_t kmin = 0xffffffffu, kmax = 0u;
  for (int i = blockIdx.x; i < M - 1; i += gridDim.x) {
    const int4 ii[2] = {pr[(int64_t)i * Mp + i], pr[MpMp + (int64_t)i * Mp + i]};
    const int64_t base = pair_rank(M, i, i + 1) - (i + 1);
    for (int j = i + 1 + threadIdx.x; j < M; j += blockDim.x) {
      int t[2][9];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int4 p = pr[c * MpMp + (int64_t)i * Mp + j];
        const int4 jj = pr[c * MpMp + (int64_t)j * Mp + j];
        const int n[4] = {p.x, p.y, p.z, p.w};
        const int mi[2] = {ii[c].x, ii[c].w}, mj[2] = {jj.x, jj.w};
        pair_cells(n, mi, mj, c ? N1 : N0, t[c]);
      }
      float k2 = 0.f;
#pragma unroll
      for (int x = 0; x < 9; ++x) {
        const int r0 = t[0][x], r1 = t[1][x];
        k2 += L[r0 + r1 + 1] - (L[r0] + L[r1]);
      }
      score[base + j] = k2;
      const uint32_t key = f2key(k2);
      kmin = key < kmin ? key : kmin;
      kmax = key > kmax ? key : kmax;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t a = __shfl_xor(kmin, off), b = __shfl_xor(kmax, off);
    kmin = a < kmin ? a : kmin;
    kmax = b > kmax ? b : kmax;
  }
  if ((threadIdx.x & 63) == 0 && kmax != 0u) {
    atomicMin(&keyrange[0], kmin);
    atomicMax(&keyrange[1], kmax);
  }
}

template <bool LDS>
hipError_t launch_pair_scores_t(const epi3_dataset &d, float *score, uint32_t *keyrange,
                                hipStream_t s) {
  const int M = d.n_snps;
  const int lf_len = d.n_samples + 2;
  const int lds = LDS ? lf_len * 4 : 0;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&pair_scores_kernel<LDS>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  int dev = 0, n_cu = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pair_scores_kernel<LDS>, 256, lds);
  if (e != hipSuccess) return e;
  int64_t blocks = (int64_t)n_cu * (per_cu > 0 ? per_cu : 1);
  if (blocks > M - 1) blocks = M - 1;
  hipLaunchKernelGGL(pair_scores_kernel<LDS>, dim3((unsigned)blocks), dim3(256), lds, s, d.pairs,
                     M, d.snp_stride, d.n_controls, d.n_cases, d.lf32, lf_len, score, keyrange);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pair_scores(const epi3_dataset &d, float *score, uint32_t *keyrange,
                              hipStream_t s) {
  if (d.n_snps < 2) return hipSuccess;
  return lf_in_lds(d.n_samples + 2) ? launch_pair_scores_t<true>(d, score, keyrange, s)
                                    : launch_pair_scores_t<false>(d, score, keyrange, s);
}

}  // namespace epi3
