// Fourth-order scan: K2 of every quad of SNPs.
//
// Eq. 1 holds for any number of interacting SNPs; for quads the table has
// 3^4 = 81 rows per class.  Per class and quad the 16 cells with all four
// genotypes in {0, 1} and the 8 corner cells of each of the four sub-triplets
// are counted by AND + POPCNT over the class's words (the paper's table
// filling, Alg. 2, with one more SNP); the rest follow by inclusion-exclusion
// (quad_cells).  One thread per quad, quads by lexicographic rank, so the
// lanes of a wave share (i, j, k) and read consecutive l.
#include "epi3_internal.h"

namespace epi3 {
namespace {

template <bool LDS>
__global__ void __launch_bounds__(256) quad_scores_kernel(
    const uint32_t *__restrict__ planes, const int32_t *__restrict__ pairs, int32_t M, int32_t Mp,
    int32_t W0, int32_t W1, int32_t N0, int32_t N1, const float *__restrict__ lf32, int32_t lf_len,
    int64_t Q, float *__restrict__ score, uint32_t *__restrict__ keyrange) {
  extern __shared__ float tab[];
  const float *L = lf32;
  if (LDS) {
    for (int x = threadIdx.x; x < lf_len; x += blockDim.x) tab[x] = lf32[x];
    __syncthreads();
    L = tab;
  }
  const int64_t MpMp4 = (int64_t)Mp * Mp * 4;
  uint32_t kmin = 0xffffffffu, kmax = 0u;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Q;
       r += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k, l;
    decode_quad_rank(M, r, i, j, k, l);
    uint32_t cnt[48];
    int t0[81], t1[81];
    quad_counts(planes, Mp, 0, W0, 1, i, j, k, l, cnt);
    quad_cells(cnt, pairs, Mp, i, j, k, l, N0, t0);
    quad_counts(planes, Mp, W0, W0 + W1, 1, i, j, k, l, cnt);
    quad_cells(cnt, pairs + MpMp4, Mp, i, j, k, l, N1, t1);
    float k2 = 0.f;  // rows in order: L[r + 1] - (L[r_0] + L[r_1])
#pragma unroll
    for (int x = 0; x < 81; ++x) {
      const int r0 = t0[x], r1 = t1[x];
      k2 += L[r0 + r1 + 1] - (L[r0] + L[r1]);
    }
    score[r] = k2;
    const uint32_t key = f2key(k2);
    kmin = key < kmin ? key : kmin;
    kmax = key > kmax ? key : kmax;
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
hipError_t launch_quad_scores_t(const epi3_dataset &d, float *score, uint32_t *keyrange,
                                hipStream_t s) {
  const int M = d.n_snps;
  const int64_t Q = c4(M);
  const int lf_len = d.n_samples + 2;
  const int lds = LDS ? lf_len * 4 : 0;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&quad_scores_kernel<LDS>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  int dev = 0, n_cu = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, quad_scores_kernel<LDS>, 256, lds);
  if (e != hipSuccess) return e;
  int64_t blocks = (int64_t)n_cu * (per_cu > 0 ? per_cu : 1) * 4;
  const int64_t need = (Q + 255) / 256;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL(quad_scores_kernel<LDS>, dim3((unsigned)blocks), dim3(256), lds, s,
                     static_cast<const uint32_t *>(d.planes), d.pairs, M, d.snp_stride, d.words[0],
                     d.words[1], d.n_controls, d.n_cases, d.lf32, lf_len, Q, score, keyrange);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_quad_scores(const epi3_dataset &d, float *score, uint32_t *keyrange,
                              hipStream_t s) {
  if (d.n_snps < 4) return hipSuccess;
  return lf_in_lds(d.n_samples + 2) ? launch_quad_scores_t<true>(d, score, keyrange, s)
                                    : launch_quad_scores_t<false>(d, score, keyrange, s);
}

}  // namespace epi3
