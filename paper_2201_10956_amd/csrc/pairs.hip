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

// Block row i, thread per j > i: FP32 K2 by lexicographic pair rank (rows in
// order, each L[r + 1] - (L[r_0] + L[r_1])) and the score's key range.
__global__ void __launch_bounds__(256) pair_scores_kernel(const int32_t *__restrict__ pairs,
                                                          int32_t M, int32_t Mp, int32_t N0,
                                                          int32_t N1, const float *__restrict__ lf32,
                                                          float *__restrict__ score,
                                                          uint32_t *__restrict__ keyrange) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t kmin = 0xffffffffu, kmax = 0u;
  if (j > i && j < M) {
    const int4 *pr = reinterpret_cast<const int4 *>(pairs);
    int t[2][9];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int64_t cb = (int64_t)c * Mp * Mp;
      const int4 p = pr[cb + (int64_t)i * Mp + j];
      const int4 ii = pr[cb + (int64_t)i * Mp + i], jj = pr[cb + (int64_t)j * Mp + j];
      const int n[4] = {p.x, p.y, p.z, p.w};
      const int mi[2] = {ii.x, ii.w}, mj[2] = {jj.x, jj.w};
      pair_cells(n, mi, mj, c ? N1 : N0, t[c]);
    }
    float k2 = 0.f;
#pragma unroll
    for (int x = 0; x < 9; ++x) {
      const int r0 = t[0][x], r1 = t[1][x];
      k2 += lf32[r0 + r1 + 1] - (lf32[r0] + lf32[r1]);
    }
    score[pair_rank(M, i, j)] = k2;
    kmin = kmax = f2key(k2);
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

}  // namespace

hipError_t launch_pair_scores(const epi3_dataset &d, float *score, uint32_t *keyrange,
                              hipStream_t s) {
  const int M = d.n_snps;
  if (M < 2) return hipSuccess;
  dim3 grid((unsigned)((M + 255) / 256), (unsigned)(M - 1));
  hipLaunchKernelGGL(pair_scores_kernel, grid, dim3(256), 0, s, d.pairs, M, d.snp_stride,
                     d.n_controls, d.n_cases, d.lf32, score, keyrange);
  return hipGetLastError();
}

}  // namespace epi3
