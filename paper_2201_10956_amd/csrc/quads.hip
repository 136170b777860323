// Fourth-order scan: K2 of every quad of SNPs.
//
// Eq. 1 holds for any number of interacting SNPs; for quads the table has
// 3^4 = 81 rows per class.  Per class and quad the 16 cells with all four
// genotypes in {0, 1} are counted by AND + POPCNT over the class's words (the
// paper's table filling, Alg. 2, with one more SNP); the 8 corner cells of
// each of the four sub-triplets come from a table counted once per triplet
// beforehand (they do not depend on the fourth SNP), and the rest follow by
// inclusion-exclusion (quad_cells).  One thread per quad, quads by
// lexicographic rank, so the lanes of a wave share (i, j, k) and read
// consecutive l.
#include "epi3_internal.h"

namespace epi3 {
namespace {

// Corner cells of every triplet per class: t3[c * T + rank] = cells
// 4 a + 2 b + c (a, b, c in {0, 1}) as 8 x 16 bits, two per word, low half
// first.  Thread per triplet.
__global__ void __launch_bounds__(256) triplet_corners_kernel(const uint32_t *__restrict__ planes,
                                                              int32_t M, int32_t Mp, int32_t W0,
                                                              int32_t W1, int64_t T,
                                                              uint4 *__restrict__ t3) {
  const uint2 *pv = reinterpret_cast<const uint2 *>(planes);
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < T;
       r += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    decode_rank(M, r, i, j, k);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint32_t n[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int w = c ? W0 : 0; w < (c ? W0 + W1 : W0); ++w) {
        const uint2 *row = pv + (int64_t)w * Mp;
        const uint2 xi = row[i], xj = row[j], xk = row[k];
        const uint32_t X[3][2] = {{xi.x, xi.y}, {xj.x, xj.y}, {xk.x, xk.y}};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const uint32_t ij = X[0][a] & X[1][b];
            n[4 * a + 2 * b] += __builtin_popcount(ij & X[2][0]);
            n[4 * a + 2 * b + 1] += __builtin_popcount(ij & X[2][1]);
          }
      }
      t3[c * T + r] = make_uint4(n[0] | (n[1] << 16), n[2] | (n[3] << 16), n[4] | (n[5] << 16),
                                 n[6] | (n[7] << 16));
    }
  }
}

__device__ __forceinline__ void unpack8(uint4 v, uint32_t *n) {
  n[0] = v.x & 0xffffu; n[1] = v.x >> 16; n[2] = v.y & 0xffffu; n[3] = v.y >> 16;
  n[4] = v.z & 0xffffu; n[5] = v.z >> 16; n[6] = v.w & 0xffffu; n[7] = v.w >> 16;
}

// T3: sub-triplet corners from the triplet table (else counted per quad).
template <bool LDS, bool T3>
__global__ void __launch_bounds__(256) quad_scores_kernel(
    const uint32_t *__restrict__ planes, const int32_t *__restrict__ pairs, int32_t M, int32_t Mp,
    int32_t W0, int32_t W1, int32_t N0, int32_t N1, const float *__restrict__ lf32, int32_t lf_len,
    int64_t Q, const uint4 *__restrict__ t3, int64_t T, float *__restrict__ score,
    uint32_t *__restrict__ keyrange) {
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
    auto counts = [&](int c) {
      const int w0 = c ? W0 : 0, w1 = c ? W0 + W1 : W0;
      if (T3) {
        quad_corner_counts(planes, Mp, w0, w1, i, j, k, l, cnt);
        const uint4 *tc = t3 + c * T;
        unpack8(tc[lex_base(M, i, j) + k], cnt + 16);
        unpack8(tc[lex_base(M, i, j) + l], cnt + 24);
        unpack8(tc[lex_base(M, i, k) + l], cnt + 32);
        unpack8(tc[lex_base(M, j, k) + l], cnt + 40);
      } else {
        quad_counts(planes, Mp, w0, w1, 1, i, j, k, l, cnt);
      }
    };
    counts(0);
    quad_cells(cnt, pairs, Mp, i, j, k, l, N0, t0);
    counts(1);
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

template <bool LDS, bool T3>
hipError_t launch_quad_scores_t(const epi3_dataset &d, const uint4 *t3, float *score,
                                uint32_t *keyrange, hipStream_t s) {
  const int M = d.n_snps;
  const int64_t Q = c4(M), T = c3(M);
  const int lf_len = d.n_samples + 2;
  const int lds = LDS ? lf_len * 4 : 0;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&quad_scores_kernel<LDS, T3>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  int dev = 0, n_cu = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (T3) {
    int64_t tb = (T + 255) / 256;
    if (tb > (int64_t)n_cu * 16) tb = (int64_t)n_cu * 16;
    hipLaunchKernelGGL(triplet_corners_kernel, dim3((unsigned)tb), dim3(256), 0, s,
                       static_cast<const uint32_t *>(d.planes), M, d.snp_stride, d.words[0],
                       d.words[1], T, const_cast<uint4 *>(t3));
  }
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, quad_scores_kernel<LDS, T3>, 256, lds);
  if (e != hipSuccess) return e;
  int64_t blocks = (int64_t)n_cu * (per_cu > 0 ? per_cu : 1) * 4;
  const int64_t need = (Q + 255) / 256;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL((quad_scores_kernel<LDS, T3>), dim3((unsigned)blocks), dim3(256), lds, s,
                     static_cast<const uint32_t *>(d.planes), d.pairs, M, d.snp_stride, d.words[0],
                     d.words[1], d.n_controls, d.n_cases, d.lf32, lf_len, Q, t3, T, score, keyrange);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_triplet_corners(const epi3_dataset &d, void *t3, hipStream_t s) {
  const int M = d.n_snps;
  const int64_t T = c3(M);
  if (T == 0) return hipSuccess;
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  int64_t tb = (T + 255) / 256;
  if (tb > (int64_t)n_cu * 16) tb = (int64_t)n_cu * 16;
  hipLaunchKernelGGL(triplet_corners_kernel, dim3((unsigned)tb), dim3(256), 0, s,
                     static_cast<const uint32_t *>(d.planes), M, d.snp_stride, d.words[0],
                     d.words[1], T, static_cast<uint4 *>(t3));
  return hipGetLastError();
}

hipError_t launch_quad_scores(const epi3_dataset &d, void *t3, float *score, uint32_t *keyrange,
                              hipStream_t s) {
  if (d.n_snps < 4) return hipSuccess;
  const uint4 *t = static_cast<const uint4 *>(t3);
  if (lf_in_lds(d.n_samples + 2))
    return t ? launch_quad_scores_t<true, true>(d, t, score, keyrange, s)
             : launch_quad_scores_t<true, false>(d, t, score, keyrange, s);
  return t ? launch_quad_scores_t<false, true>(d, t, score, keyrange, s)
           : launch_quad_scores_t<false, false>(d, t, score, keyrange, s);
}

}  // namespace epi3
