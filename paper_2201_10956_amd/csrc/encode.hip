// Encoding kernels: genotype bytes -> per-genotype sample bit-planes, byte
// planes for the matrix-core path, and pairwise tables.
//
// Binarized format (Problem Formulation section, Fig. 1 text): SNP x is held
// as one bit-plane per genotype value, one bit per sample.  Reduced format
// (CPU approaches section): plane 2 is never stored because a sample is in
// plane 2 exactly when it is in neither plane 0 nor plane 1, and samples are
// split into a controls array and a cases array.  32-bit words (start of the
// Approaches section).  SNP-minor order (GPU approaches section: consecutive
// SNPs adjacent in memory so that lanes owning consecutive SNPs coalesce).
#include "epi3_internal.h"

namespace epi3 {

// planes[w][m][0..1]: bit b of word w = sample list[w * 32 + b] has genotype
// 0 (plane 0) / 1 (plane 1).  list < 0 marks padding; padding bits stay 0 in
// both planes.  SNP slots m >= M are zero.  One wave per SNP and group of 64
// words: per step the 64 lanes read the genotype bytes of 64 consecutive
// list positions (two words; within a class the list is in sample order, so
// the reads fall in a few cache lines of the SNP's row) and two ballots form
// both planes of both words.
constexpr int kEncWords = 64;  // words per wave

__global__ void __launch_bounds__(256) encode_kernel(const uint8_t *__restrict__ geno, int64_t ld,
                                                     const int32_t *__restrict__ list, int32_t M,
                                                     int32_t Mp, int32_t Wtot,
                                                     uint32_t *__restrict__ planes,
                                                     int32_t *__restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int m = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (m >= Mp) return;
  const int w0 = blockIdx.y * kEncWords;
  const uint8_t *row = geno + (int64_t)(m < M ? m : 0) * ld;
  uint2 *out = reinterpret_cast<uint2 *>(planes);
  bool bad = false;
  for (int w = w0; w < w0 + kEncWords && w < Wtot; w += 2) {
    const int wl = w + (lane >> 5);  // this lane's word
    int g = 3;                       // no genotype: padding, SNP slot >= M, word >= Wtot
    if (m < M && wl < Wtot) {
      const int sidx = list[(int64_t)wl * 32 + (lane & 31)];
      if (sidx >= 0) {
        g = row[sidx];
        bad |= g > 2;
      }
    }
    const unsigned long long z = __ballot(g == 0), o = __ballot(g == 1);
    if (lane == 0) out[(int64_t)w * Mp + m] = make_uint2((uint32_t)z, (uint32_t)o);
    if (lane == 32 && w + 1 < Wtot)
      out[(int64_t)(w + 1) * Mp + m] = make_uint2((uint32_t)(z >> 32), (uint32_t)(o >> 32));
  }
  if (__ballot(bad) != 0ull && lane == 0) atomicOr(status, 1);
}

// bytes[m][p][s] = 1 if sample s of SNP m has genotype p (p = 0, 1), else 0;
// samples s >= N and SNPs m >= M are 0.  S is a multiple of 4.
__global__ void __launch_bounds__(256) encode_bytes_kernel(const uint8_t *__restrict__ geno,
                                                           int64_t ld, int32_t M, int32_t N,
                                                           int32_t Mp, int32_t S,
                                                           uint32_t *__restrict__ bytes) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;  // dword within a row
  const int S4 = S >> 2;
  if (q >= S4) return;
  for (int m = blockIdx.y; m < Mp; m += gridDim.y) {
    uint32_t v0 = 0, v1 = 0;
    if (m < M) {
      const uint8_t *row = geno + (int64_t)m * ld;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int s = 4 * q + b;
        if (s < N) {
          const uint32_t g = row[s];
          v0 |= (uint32_t)(g == 0u) << (8 * b);
          v1 |= (uint32_t)(g == 1u) << (8 * b);
        }
      }
    }
    bytes[((int64_t)m * 2 + 0) * S4 + q] = v0;
    bytes[((int64_t)m * 2 + 1) * S4 + q] = v1;
  }
}

// nib[m][p][s / 2]: E2M1 value 1.0 (nibble 0x2) if sample s of SNP m has
// genotype p, else 0.0; samples 2d and 2d + 1 share byte d (low nibble first).
__global__ void __launch_bounds__(256) encode_nibbles_kernel(const uint8_t *__restrict__ geno,
                                                             int64_t ld, int32_t M, int32_t N,
                                                             int32_t Mp, int32_t S,
                                                             uint32_t *__restrict__ nib) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;  // dword of a row: 8 samples
  const int S8 = S >> 3;
  if (q >= S8) return;
  for (int m = blockIdx.y; m < Mp; m += gridDim.y) {
    uint32_t v0 = 0, v1 = 0;
    if (m < M) {
      const uint8_t *row = geno + (int64_t)m * ld;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int s = 8 * q + b;
        if (s < N) {
          const uint32_t g = row[s];
          v0 |= (uint32_t)(g == 0u) << (4 * b + 1);
          v1 |= (uint32_t)(g == 1u) << (4 * b + 1);
        }
      }
    }
    nib[((int64_t)m * 2 + 0) * S8 + q] = v0;
    nib[((int64_t)m * 2 + 1) * S8 + q] = v1;
  }
}

// Per-class 0/1 value planes for the matrix cores, through the class sample
// list: position p of class c is sample list[off_c + p] (p < len_c), else
// padding.  bytes[c][m][g][p] = 1 and nib[c][m][g][p / 2] nibble = 0x2 (E2M1
// 1.0) when that sample has genotype g in {0, 1}; padding and SNPs m >= M
// are 0.  One thread per 8 positions.
__global__ void __launch_bounds__(256) encode_values_kernel(
    const uint8_t *__restrict__ geno, int64_t ld, const int32_t *__restrict__ list, int32_t off0,
    int32_t len0, int32_t off1, int32_t len1, int32_t M, int32_t Mp, int32_t S,
    uint32_t *__restrict__ bytes, uint32_t *__restrict__ nib) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;  // positions 8q .. 8q + 7
  if (q >= S / 8) return;
  const int c = blockIdx.z;
  const int off = c ? off1 : off0, len = c ? len1 : len0;
  for (int m = blockIdx.y; m < Mp; m += gridDim.y) {
    uint32_t b0[2] = {0, 0}, b1[2] = {0, 0}, n0 = 0, n1 = 0;
    if (m < M) {
      const uint8_t *row = geno + (int64_t)m * ld;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int p = 8 * q + b;
        if (p < len) {
          const uint32_t g = row[list[off + p]];
          const uint32_t is0 = g == 0u, is1 = g == 1u;
          b0[b >> 2] |= is0 << (8 * (b & 3));
          b1[b >> 2] |= is1 << (8 * (b & 3));
          n0 |= is0 << (4 * b + 1);
          n1 |= is1 << (4 * b + 1);
        }
      }
    }
    const int64_t rb = ((int64_t)c * Mp + m) * 2;  // row of (class, snp, plane 0)
    reinterpret_cast<uint2 *>(bytes)[(rb + 0) * (S / 8) + q] = make_uint2(b0[0], b0[1]);
    reinterpret_cast<uint2 *>(bytes)[(rb + 1) * (S / 8) + q] = make_uint2(b1[0], b1[1]);
    nib[(rb + 0) * (S / 8) + q] = n0;
    nib[(rb + 1) * (S / 8) + q] = n1;
  }
}

// Pairwise tables out[c][x][y] = (n00, n01, n10, n11), n_ab = number of
// samples of class c with genotype a at SNP x and b at SNP y (a, b in {0, 1}),
// by AND + POPCNT over the class's words (the MASKED layout's case tables
// restrict x to the mask's samples).  The diagonal holds the per-SNP counts
// (n_x(0), 0, 0, n_x(1)).  Workgroup tile: 64 x by 64 y, 16 x per
// wave read as wave-uniform scalars, y = lane; a word of y planes feeds 64
// AND + 64 popcounts.  Only tiles on or above the diagonal count; each writes
// (x, y) and its mirror (y, x) = (n00, n10, n01, n11).
constexpr int kPairX = 16;  // x rows per wave

__global__ void __launch_bounds__(256) pairs_kernel(const uint32_t *__restrict__ planes, int32_t Mp,
                                                    int32_t W0, int32_t W1,
                                                    const uint32_t *__restrict__ mask,
                                                    int32_t *__restrict__ pairs) {
  const int xb = blockIdx.y, yb = blockIdx.x;
  if (yb < xb) return;  // below the diagonal: written as mirrors
  const int lane = threadIdx.x & 63;
  const int x0 = __builtin_amdgcn_readfirstlane(xb * 64 + (threadIdx.x >> 6) * kPairX);
  const int y = yb * 64 + lane;
  const int c = blockIdx.z;
  const int w0 = c == 0 ? 0 : W0;
  const int w1 = c == 0 ? W0 : W0 + W1;
  uint32_t acc[kPairX][4];
#pragma unroll
  for (int r = 0; r < kPairX; ++r) acc[r][0] = acc[r][1] = acc[r][2] = acc[r][3] = 0u;
  cptr<uint32_t> pc = as_const(planes);
  const uint2 *pv = reinterpret_cast<const uint2 *>(planes);
  for (int w = w0; w < w1; ++w) {
    const uint2 yv = pv[(int64_t)w * Mp + y];
    const uint32_t mk = mask ? as_const(mask)[w] : 0xffffffffu;
    cptr<uint32_t> xr = pc + ((int64_t)w * Mp + x0) * 2;
#pragma unroll
    for (int r = 0; r < kPairX; ++r) {
      const uint32_t a0 = xr[2 * r] & mk, a1 = xr[2 * r + 1] & mk;
      acc[r][0] += __builtin_popcount(a0 & yv.x);
      acc[r][1] += __builtin_popcount(a0 & yv.y);
      acc[r][2] += __builtin_popcount(a1 & yv.x);
      acc[r][3] += __builtin_popcount(a1 & yv.y);
    }
  }
  int4 *out = reinterpret_cast<int4 *>(pairs) + (int64_t)c * Mp * Mp;
#pragma unroll
  for (int r = 0; r < kPairX; ++r) {
    const int x = x0 + r;
    out[(int64_t)x * Mp + y] = make_int4((int)acc[r][0], (int)acc[r][1], (int)acc[r][2], (int)acc[r][3]);
    if (y != x)
      out[(int64_t)y * Mp + x] = make_int4((int)acc[r][0], (int)acc[r][2], (int)acc[r][1], (int)acc[r][3]);
  }
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x)
    p[x] = v;
}

hipError_t launch_encode(const uint8_t *geno, int64_t ld, const int32_t *sample_list, int32_t M,
                         int32_t Mp, int32_t W0, int32_t W1, uint32_t *planes, int32_t *status,
                         hipStream_t s) {
  const int Wtot = W0 + W1;
  if (Wtot <= 0) return hipSuccess;
  dim3 grid((Mp + 3) / 4, (Wtot + kEncWords - 1) / kEncWords);
  hipLaunchKernelGGL(encode_kernel, grid, dim3(256), 0, s, geno, ld, sample_list, M, Mp, Wtot,
                     planes, status);
  return hipGetLastError();
}

hipError_t launch_encode_bytes(const uint8_t *geno, int64_t ld, int32_t M, int32_t N, int32_t Mp,
                               int32_t S, uint8_t *bytes, hipStream_t s) {
  const int S4 = S / 4;
  dim3 grid((S4 + 255) / 256, Mp < 65535 ? Mp : 65535);
  hipLaunchKernelGGL(encode_bytes_kernel, grid, dim3(256), 0, s, geno, ld, M, N, Mp, S,
                     reinterpret_cast<uint32_t *>(bytes));
  return hipGetLastError();
}

hipError_t launch_encode_nibbles(const uint8_t *geno, int64_t ld, int32_t M, int32_t N, int32_t Mp,
                                 int32_t S, uint8_t *nib, hipStream_t s) {
  const int S8 = S / 8;
  dim3 grid((S8 + 255) / 256, Mp < 65535 ? Mp : 65535);
  hipLaunchKernelGGL(encode_nibbles_kernel, grid, dim3(256), 0, s, geno, ld, M, N, Mp, S,
                     reinterpret_cast<uint32_t *>(nib));
  return hipGetLastError();
}

hipError_t launch_encode_values(const uint8_t *geno, int64_t ld, const int32_t *list, int32_t off0,
                                int32_t len0, int32_t off1, int32_t len1, int32_t classes,
                                int32_t M, int32_t Mp, int32_t S, uint8_t *bytes, uint8_t *nib,
                                hipStream_t s) {
  dim3 grid((S / 8 + 255) / 256, Mp < 65535 ? Mp : 65535, classes);
  hipLaunchKernelGGL(encode_values_kernel, grid, dim3(256), 0, s, geno, ld, list, off0, len0, off1,
                     len1, M, Mp, S, reinterpret_cast<uint32_t *>(bytes),
                     reinterpret_cast<uint32_t *>(nib));
  return hipGetLastError();
}

hipError_t launch_pairs(const uint32_t *planes, int32_t Mp, int32_t M, int32_t W0, int32_t W1,
                        int32_t n_classes, const uint32_t *mask, int32_t *pairs, hipStream_t s) {
  (void)M;
  if (Mp % 64 != 0) return hipErrorInvalidValue;  // tiles of 64 x 64 SNPs cover the stride exactly
  dim3 grid(Mp / 64, Mp / 64, n_classes);
  hipLaunchKernelGGL(pairs_kernel, grid, dim3(256), 0, s, planes, Mp, W0, W1, mask, pairs);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace epi3
