// Internal declarations shared by the HIP translation units of libepi3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "epi3.h"

namespace epi3 {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kSnpPad = 64;      // plane arrays hold roundup(M, 64) + 64 SNP slots
constexpr int kHistBins = 2048;  // radix-select bins per pass
constexpr int kHistPasses = 3;   // 3 x 11 bits >= 32-bit keys
// Sampled first bound: every kSampleStride-th block of kSampleBlock scores.
constexpr int kSampleBlock = 1024;
constexpr int kSampleStride = 32;
// Whether a selection over T scores for k hits starts from the sampled bound
// (the sample must hold comfortably more than k scores).
inline bool sample_select(int64_t T, int64_t k) { return T >= (1ll << 22) && k * 512 <= T; }

// Pointer into the constant address space: uniform loads through it become
// scalar (s_load) instructions.  Only used for memory no kernel writes while
// the reading kernel runs.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
  return (cptr<T>)p;
}

__host__ __device__ __forceinline__ int64_t c2(int64_t x) { return x < 2 ? 0 : x * (x - 1) / 2; }
__host__ __device__ __forceinline__ int64_t c3(int64_t x) {
  return x < 3 ? 0 : x * (x - 1) / 2 * (x - 2) / 3;
}

// Lexicographic rank of i < j < k < M among all triplets.
// Lexicographic rank of the pair (i, j), i < j < M.
__host__ __device__ __forceinline__ int64_t pair_rank(int64_t M, int64_t i, int64_t j) {
  return c2(M) - c2(M - i) + (j - i - 1);
}
__host__ __device__ __forceinline__ int64_t lex_base(int64_t M, int64_t i, int64_t j) {
  return c3(M) - c3(M - i) + c2(M - 1 - i) - c2(M - j) - j - 1;  // + k gives the rank
}

// Order-preserving map of a float to an unsigned key (and back).
__host__ __device__ __forceinline__ uint32_t f2key(float f) {
  uint32_t b;
  __builtin_memcpy(&b, &f, 4);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ __forceinline__ float key2f(uint32_t k) {
  uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  float f;
  __builtin_memcpy(&f, &b, 4);
  return f;
}

// One scan job as seen by the count kernels: a SPLIT data set, its score
// plane and its share of the global tile queue.
struct Job {
  const uint32_t *planes;  // [W0 + W1][Mp][2]
  const int32_t *pairs;    // [2][Mp][Mp][4]
  float *score;            // [T] FP32 K2 by lexicographic rank
  const int64_t *jprefix;  // [M + 1] job-local tiles before pivot j
  uint32_t *counts;        // optional [T][2][27]
  uint32_t *keyrange;      // [2] atomic min / max of f2key(score)
  int64_t tile_begin;      // first global tile of this job
  int64_t n_tiles;
  int64_t T;
  int32_t M, Mp, W0, W1, N0, N1;
  int32_t P;               // pivots i per tile (4 or 8)
  int32_t pad;
};

// Per-job radix-select state.
struct SelState {
  uint32_t kmin, kmax;     // key range of the score plane (written by the count kernel)
  uint32_t lo;             // lower end of the key window holding the k-th key
  int32_t shift;           // bin width of the current pass = 1 << shift
  uint64_t krem;           // 1-based rank of the k-th key inside the window
  uint32_t done;           // window collapsed to one key
  uint32_t kth;            // key of the k-th smallest score
  float thr;               // candidate threshold (FP32, rounded up)
  uint32_t overflow;       // candidates beyond capacity
  unsigned long long ncand;
  int64_t keff;            // min(k, T)
  int64_t T;
  int32_t k;
  uint32_t whi;            // last key of the current window (set with lo)
  float ub;                // compaction bound: last key of the first window + 2 e(N), as float
  uint32_t cmode;          // 1 once the compaction pass ran
  unsigned long long cn;   // keys <= ub found by the compaction pass
};

// One scored candidate.
struct CandRec {
  uint64_t key;            // bit pattern of the FP64 K2 (non-negative => ordered)
  int64_t rank;            // lexicographic rank (tie-break)
  uint32_t i, j, k, l;
  float k2f;
  double k2;
  uint32_t counts[162];     // [class][cells]: 27 (triplets), 9 (pairs) or 81 (quads) per class
};

// Phenotype batch for the matrix-core kernel: one MASKED data set and up to
// 64 phenotypes (case masks).
struct PermJob {
  const uint8_t *bytes;       // [Mp][2][S] 0/1 genotype values (bytes, or E2M1 nibbles)
  const uint8_t *ph;          // [64][S] 0/1 case values per phenotype (same format)
  const int32_t *tot_pairs;   // [Mp][Mp][4] pairwise tables over all samples
  const int32_t *case_pairs;  // [Mp][Mp][Qp] uint2 (n00 | n01 << 16, n10 | n11 << 16): pairwise tables
                              // over each phenotype's cases (y >= x)
  const int32_t *n1;          // [Qp] cases per phenotype
  float *score;               // [Q][T]
  const int64_t *jprefix;     // [M + 1]
  uint4 *corners;             // scratch: [pass tile][4 pivots i][16 k][64 q] 8 x uint16 case cells
  uint4 *totals;              // scratch: [pass tile][4 pivots i][16 k] 8 x uint16 all-sample cells
  int64_t n_tiles, T;
  int32_t M, Mp, S, N, Q, Qp;  // S: bytes per staged row (samples for bytes, samples / 2 for nibbles)
};

// Where the phenotype-batch finish kernel puts its FP32 scores.
enum { kPermOutPlane = 0, kPermOutSample = 1, kPermOutBounded = 2 };
struct PermOut {
  int32_t mode;          // kPermOut*
  int32_t pad;
  // sample: the launch's tiles are sample tiles sample_base + n; the score of
  // slot s (= 16 wave + kk) of sample tile m of phenotype q goes to
  // sample[q * sample_T + 64 m + s] (invalid slots keep what the buffer held)
  float *sample;
  int64_t sample_T;
  int64_t sample_base;
  // bounded: phenotype q appends (key, rank) of every score <= st[q].ub to
  // ckey / crank [q * ccap + pos], pos from st[q].cn
  uint32_t *ckey;
  int64_t *crank;
  int64_t ccap;
};

// Where the plain matrix-core finish kernel puts its FP32 scores (modes as
// for PermOut).  The launch's slots q are global tiles tile_begin + q stride.
struct PlainOut {
  int32_t mode;          // kPermOut*
  int32_t pad;
  int64_t stride;
  // sample: the score of triplet x (0 .. 4095, the tile's triplet order) of
  // slot q goes to sample[(sample_base + q) 4096 + x] (slots of no triplet
  // keep what the buffer held); its key range to range[0..1]
  float *sample;
  int64_t sample_base;
  uint32_t *range;
  // bounded: (key, rank) of every score <= st->ub appended to ckey / crank at
  // positions from st->cn (entries past ccap are dropped, st->cn still counts)
  SelState *st;
  uint32_t *ckey;
  int64_t *crank;
  int64_t ccap;
};

// Plain two-class scan on the matrix cores: one SPLIT data set, counted in
// passes of tiles whose corner cells go through a scratch buffer
// ([pass tile][class][16 i][JB j][256 / JB k] 8 x uint16 cells).
struct PlainJob {
  const uint8_t *vals;     // [2][Mp][2][Sb] 0/1 values per class (bytes, or E2M1 nibbles)
  const int32_t *pairs;    // [2][Mp][Mp][4]
  float *score;            // [T] FP32 K2 by lexicographic rank
  uint32_t *counts;        // optional [T][2][27]
  uint32_t *keyrange;      // [2] atomic min / max of f2key(score)
  const int64_t *jprefix;  // [M + 1] tiles before pivot j
  int64_t n_tiles, T;
  int32_t M, Mp, Sb, Sb0, Sb1, N0, N1, JB;  // Sb: bytes per row; Sb0 / Sb1: bytes holding each class
};

// Selection job: one score plane plus its candidate buffers.
struct SelJob {
  const float *score;
  int64_t T;
  SelState *st;
  uint32_t *hist;          // [kHistBins]
  int64_t *cand;           // [cap] ranks
  uint32_t *candkey;       // [cap] their FP32 score keys
  CandRec *rec;            // [cap]
  epi3_hit *hits;          // [k]
  int64_t cap;
  uint32_t *ckey;          // [ccap] keys of the compacted low end of the plane
  int64_t *crank;          // [ccap] their ranks
  int64_t ccap;
  double err2;             // 2 e(N)
  // data needed to recount a candidate
  const uint32_t *planes;
  const int32_t *pairs;    // [classes][Mp][Mp][4]; MASKED: totals at class 0
  const int32_t *case_pairs; // MASKED: case pairs (uint2, 16-bit counts) of the job's mask (pair (x,y) at
                             // uint2 index (x * Mp + y) * case_stride), else NULL
  const uint32_t *case_mask; // MASKED: [W] mask words, else NULL
  const int32_t *n1_dev;     // MASKED: device count of cases (overrides N1), else NULL
  int64_t case_stride;
  const double *lf64;
  int32_t M, Mp, W0, W1, N0, N1;
  int32_t layout;
  int32_t k;
  int32_t sample;          // 1: the first bound comes from a radix select on a sample (sample_select),
                           // or (score == NULL) from the batch's sample pass with the list already built
  int32_t order;           // 2: pairs (9-row tables, pair_hits); 4: quads (81 rows, quad_hits);
                           // else triplets
  epi3_pair_hit *pair_hits;  // [k] (order 2)
  epi3_quad_hit *quad_hits;  // [k] (order 4)
  // candidate capacities above kRankDirectMax order the candidates by a
  // bitonic sort of (FP64 key, index) pairs in these buffers of sortP entries
  // (a power of two >= cap) instead of counting, for each, the candidates
  // before it; sortP = 0 otherwise
  uint64_t *skey;
  uint32_t *sidx;
  int64_t sortP;
};

constexpr int64_t kRankDirectMax = 16384;
inline int64_t sort_len(int64_t cap) {
  if (cap <= kRankDirectMax) return 0;
  int64_t p = 1;
  while (p < cap) p <<= 1;
  return p;
}

// The 27 cells of one class from the 8 counted corner cells n[4a + 2b + c]
// (a, b, c in {0, 1}), the pairwise tables pij[2a + b], pik[2a + c],
// pjk[2b + c], the per-SNP counts mi[a], mj[b], mk[c] and the class size.
// Every sample of the class is in exactly one row, so each missing cell is
// a margin minus the cells already known.
__device__ __forceinline__ void complete_table(const uint32_t n[8], const int pij[4],
                                               const int pik[4], const int pjk[4], const int mi[2],
                                               const int mj[2], const int mk[2], int Nc, int t[27]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) t[9 * a + 3 * b + c] = (int)n[4 * a + 2 * b + c];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
      t[9 * a + 3 * b + 2] = pij[2 * a + b] - t[9 * a + 3 * b] - t[9 * a + 3 * b + 1];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
      t[9 * a + 6 + c] = pik[2 * a + c] - t[9 * a + c] - t[9 * a + 3 + c];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c)
      t[18 + 3 * b + c] = pjk[2 * b + c] - t[3 * b + c] - t[9 + 3 * b + c];
#pragma unroll
  for (int a = 0; a < 2; ++a)
    t[9 * a + 8] = mi[a] - pij[2 * a] - pij[2 * a + 1] - t[9 * a + 6] - t[9 * a + 7];
#pragma unroll
  for (int b = 0; b < 2; ++b)
    t[18 + 3 * b + 2] = mj[b] - pij[b] - pij[2 + b] - t[18 + 3 * b] - t[18 + 3 * b + 1];
#pragma unroll
  for (int c = 0; c < 2; ++c)
    t[24 + c] = mk[c] - pik[c] - pik[2 + c] - t[18 + c] - t[21 + c];
  int s = 0;
#pragma unroll
  for (int x = 0; x < 26; ++x) s += t[x];
  t[26] = Nc - s;
}

// The 9 cells t[3 a + b] of one class of a pair (a, b in {0, 1, 2}) from the
// counted cells n[2 a + b] (a, b in {0, 1}), the per-SNP counts mi[a], mj[b]
// and the class size: every sample of the class is in exactly one row.
__device__ __forceinline__ void pair_cells(const int n[4], const int mi[2], const int mj[2], int Nc,
                                           int t[9]) {
  t[0] = n[0];
  t[1] = n[1];
  t[3] = n[2];
  t[4] = n[3];
  t[2] = mi[0] - n[0] - n[1];
  t[5] = mi[1] - n[2] - n[3];
  t[6] = mj[0] - n[0] - n[2];
  t[7] = mj[1] - n[1] - n[3];
  t[8] = Nc - (t[0] + t[1] + t[2] + t[3] + t[4] + t[5] + t[6] + t[7]);
}

// Counts of one class of the quad (i, j, k, l) over words [w0, w1) with
// stride `step` (one thread: 1; the lanes of a wave: 64 from w0 + lane):
// cnt[8 a + 4 b + 2 c + d] = sum popc(X_i[a] & X_j[b] & X_k[c] & X_l[d]),
// then the corner cells of the four sub-triplets, each indexed by its own
// (x, y, z) in {0, 1}^3 as 4 x + 2 y + z: cnt[16 + ...] (i, j, k),
// cnt[24 + ...] (i, j, l), cnt[32 + ...] (i, k, l), cnt[40 + ...] (j, k, l).
__device__ __forceinline__ void quad_counts(const uint32_t *planes, int64_t Mp, int w0, int w1,
                                            int step, int i, int j, int k, int l,
                                            uint32_t cnt[48]) {
#pragma unroll
  for (int x = 0; x < 48; ++x) cnt[x] = 0u;
  const uint2 *pv = reinterpret_cast<const uint2 *>(planes);
  for (int w = w0; w < w1; w += step) {
    const uint2 *row = pv + (int64_t)w * Mp;
    const uint2 xi = row[i], xj = row[j], xk = row[k], xl = row[l];
    const uint32_t X[4][2] = {{xi.x, xi.y}, {xj.x, xj.y}, {xk.x, xk.y}, {xl.x, xl.y}};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const uint32_t ij = X[0][a] & X[1][b];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const uint32_t ijk = ij & X[2][c];
          cnt[16 + 4 * a + 2 * b + c] += __builtin_popcount(ijk);
#pragma unroll
          for (int d = 0; d < 2; ++d)
            cnt[8 * a + 4 * b + 2 * c + d] += __builtin_popcount(ijk & X[3][d]);
        }
#pragma unroll
        for (int d = 0; d < 2; ++d) cnt[24 + 4 * a + 2 * b + d] += __builtin_popcount(ij & X[3][d]);
      }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const uint32_t kl = X[2][c] & X[3][d];
#pragma unroll
        for (int a = 0; a < 2; ++a) cnt[32 + 4 * a + 2 * c + d] += __builtin_popcount(X[0][a] & kl);
#pragma unroll
        for (int b = 0; b < 2; ++b) cnt[40 + 4 * b + 2 * c + d] += __builtin_popcount(X[1][b] & kl);
      }
  }
}

// Only the 16 quad corner cells of quad_counts (cnt[0..15]).
__device__ __forceinline__ void quad_corner_counts(const uint32_t *planes, int64_t Mp, int w0, int w1,
                                                   int i, int j, int k, int l, uint32_t cnt[16]) {
#pragma unroll
  for (int x = 0; x < 16; ++x) cnt[x] = 0u;
  const uint2 *pv = reinterpret_cast<const uint2 *>(planes);
  for (int w = w0; w < w1; ++w) {
    const uint2 *row = pv + (int64_t)w * Mp;
    const uint2 xi = row[i], xj = row[j], xk = row[k], xl = row[l];
    const uint32_t X[4][2] = {{xi.x, xi.y}, {xj.x, xj.y}, {xk.x, xk.y}, {xl.x, xl.y}};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const uint32_t ij = X[0][a] & X[1][b];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const uint32_t ijk = ij & X[2][c];
#pragma unroll
          for (int d = 0; d < 2; ++d)
            cnt[8 * a + 4 * b + 2 * c + d] += __builtin_popcount(ijk & X[3][d]);
        }
      }
  }
}

// The 81 cells t[27 a + 9 b + 3 c + d] (a, b, c, d in {0, 1, 2}) of one class
// of the quad (i, j, k, l) from its counts (quad_counts) and the class's
// pairwise tables pairs[x][y] (int4 (n00, n01, n10, n11), per-SNP counts on
// the diagonal) and size.  Each sub-triplet's 27 cells come from its corners
// (complete_table); then the rows with a 2 at SNP i, j, k, l in turn: a count
// with a 2 at one SNP is the sub-triplet table without that SNP minus the
// rows with 0 and 1 there (every sample of the class is in one row).
// SH scales every count by 2^SH (SH = 2: cells as byte offsets into an FP32
// table); cnt and Nc must come scaled alike, the pairwise tables are scaled here.
// ml_in: the per-SNP counts of SNP l already scaled (NULL: read from the
// pairwise table's diagonal).
template <int SH = 0>
__device__ __forceinline__ void quad_cells(const uint32_t cnt[48], const int32_t *pairs, int64_t Mp,
                                           int i, int j, int k, int l, int Nc, int t[81],
                                           const int *ml_in = nullptr) {
  const int4 *pr = reinterpret_cast<const int4 *>(pairs);
  auto pair = [&](int x, int y, int v[4]) {
    const int4 p = pr[(int64_t)x * Mp + y];
    v[0] = p.x << SH; v[1] = p.y << SH; v[2] = p.z << SH; v[3] = p.w << SH;
  };
  auto marg = [&](int x, int v[2]) {
    const int4 p = pr[(int64_t)x * Mp + x];
    v[0] = p.x << SH; v[1] = p.w << SH;
  };
  int pij[4], pik[4], pil[4], pjk[4], pjl[4], pkl[4], mi[2], mj[2], mk[2], ml[2];
  pair(i, j, pij); pair(i, k, pik); pair(i, l, pil);
  pair(j, k, pjk); pair(j, l, pjl); pair(k, l, pkl);
  marg(i, mi); marg(j, mj); marg(k, mk);
  if (ml_in) {
    ml[0] = ml_in[0];
    ml[1] = ml_in[1];
  } else {
    marg(l, ml);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int d = 0; d < 2; ++d) t[27 * a + 9 * b + 3 * c + d] = (int)cnt[8 * a + 4 * b + 2 * c + d];
  int T[27];
  // a = 2 (b, c, d in {0, 1}) from the (j, k, l) table
  complete_table(cnt + 40, pjk, pjl, pkl, mj, mk, ml, Nc, T);
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int d = 0; d < 2; ++d)
        t[54 + 9 * b + 3 * c + d] = T[9 * b + 3 * c + d] - t[9 * b + 3 * c + d] - t[27 + 9 * b + 3 * c + d];
  // b = 2 (c, d in {0, 1}) from the (i, k, l) table
  complete_table(cnt + 32, pik, pil, pkl, mi, mk, ml, Nc, T);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int d = 0; d < 2; ++d)
        t[27 * a + 18 + 3 * c + d] = T[9 * a + 3 * c + d] - t[27 * a + 3 * c + d] - t[27 * a + 9 + 3 * c + d];
  // c = 2 (d in {0, 1}) from the (i, j, l) table
  complete_table(cnt + 24, pij, pil, pjl, mi, mj, ml, Nc, T);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int d = 0; d < 2; ++d)
        t[27 * a + 9 * b + 6 + d] = T[9 * a + 3 * b + d] - t[27 * a + 9 * b + d] - t[27 * a + 9 * b + 3 + d];
  // d = 2 from the (i, j, k) table
  complete_table(cnt + 16, pij, pik, pjk, mi, mj, mk, Nc, T);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        t[27 * a + 9 * b + 3 * c + 2] = T[9 * a + 3 * b + c] - t[27 * a + 9 * b + 3 * c] - t[27 * a + 9 * b + 3 * c + 1];
}

// Lexicographic rank of the quad (i, j, k, l), i < j < k < l < M.
__host__ __device__ __forceinline__ int64_t c4(int64_t x) {
  return x < 4 ? 0 : x * (x - 1) / 2 * (x - 2) / 3 * (x - 3) / 4;
}
__host__ __device__ __forceinline__ int64_t quad_rank(int64_t M, int64_t i, int64_t j, int64_t k,
                                                      int64_t l) {
  return c4(M) - c4(M - i) + c3(M - 1 - i) - c3(M - j) + c2(M - 1 - j) - c2(M - k) + (l - k - 1);
}

// Triplet (i, j, k) of lexicographic rank `rank` among the triplets of M SNPs.
__device__ __forceinline__ void decode_rank(int64_t M, int64_t rank, int &i, int &j, int &k) {
  const int64_t C = c3(M);
  int lo = 0, hi = (int)M - 3;  // last i with first rank <= rank
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (C - c3(M - mid) <= rank) lo = mid; else hi = mid - 1;
  }
  i = lo;
  const int64_t r1 = rank - (C - c3(M - i));
  // within i: pivots j > i, each with M - 1 - j values of k
  int jl = i + 1, jh = (int)M - 2;
  while (jl < jh) {
    const int mid = (jl + jh + 1) >> 1;
    if (c2(M - 1 - i) - c2(M - mid) <= r1) jl = mid; else jh = mid - 1;
  }
  j = jl;
  k = (int)(rank - lex_base(M, i, j));
}

// Quad (i, j, k, l) of lexicographic rank `rank` among the quads of M SNPs.
__device__ __forceinline__ void decode_quad_rank(int64_t M, int64_t rank, int &i, int &j, int &k,
                                                 int &l) {
  const int64_t C = c4(M);
  int lo = 0, hi = (int)M - 4;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (C - c4(M - mid) <= rank) lo = mid; else hi = mid - 1;
  }
  i = lo;
  const int64_t r1 = rank - (C - c4(M - i));
  lo = i + 1;
  hi = (int)M - 3;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (c3(M - 1 - i) - c3(M - mid) <= r1) lo = mid; else hi = mid - 1;
  }
  j = lo;
  const int64_t r2 = r1 - (c3(M - 1 - i) - c3(M - j));
  lo = j + 1;
  hi = (int)M - 2;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (c2(M - 1 - j) - c2(M - mid) <= r2) lo = mid; else hi = mid - 1;
  }
  k = lo;
  l = (int)(r2 - (c2(M - 1 - j) - c2(M - k))) + k + 1;
}

// Log-factorial table entry at byte offset b (b = 4 n for L[n]).
__device__ __forceinline__ float lf_at(const float *L, int b) {
  return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(L) + b);
}
// The same for a table at LDS address 0 (the start of the dynamic LDS block
// of a kernel that declares no static LDS): the byte offset is the address,
// so a lookup is a single ds_read.
__device__ __forceinline__ float lf_at_lds0(int b) {
  return *(const __attribute__((address_space(3))) float *)(uintptr_t)(uint32_t)b;
}

// The FP32 log-factorial table sits in LDS when it fits in this many bytes
// (two workgroups per CU); larger tables are read from global memory.
constexpr int64_t kLdsTableBytes = 80 * 1024;
inline bool lf_in_lds(int32_t lf_len) { return (int64_t)lf_len * 4 <= kLdsTableBytes; }

// ---- host-side launchers (defined in the .hip files) ----
hipError_t launch_encode(const uint8_t *geno, int64_t ld, const int32_t *sample_list,
                         int32_t M, int32_t Mp, int32_t W0, int32_t W1, uint32_t *planes,
                         int32_t *status, hipStream_t s);
hipError_t launch_encode_bytes(const uint8_t *geno, int64_t ld, int32_t M, int32_t N, int32_t Mp,
                               int32_t S, uint8_t *bytes, hipStream_t s);
hipError_t launch_encode_nibbles(const uint8_t *geno, int64_t ld, int32_t M, int32_t N, int32_t Mp,
                                 int32_t S, uint8_t *nib, hipStream_t s);
hipError_t launch_encode_values(const uint8_t *geno, int64_t ld, const int32_t *list, int32_t off0,
                                int32_t len0, int32_t off1, int32_t len1, int32_t classes,
                                int32_t M, int32_t Mp, int32_t S, uint8_t *bytes, uint8_t *nib,
                                hipStream_t s);
hipError_t launch_pairs(const uint32_t *planes, int32_t Mp, int32_t M, int32_t W0, int32_t W1,
                        int32_t n_classes, const uint32_t *mask, int32_t *pairs, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_tile_prefix(Job *jobs_dev, int32_t n_jobs, hipStream_t s);
int64_t host_tiles(int64_t M, int P);
hipError_t launch_write_jobs(const Job *jobs_host, int32_t n, Job *dst_dev, hipStream_t s);
hipError_t launch_count_valu(const Job *jobs_dev, int32_t n_jobs, int64_t total_tiles,
                             unsigned long long *queue, const float *lf32, int32_t lf_len,
                             int32_t P_lo, int32_t P_hi, bool counts, hipStream_t s);
// sampled: at least one job has SelJob::sample set.
hipError_t launch_select(SelJob *sel_dev, int32_t n_jobs, int64_t max_T, int64_t max_cap,
                         int32_t max_k, bool sampled, hipStream_t s);
hipError_t launch_write_seljobs(const SelJob *h, int32_t n, SelJob *dst_dev, hipStream_t s);
// The k-th smallest key of each job's plane only (st->kth, done = 1; jobs
// with fewer than k keys in their key range end with done = 0).
hipError_t launch_select_kth(SelJob *sel_dev, int32_t n_jobs, int64_t max_T, hipStream_t s);
// After a sample pass: main job x's compacted list bound = the sample's k-th
// score + 2 e(N) (rounded up; +inf if the sample had no k-th score), empty list.
hipError_t launch_sample_bound(SelJob *main_dev, const SelJob *sample_dev, int32_t n_jobs,
                               hipStream_t s);
hipError_t launch_init_select(SelJob *sel_dev, int32_t n_jobs, hipStream_t s);
hipError_t launch_score_triplets(const epi3_dataset &d, const uint32_t *ijk, int64_t n,
                                 uint32_t *counts, float *k2f, double *k2, hipStream_t s);

hipError_t launch_perm_prefix(PermJob *pj_dev, hipStream_t s);
hipError_t launch_mask_bytes(const uint32_t *const *masks_dev, int32_t Q, int32_t Qp, int32_t N,
                             int32_t S, uint8_t *ph, int32_t *n1, bool fp4, hipStream_t s);
hipError_t launch_case_pairs(const uint32_t *planes, int32_t Mp, int32_t W,
                             const uint32_t *const *masks_dev, int32_t Q, int32_t Qp, int32_t *out,
                             hipStream_t s);
// Pair scan: FP32 K2 of every pair of a SPLIT data set from its pairwise
// tables, by lexicographic pair rank; key range into keyrange[0..1].
hipError_t launch_pair_scores(const epi3_dataset &d, float *score, uint32_t *keyrange, hipStream_t s);
// Quad scan: FP32 K2 of every quad of a SPLIT data set, by lexicographic quad
// rank; key range into keyrange[0..1].  t3: device buffer of
// quad_triplet_table_bytes for the triplet corner table (classes of at most
// 65535 samples), or NULL to count the sub-triplet corners per quad.
inline int64_t quad_triplet_table_bytes(int64_t M) { return 2 * 16 * (M < 3 ? 0 : M * (M - 1) / 2 * (M - 2) / 3); }
// Corner cells of every triplet per class into t3 (quad_triplet_table_bytes).
hipError_t launch_triplet_corners(const epi3_dataset &d, void *t3, hipStream_t s);
// Quad scan with the counts on the matrix cores (FP4 value planes, classes of
// at most 65535 samples): tiles of 4 i x 1 j x 16 k x 32 l, counted and
// scored pass by pass through a scratch buffer of pass_tiles tiles.
constexpr int64_t kQuadTileScratch = 128 * 1024;  // bytes per tile, both classes
int64_t host_quad_tiles(int32_t M);
hipError_t launch_quad_prefix(int32_t M, int64_t *jprefix, hipStream_t s);
// counts tiles [tile_begin, tile_begin + n_tiles) into scratch slots from 0
hipError_t launch_count_mfma_quad(const epi3_dataset &d, const int64_t *jprefix,
                                  unsigned long long *queue, int64_t tile_begin, int64_t n_tiles,
                                  void *scratch, hipStream_t s);
// completes and scores the quads of those tiles (t3: launch_triplet_corners)
hipError_t launch_finish_quad(const epi3_dataset &d, const void *scratch, const int64_t *jprefix,
                              const void *t3, int64_t tile_begin, int64_t n_tiles, float *score,
                              uint32_t *keyrange, hipStream_t s);
hipError_t launch_quad_scores(const epi3_dataset &d, void *t3, float *score, uint32_t *keyrange,
                              hipStream_t s);
int64_t host_perm_tiles(int64_t M);
// Count / finish the tiles tile_begin + n * stride, n in [0, n_tiles); their
// corner cells go to scratch slot n.
hipError_t launch_count_mfma_perm(const PermJob *pj_dev, int64_t tile_begin, int64_t n_tiles,
                                  int64_t stride, unsigned long long *queue, bool fp4,
                                  hipStream_t s);
hipError_t launch_finish_perm(const PermJob *pj_dev, int64_t tile_begin, int64_t n_tiles,
                              int64_t stride, SelState *st, const float *lf32, int32_t lf_len,
                              const PermOut &out, hipStream_t s);
// Count and score in one kernel (FP4 operands, sample or bounded output, the
// log-factorial table of lf_len entries in LDS: perm_fused_ok); no scratch.
bool perm_fused_ok(int32_t lf_len);
hipError_t launch_count_score_perm(const PermJob *pj_dev, int64_t tile_begin, int64_t n_tiles,
                                   int64_t stride, unsigned long long *queue, SelState *st,
                                   const float *lf32, int32_t lf_len, const PermOut &out,
                                   hipStream_t s);
// Triplets (i < j < k < M) in the phenotype-batch tiles 0, stride, 2 stride, ...
int64_t host_perm_sample_valid(int64_t M, int64_t stride);
constexpr int64_t kPermTileScratch = 64 * 64 * 16 + 64 * 16;  // bytes per tile (corners + totals)
hipError_t launch_write_permjob(const PermJob &h, PermJob *dst_dev, hipStream_t s);
hipError_t launch_write_ptrs(const uint32_t *const *h, int32_t n, const uint32_t **dst_dev,
                             hipStream_t s);

int64_t host_plain_tiles(int64_t M, int JB);
constexpr int kPlainI = 16;  // pivots i per plain matrix-core tile (x JB j x 256 / JB k)
constexpr int64_t kPlainTileScratch = 2ll * kPlainI * 256 * 16;  // bytes per tile, both classes
hipError_t launch_write_plainjob(const PlainJob &h, PlainJob *dst_dev, hipStream_t s);
hipError_t launch_plain_prefix(PlainJob *pj_dev, hipStream_t s);
// Plain matrix-core count / finish of the global tiles tile_begin + q stride,
// q < n_tiles, of n_jobs data sets (same JB and operand type): job x owns
// global tiles job_begin[x] .. job_begin[x + 1] (device int64 [n_jobs + 1]);
// slot q's corner cells sit in scratch slot q of `corners`.
hipError_t launch_count_mfma_plain(const PlainJob *jobs, const int64_t *job_begin, int32_t n_jobs,
                                   int JB, bool fp4, uint4 *corners, int64_t tile_begin,
                                   int64_t n_tiles, int64_t stride, unsigned long long *queue,
                                   hipStream_t s);
hipError_t launch_finish_plain(const PlainJob *jobs, const int64_t *job_begin, int32_t n_jobs,
                               int JB, const uint4 *corners, int64_t tile_begin, int64_t n_tiles,
                               const float *lf32, int32_t lf_len, bool counts, const PlainOut &out,
                               hipStream_t s);
// Triplets (i < j < k < M) in the plain tiles 0, stride, 2 stride, ... of a
// data set of M SNPs (tile JB); the number of such tiles in *n_sample.
int64_t host_plain_sample_valid(int64_t M, int JB, int64_t stride, int64_t *n_sample);
hipError_t launch_write_i64(const int64_t *h, int32_t n, int64_t *dst_dev, hipStream_t s);

int tile_P_default(int32_t M, int32_t N);

// Device address of the current device's copy of the static scan workspace
// (looked up once per device; out may be NULL to only set it up).
int static_scratch_ptr(void **out);

}  // namespace epi3
