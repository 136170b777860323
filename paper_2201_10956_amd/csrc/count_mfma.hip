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
// FP4 (E2M1) operands run the same products on the scaled f8f6f4 matrix
// instructions.  Batches selected by bound count and score in one kernel
// (count_score_perm_kernel): each wave scores its tile's tables from its
// accumulators; otherwise the corner cells go through a scratch buffer to
// finish_perm_kernel.
//
// Fragment layout of v_mfma_i32_32x32x32_i8 (gfx950, checked on hardware):
// lane l supplies A row l % 32 and B column l % 32 with 16 consecutive K
// values starting at 16 (l / 32); the result of row r, column c is in lane
// c + 32 ((r / 4) % 2), register 4 (r / 8) + r % 4.
#include <algorithm>

#include "epi3_internal.h"

namespace epi3 {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kPermKB = 16;  // k values per wave tile (4 row tiles x 4 triplets)
constexpr int kPermT = 4;    // row tiles per wave tile (one per lane of a quad)

// k-blocks are aligned to multiples of kPermKB for every pivot, so tiles of
// different j share (i-block, k-block) pairs; block kb of pivot j is global
// block perm_kb_lo(j) + kb and may start at or below j (those k are dropped).
__host__ __device__ __forceinline__ int perm_kb_lo(int64_t j) { return (int)((j + 1) / kPermKB); }
__host__ __device__ __forceinline__ int perm_nkb(int64_t M, int64_t j) {
  return (int)((M - 1) / kPermKB) - perm_kb_lo(j) + 1;
}
// i-block and k-block of tile rr of pivot j: bands of 8 i-blocks, k-block
// major within a band, so the tiles one XCD works on at a time share the
// operand rows of 8 i-blocks and of a few k-blocks (and their case pair rows).
__host__ __device__ __forceinline__ void perm_tile_ib_kb(int rr, int j, int nkb, int &ib, int &kb) {
  const int nib = (j + 3) / 4;
  const int band = rr / (8 * nkb);
  const int rest = nib - 8 * band;
  const int bcnt = rest < 8 ? rest : 8;
  const int pos = rr - band * 8 * nkb;
  kb = pos / bcnt;
  ib = 8 * band + (pos - kb * bcnt);
}
__host__ __device__ __forceinline__ int64_t perm_tiles_of_j(int64_t M, int64_t j) {
  if (j < 1 || j > M - 2) return 0;
  return ((j + 3) / 4) * perm_nkb(M, j);
}

__device__ __forceinline__ int64_t rfl64p(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// acc + popcount(x) as one v_bcnt_u32_b32 (the compiler would otherwise
// reassociate chains of counts into v_bcnt(x, 0) plus v_add3).
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
  return r;
}

// acc + popcounts of the four words of x.
__device__ __forceinline__ uint32_t popc4_acc(v4i x, uint32_t acc) {
  acc = bcnt_acc((uint32_t)x.x, acc);
  acc = bcnt_acc((uint32_t)x.y, acc);
  acc = bcnt_acc((uint32_t)x.z, acc);
  return bcnt_acc((uint32_t)x.w, acc);
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
// With FP4, the row holds E2M1 nibbles (1.0 = 0x2, two samples per byte, low
// nibble first) and is S / 2 bytes long.
__global__ void __launch_bounds__(256) mask_bytes_kernel(const uint32_t *const *masks, int32_t Q,
                                                         int32_t N, int32_t S, uint8_t *ph,
                                                         int32_t *n1, int fp4) {
  const int q = blockIdx.x;
  __shared__ int red[256];
  int cnt = 0;
  const int per = fp4 ? 8 : 4;           // samples per dword
  const int rowb = fp4 ? S / 2 : S;      // bytes per row
  uint32_t *row = reinterpret_cast<uint32_t *>(ph + (int64_t)q * rowb);
  for (int d = threadIdx.x; d < rowb / 4; d += blockDim.x) {
    uint32_t v = 0;
    if (q < Q) {
      for (int b = 0; b < per; ++b) {
        const int s = per * d + b;
        if (s < N) {
          const uint32_t bit = (masks[q][s >> 5] >> (s & 31)) & 1u;
          v |= fp4 ? (bit << (4 * b + 1)) : (bit << (8 * b));
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

// Case pairs of every phenotype: out[x][y][q] = (n(0,0) | n(0,1) << 16, n(1,0) | n(1,1) << 16)
// over the samples whose bit is set in mask q, for y >= x (every reader looks
// up pairs in increasing SNP order, and the diagonal for the per-SNP counts;
// waves whose 64 y all lie below x write nothing).  One wave per (x, 64 y);
// the block's z index selects a group of 16 phenotypes.
__global__ void __launch_bounds__(256) case_pairs_kernel(const uint32_t *__restrict__ planes,
                                                         int32_t Mp, int32_t W,
                                                         const uint32_t *const *masks, int32_t Q,
                                                         int32_t Qp, int32_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int x = __builtin_amdgcn_readfirstlane(blockIdx.y * 4 + (threadIdx.x >> 6));
  const int y = blockIdx.x * 64 + lane;
  const int q0 = blockIdx.z * 16;
  if (x >= Mp || (int)blockIdx.x * 64 + 63 < x) return;
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
  // two 16-bit counts per word (counts stay below 2^16: the matrix-core paths
  // take at most 65535 samples per class)
  uint2 *o = reinterpret_cast<uint2 *>(out) + ((int64_t)x * Mp + y) * Qp;
#pragma unroll
  for (int t = 0; t < 16; ++t)
    if (q0 + t < Qp)
      o[q0 + t] = make_uint2(acc[t][0] | (acc[t][1] << 16), acc[t][2] | (acc[t][3] << 16));
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


template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

// Bytes of an FP32 log-factorial table of lf_len entries in LDS (16-byte multiple).
__host__ __device__ __forceinline__ int finish_perm_table_bytes(int lf_len) {
  return (lf_len * 4 + 15) / 16 * 16;
}
// LDS of the count-and-score kernel: the table, then staging, tile slot,
// totals exchange, the tile's all-sample cells and the key ranges.
__host__ __device__ __forceinline__ int perm_score_lds_bytes(int lf_len) {
  return finish_perm_table_bytes(lf_len) + 2 * kStageBytes + 2 * 8 + 2 * 64 * 4 * 4 + 4 * kPermKB * 16 +
         64 * 2 * 4;
}

// Workgroup tile: pivot j, four pivots i = 4 ib + wave (one per wave), 16
// consecutive k > j, 64 phenotypes.  Phenotype bytes, the k planes and the
// pair words are staged per chunk of kKC samples in double-buffered LDS; each
// wave then runs 8 MFMAs per 32 samples (4 row tiles of 4 triplets x 8
// corner cells, 2 column tiles of 32 phenotypes).
// FP4: operands are E2M1 nibbles (each staged byte holds two samples, so a
// 32-byte step covers 64 samples) on v_mfma_scale_f32_32x32x64_f8f6f4 with
// unit scales; accumulation in FP32 is exact for counts below 2^24.  The
// all-sample corner counts (the phenotype-independent column) come from one
// 16 x 16 x 128 product per wave and chunk over the staged pair and k rows;
// int8 operands count them by popcounts of the A rows.
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

typedef float v4f __attribute__((ext_vector_type(4)));
// 16 x 16 x 128 FP4 product with unit scales (all-sample corner counts)
__device__ __forceinline__ v4f tot_mma(v4i a, v4i b, v4f c) {
  const v8i a8 = {a.x, a.y, a.z, a.w, 0, 0, 0, 0};
  const v8i b8 = {b.x, b.y, b.z, b.w, 0, 0, 0, 0};
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, b8, c, 4, 4, 0, 127, 0, 127);
}

template <bool FP4>
struct PermAcc {
  typedef v16i type;
  static __device__ __forceinline__ type mma(v4i a, v4i b, type c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ uint32_t get(const type &c, int v) { return (uint32_t)c[v]; }
};
template <>
struct PermAcc<true> {
  typedef v16f type;
  static __device__ __forceinline__ type mma(v4i a, v4i b, type c) {
    const v8i a8 = {a.x, a.y, a.z, a.w, 0, 0, 0, 0};
    const v8i b8 = {b.x, b.y, b.z, b.w, 0, 0, 0, 0};
    // cbsz = blgp = 4: both operands FP4 (E2M1); scale exponents 127 = 2^0
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, c, 4, 4, 0, 127, 0, 127);
  }
  static __device__ __forceinline__ uint32_t get(const type &c, int v) { return (uint32_t)c[v]; }
};

// x from quad lane TT in every lane of each quad (DPP quad_perm broadcast;
// the compiler folds it into the AND that consumes it).
template <int TT>
__device__ __forceinline__ v4i quad_bcast(v4i x) {
  constexpr int sel = TT * 0x55;
  v4i y;
  y.x = __builtin_amdgcn_update_dpp(0, x.x, sel, 0xf, 0xf, true);
  y.y = __builtin_amdgcn_update_dpp(0, x.y, sel, 0xf, 0xf, true);
  y.z = __builtin_amdgcn_update_dpp(0, x.z, sel, 0xf, 0xf, true);
  y.w = __builtin_amdgcn_update_dpp(0, x.w, sel, 0xf, 0xf, true);
  return y;
}

// Completes and scores, in the count kernel, the 16 x 64 (triplet,
// phenotype) case tables of one wave's pivot i of a tile (k = k0 .. k0 + 15,
// lane = phenotype), as finish_perm_kernel does from the corner scratch: the
// same cells, the same FP32 row order, the same outputs.  The accumulators
// hold, in lane (q, h), the case cells with genotype h at SNP k of phenotype
// q mod 32 + 32 qb; one lane-half swap per register pair (qb = 0, 1) leaves
// lane q with both genotypes of phenotype q.  Lanes 0..15 complete the
// all-sample tables (cells from the tile's totals in LDS) and write, per k,
// the 27 cells x 4 and their L[cell + 1] to the wave's part of the idle
// staging buffer (`row`, 224 bytes per k), which every lane then reads as
// broadcasts.  The log-factorial table sits at LDS address 0.
template <int FUSE>
__device__ __forceinline__ void fused_score(const PermJob &pj, v16f (&acc)[kPermT][2],
                                            const uint4 *tot16, uint32_t *rows,
                                            SelState *__restrict__ st, const PermOut &out, int i,
                                            int j, int k0, int64_t slot, int wave, int lane,
                                            uint32_t &kmin, uint32_t &kmax) {
  // the pivot is uniform over the wave: scalar row addresses below
  i = __builtin_amdgcn_readfirstlane(i);
  wave = __builtin_amdgcn_readfirstlane(wave);
  const int M = pj.M, Mp = pj.Mp, Q = pj.Q, Qp = pj.Qp;
  const int kk_lo = j + 1 - k0 > 0 ? j + 1 - k0 : 0;
  const int kk_hi = M - k0 < kPermKB ? M - k0 : kPermKB;
  // case cells of phenotype q = lane: genotype 0 of SNP k in the low half,
  // genotype 1 in the high half of each register, (a, b) = v % 4
  uint32_t cc[kPermT][16];
#pragma unroll
  for (int tt = 0; tt < kPermT; ++tt)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const auto sw = __builtin_amdgcn_permlane32_swap((uint32_t)acc[tt][0][v],
                                                       (uint32_t)acc[tt][1][v], false, false);
      cc[tt][v] = sw[0] | (sw[1] << 16);
    }
  // all-sample tables, lane kk = triplet (i, j, k0 + kk)
  if (lane >= kk_lo && lane < kk_hi) {
    const int4 *tp = reinterpret_cast<const int4 *>(pj.tot_pairs);
    const int k = k0 + lane;
    const uint4 tq = tot16[lane];
    const uint32_t tn[8] = {(tq.x & 0xffffu) << 2, (tq.x >> 16) << 2, (tq.y & 0xffffu) << 2,
                            (tq.y >> 16) << 2, (tq.z & 0xffffu) << 2, (tq.z >> 16) << 2,
                            (tq.w & 0xffffu) << 2, (tq.w >> 16) << 2};
    const int4 a = tp[(int64_t)i * Mp + j], b = tp[(int64_t)i * Mp + k], c = tp[(int64_t)j * Mp + k];
    const int4 ii4 = tp[(int64_t)i * Mp + i], jj4 = tp[(int64_t)j * Mp + j], kk4 = tp[(int64_t)k * Mp + k];
    const int tij[4] = {a.x << 2, a.y << 2, a.z << 2, a.w << 2};
    const int tik[4] = {b.x << 2, b.y << 2, b.z << 2, b.w << 2};
    const int tjk[4] = {c.x << 2, c.y << 2, c.z << 2, c.w << 2};
    const int mi[2] = {ii4.x << 2, ii4.w << 2}, mj[2] = {jj4.x << 2, jj4.w << 2};
    const int mk[2] = {kk4.x << 2, kk4.w << 2};
    int t4[27];
    complete_table(tn, tij, tik, tjk, mi, mj, mk, pj.N << 2, t4);
    uint32_t *row = rows + lane * 56;
#pragma unroll
    for (int x = 0; x < 27; ++x) {
      row[x] = (uint32_t)t4[x];
      row[28 + x] = __float_as_uint(lf_at_lds0(t4[x] + 4));
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  typedef unsigned u2e __attribute__((ext_vector_type(2)));
  gptr<u2e> cp = (gptr<u2e>)pj.case_pairs;
  auto cp_row = [&](int x, int y) { return cp + ((int64_t)x * Mp + y) * Qp; };
  auto lo4 = [](unsigned v) { return (int)((v & 0xffffu) << 2); };
  auto hi4 = [](unsigned v) { return (int)((v >> 16) << 2); };
  const int q = lane, qc = q < Q ? q : 0;
  const int n1x4 = pj.n1[qc] << 2;
  const float ubq = FUSE == kPermOutBounded ? st[qc].ub : 0.f;
  const u2e cij = cp_row(i, j)[qc];
  const u2e cii = cp_row(i, i)[qc], cjj = cp_row(j, j)[qc];
  const int aij[4] = {lo4(cij.x), hi4(cij.x), lo4(cij.y), hi4(cij.y)};
  const int mi[2] = {lo4(cii.x), hi4(cii.y)}, mj[2] = {lo4(cjj.x), hi4(cjj.y)};
  const int64_t base = lex_base(M, i, j) + k0;
  // rows k0 .. k0 + 15 lie below the padded stride Mp (k0 + 15 < M + 16):
  // loaded for every k, used for k in (j, M) only; one k ahead, through
  // uniform row pointers advanced by one k per step
  gptr<u2e> pik = cp_row(i, k0), pjk = cp_row(j, k0), pkk = cp_row(k0, k0);
  const int64_t dkk = (int64_t)(Mp + 1) * Qp;
  u2e cik_n = pik[qc], cjk_n = pjk[qc], ckk_n = pkk[qc];
#pragma unroll
  for (int tt = 0; tt < kPermT; ++tt)
#pragma unroll
    for (int t4 = 0; t4 < 4; ++t4) {
      const int kk = 4 * tt + t4;
      const u2e cik = cik_n, cjk = cjk_n, ckk = ckk_n;
      if (kk + 1 < kPermKB) {
        pik += Qp;
        pjk += Qp;
        pkk += dkk;
        cik_n = pik[qc];
        cjk_n = pjk[qc];
        ckk_n = pkk[qc];
      }
      if (kk < kk_lo || kk >= kk_hi) continue;  // wave-uniform
      int c4[27];
      {
        uint32_t cn[8];  // corner index 4 a + 2 b + c, x 4
#pragma unroll
        for (int ab = 0; ab < 4; ++ab) {
          const uint32_t w = cc[tt][4 * t4 + ab];
          cn[2 * ab] = (w << 2) & 0x3fffcu;
          cn[2 * ab + 1] = (w >> 14) & 0x3fffcu;
        }
        const int aik[4] = {lo4(cik.x), hi4(cik.x), lo4(cik.y), hi4(cik.y)};
        const int ajk[4] = {lo4(cjk.x), hi4(cjk.x), lo4(cjk.y), hi4(cjk.y)};
        const int mk[2] = {lo4(ckk.x), hi4(ckk.y)};
        complete_table(cn, aij, aik, ajk, mi, mj, mk, n1x4, c4);
      }
      // cells x 4 in words 0..27, their L[cell + 1] in words 28..55 (same
      // address in all lanes: broadcast reads), four rows at a time
      const uint4 *rk = reinterpret_cast<const uint4 *>(rows + kk * 56);
      float k2 = 0.f;  // rows in order: L[r + 1] - (L[r_0] + L[r_1]), r_1 = cases
#pragma unroll
      for (int x4 = 0; x4 < 7; ++x4) {
        const uint4 tv = rk[x4], lv = rk[7 + x4];
        const uint32_t ta[4] = {tv.x, tv.y, tv.z, tv.w}, la[4] = {lv.x, lv.y, lv.z, lv.w};
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const int x = 4 * x4 + y;
          if (x < 27) {
            const int r0 = (int)ta[y] - c4[x];
            k2 += __uint_as_float(la[y]) - (lf_at_lds0(r0) + lf_at_lds0(c4[x]));
          }
        }
      }
      const uint32_t key = f2key(k2);
      kmin = key < kmin ? key : kmin;
      kmax = key > kmax ? key : kmax;
      if (FUSE == kPermOutSample && q < Q)
        out.sample[(int64_t)q * out.sample_T + (out.sample_base + slot) * 64 + wave * kPermKB + kk] = k2;
      if (FUSE == kPermOutBounded && q < Q && k2 <= ubq) {
        const unsigned long long pos = atomicAdd(&st[q].cn, 1ull);
        if ((int64_t)pos < out.ccap) {
          out.ckey[(int64_t)q * out.ccap + pos] = key;
          out.crank[(int64_t)q * out.ccap + pos] = base + kk;
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // one k at a time: short live ranges
    }
}

// FUSE = kPermOutSample / kPermOutBounded (FP4 only): each wave completes
// and scores its own pivot's 16 x 64 (triplet, phenotype) tables right after
// the tile's counts, from the accumulators (as the finish kernel does from
// the corner scratch), with the log-factorial table at LDS address 0;
// nothing goes to the scratch.  FUSE = 0: corner cells out, finish_perm_kernel
// after.  The kernels below give the LDS arrays.
template <bool FP4, int FUSE>
__device__ __forceinline__ void count_perm_body(
    const PermJob *__restrict__ pjp, int64_t tile_begin, int64_t n_tiles, int64_t stride,
    unsigned long long *__restrict__ queue, SelState *__restrict__ st,
    const float *__restrict__ lf32, int lf_len, const PermOut &out, unsigned char *stage,
    int64_t *sTile, float (*sTot)[64][4], uint4 (*sT16)[kPermKB], uint32_t (*sRange)[2],
    float *sLf) {
  static_assert(FUSE == 0 || FP4, "fused scoring takes FP4 accumulators");
  typedef PermAcc<FP4> Acc;
  const PermJob pj = *pjp;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  if constexpr (FUSE != 0) {
    for (int x = tid; x < lf_len; x += 256) sLf[x] = lf32[x];
    if (tid < 64) {
      sRange[tid][0] = 0xffffffffu;
      sRange[tid][1] = 0u;
    }
  }
  uint32_t kmin = 0xffffffffu, kmax = 0u;  // FUSE: this lane's phenotype's key range
  const int r = lane & 31, g = lane >> 5;
  // A row r of a row tile = (triplet ta = r / 8, corner c = (r / 4) % 2,
  // a = (r / 2) % 2, b = r % 2): the four lanes of a quad share (ta, c) and
  // differ in (a, b), so each lane loads the k row of a different row tile
  // and the quad broadcasts it by DPP (one LDS read for the four row tiles)
  const int ta = r >> 3, rc = (r >> 2) & 1, ra = (r >> 1) & 1, rb = r & 1;
  const int M = pj.M, S = pj.S;
  gptr<uint8_t> gb = (gptr<uint8_t>)pj.bytes;
  gptr<uint8_t> gph = (gptr<uint8_t>)pj.ph;
  cptr<int64_t> pre = as_const(pj.jprefix);
  const int nch = S / kKC;  // bytes per row: a multiple of 128
  int j = -1;
  int64_t jlo = 0, jhi = 0;

  // Tile slots: the pass is cut into 8 contiguous parts, one per XCD
  // (workgroups go to the XCDs round robin, so workgroup b runs on XCD
  // b mod 8), each with its own counter in queue[0..7]; a workgroup takes the
  // next slot of its XCD's part, and once that part is done those of the
  // other parts in turn.  Consecutive slots share operand rows, which then
  // stay in one XCD's L2.  Every workgroup ends after at most 8 empty draws.
  int xq = 0;
  const int xcd = blockIdx.x & 7;
  for (;;) {
    __syncthreads();  // previous tile's readers of sTile / stage are done
    if (tid == 0) {
      int64_t sl = -1;
      while (xq < 8) {
        const int y = (xcd + xq) & 7;
        const int64_t lo = n_tiles * y / 8, hi = n_tiles * (y + 1) / 8;
        const int64_t c = (int64_t)atomicAdd(queue + y, 1ull);
        if (lo + c < hi) { sl = lo + c; break; }
        ++xq;
      }
      sTile[0] = sl < 0 ? n_tiles : sl;
    }
    __syncthreads();
    const int64_t slot = rfl64p(sTile[0]);  // scratch slot of this launch
    // FUSE: a wave that counts issues ahead of the other workgroup's waves
    // that score (their vector instructions and the matrix products share
    // the SIMD's issue), so the matrix cores stay fed while one scores
    if constexpr (FUSE != 0) __builtin_amdgcn_s_setprio(1);
    if (slot >= n_tiles) break;
    const int64_t t = tile_begin + slot * stride;
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
    const int nkb = perm_nkb(M, j);
    const int rr = (int)(t - jlo);
    int ib, kb;
    perm_tile_ib_kb(rr, j, nkb, ib, kb);
    const int i = 4 * ib + wave;  // may be >= j (then the wave's results are dropped)
    const int kbase = (perm_kb_lo(j) + kb) * kPermKB;  // k <= j or k >= M: dropped later

    // ---- staging plan: this thread's 16-byte pieces of one LDS buffer ----
    // rows [0, 64): phenotype q; [64, 96): (k, c) = k planes; [96, 112): pair rows.
    // Each chunk is loaded into registers one chunk ahead.  Pieces
    // c16 = tid + 256 u cover the phenotype and k rows (row < 96); threads
    // tid < 16 kPc cover the 16 pair rows, which keep both source words and
    // are ANDed only when stored, so no load is waited for before the current
    // chunk's matrix products are issued.
    constexpr int kPc = kKC / 16;                // pieces per row
    constexpr int kMainU = 96 * kPc / 256;       // main pieces per thread
    constexpr int kPairPieces = kRowsP * kPc;    // pair pieces (<= 256)
    static_assert(kRowsPH + kRowsXK == 96 && (96 * kPc) % 256 == 0 && kPairPieces <= 256,
                  "staging plan");
    // 32-bit byte offsets of this thread's pieces for chunk 0 (the value
    // planes and phenotype rows are far below 4 GB): scalar base + one VGPR
    uint32_t off[kMainU], offa = 0, offb = 0;
#pragma unroll
    for (int u = 0; u < kMainU; ++u) {
      const int c16 = tid + 256 * u;
      const int row = c16 / kPc, col = (c16 % kPc) * 16;
      if (row < kRowsPH) {
        off[u] = (uint32_t)(row * S + col);
      } else {
        const int x = row - kRowsPH;
        off[u] = (uint32_t)((((int64_t)(kbase + (x >> 1)) * 2 + (x & 1)) * S) + col);
      }
    }
    if (tid < kPairPieces) {
      const int x = tid / kPc, col = (tid % kPc) * 16;  // pair row x: wave x >> 2, (a, b) = x & 3
      const int ii = 4 * ib + (x >> 2);
      offa = (uint32_t)(((int64_t)ii * 2 + ((x >> 1) & 1)) * S + col);
      offb = (uint32_t)(((int64_t)j * 2 + (x & 1)) * S + col);
    }
    v4i pf[kMainU], pa, pb;
    auto fetch = [&](int ch) {
      const uint32_t c0 = (uint32_t)ch * kKC;
#pragma unroll
      for (int u = 0; u < kMainU; ++u) {
        const int row = (tid + 256 * u) / kPc;
        if (row < kRowsPH)
          pf[u] = *reinterpret_cast<gptr<v4i>>(gph + (off[u] + c0));
        else
          pf[u] = *reinterpret_cast<gptr<v4i>>(gb + (off[u] + c0));
      }
      if (tid < kPairPieces) {
        pa = *reinterpret_cast<gptr<v4i>>(gb + (offa + c0));
        pb = *reinterpret_cast<gptr<v4i>>(gb + (offb + c0));
      }
    };
    auto store = [&](int buf) {
      uint8_t *dst = stage + buf * kStageBytes;
#pragma unroll
      for (int u = 0; u < kMainU; ++u) {
        const int c16 = tid + 256 * u;
        *reinterpret_cast<v4i *>(dst + (c16 / kPc) * kRow + (c16 % kPc) * 16) = pf[u];
      }
      if (tid < kPairPieces)
        *reinterpret_cast<v4i *>(dst + (96 + tid / kPc) * kRow + (tid % kPc) * 16) = pa & pb;
    };

    typename Acc::type acc[kPermT][2];
    uint32_t tot[kPermT];
#pragma unroll
    for (int tt = 0; tt < kPermT; ++tt) {
      tot[tt] = 0u;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[tt][0][v] = acc[tt][1][v] = 0;
    }
    // FP4: the all-sample corner counts of the tile are one 16 x 16 product
    // per k half: rows = the 16 pair rows (4 pivots x (a, b)), columns = 8 k
    // x c, K = 128 samples; wave w takes k half w % 2 and the chunk's sample
    // half w / 2 (one product per chunk)
    v4f tacc = {0.f, 0.f, 0.f, 0.f};
    const int tkh = wave & 1, tsh = wave >> 1;
    const int o_ta = (kRowsPH + kRowsXK + (lane & 15)) * kRow + 64 * tsh + 16 * (lane >> 4);
    const int o_tb = (kRowsPH + 16 * tkh + (lane & 15)) * kRow + 64 * tsh + 16 * (lane >> 4);
    v4i tA, tB;
    fetch(0);
    store(0);
    __syncthreads();
    const int prow = kRowsPH + kRowsXK + wave * 4 + (ra * 2 + rb);
    const int xrow = kRowsPH + (4 * (r & 3) + ta) * 2 + rc;  // k row of row tile r % 4
    // Software pipeline over the steps of a chunk: while the matrix products
    // of step s run, the operands of step s + 1 are read from LDS (two
    // register sets, X and Y, taken in turn), and each row tile's A rows are
    // formed between the products of the previous row tile (int8: four
    // vector instructions between products, with the popcounts, by
    // scheduling-group hints; FP4 schedules better without them).  The next chunk
    // is stored to the other LDS buffer before the last step of a chunk and
    // one barrier follows, so the last step already reads the first operands
    // of the next chunk and the pipeline does not drain between chunks.
    static_assert(kKC / 32 == 4, "four steps per chunk");
    const int o_p = prow * kRow + 16 * g, o_x = xrow * kRow + 16 * g;
    const int o_b0 = r * kRow + 16 * g, o_b1 = (32 + r) * kRow + 16 * g;
#define EPI3_LD(BB, STP, P, X, B0, B1)                                              \
    P = *reinterpret_cast<const v4i *>((BB) + o_p + 32 * (STP));                  \
    X = *reinterpret_cast<const v4i *>((BB) + o_x + 32 * (STP));                  \
    B0 = *reinterpret_cast<const v4i *>((BB) + o_b0 + 32 * (STP));                \
    B1 = *reinterpret_cast<const v4i *>((BB) + o_b1 + 32 * (STP));
#define EPI3_TILE(TT, P, X, B0, B1)                                                 \
    {                                                                             \
      const v4i a_ = (P) & quad_bcast<TT>(X);                                     \
      acc[TT][0] = Acc::mma(a_, B0, acc[TT][0]);                                  \
      acc[TT][1] = Acc::mma(a_, B1, acc[TT][1]);                                  \
      if constexpr (!FP4) tot[TT] = popc4_acc(a_, tot[TT]);                       \
    }
#define EPI3_SCHED                                                                  \
    __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);                            \
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                            \
    __builtin_amdgcn_sched_barrier(0);
// FP4: a scheduling barrier between steps only; the compiler interleaves
// the four A-row ANDs of each row tile with the products itself
#define EPI3_SCHED4 __builtin_amdgcn_sched_barrier(0);
#define EPI3_STEP(P, X, B0, B1)                                                     \
    EPI3_TILE(0, P, X, B0, B1)                                                    \
    EPI3_TILE(1, P, X, B0, B1)                                                    \
    EPI3_TILE(2, P, X, B0, B1)                                                    \
    EPI3_TILE(3, P, X, B0, B1)
    v4i pX, xX, b0X, b1X, pY, xY, b0Y, b1Y;
    EPI3_LD(stage, 0, pX, xX, b0X, b1X)
    for (int ch = 0; ch < nch; ++ch) {
      const bool more = ch + 1 < nch;
      if (more) fetch(ch + 1);
      const uint8_t *buf = stage + (ch & 1) * kStageBytes;
      const uint8_t *nbuf = stage + ((ch + 1) & 1) * kStageBytes;
      if constexpr (FP4) {
        EPI3_LD(buf, 1, pY, xY, b0Y, b1Y)
        EPI3_STEP(pX, xX, b0X, b1X)
        EPI3_SCHED4
        EPI3_LD(buf, 2, pX, xX, b0X, b1X)
        EPI3_STEP(pY, xY, b0Y, b1Y)
        EPI3_SCHED4
        EPI3_LD(buf, 3, pY, xY, b0Y, b1Y)
        tA = *reinterpret_cast<const v4i *>(buf + o_ta);
        tB = *reinterpret_cast<const v4i *>(buf + o_tb);
        EPI3_STEP(pX, xX, b0X, b1X)
        tacc = tot_mma(tA, tB, tacc);
        EPI3_SCHED4
      } else {
        EPI3_LD(buf, 1, pY, xY, b0Y, b1Y)
        EPI3_STEP(pX, xX, b0X, b1X)
        EPI3_SCHED
        EPI3_LD(buf, 2, pX, xX, b0X, b1X)
        EPI3_STEP(pY, xY, b0Y, b1Y)
        EPI3_SCHED
        EPI3_LD(buf, 3, pY, xY, b0Y, b1Y)
        EPI3_STEP(pX, xX, b0X, b1X)
        EPI3_SCHED
      }
      // the products above stay before the branch (they would otherwise be
      // sunk to their first use below it)
#pragma unroll
      for (int tt = 0; tt < kPermT; ++tt) asm volatile("" : "+v"(acc[tt][0]), "+v"(acc[tt][1]));
      if constexpr (FP4) asm volatile("" : "+v"(tacc));
      if (more) store((ch + 1) & 1);
      __syncthreads();
      // after the last chunk this reads the other buffer's stale contents,
      // which no product uses
      EPI3_LD(nbuf, 0, pX, xX, b0X, b1X)
      EPI3_STEP(pY, xY, b0Y, b1Y)
      if constexpr (FP4) {
        EPI3_SCHED4
      } else {
        EPI3_SCHED
      }
    }
#undef EPI3_LD
#undef EPI3_TILE
#undef EPI3_SCHED
#undef EPI3_SCHED4
#undef EPI3_STEP

    if constexpr (FP4) {
      // lane l holds column l % 16 = (k = 8 tkh + (l % 16) / 2, c = l % 2) and
      // rows 4 (l / 16) + v = (pivot l / 16, (a, b) = v)
      if (tsh == 1) {
#pragma unroll
        for (int v = 0; v < 4; ++v) sTot[tkh][lane][v] = tacc[v];
      }
      __syncthreads();
      if (tsh == 0) {
        const int p = lane >> 4;
        if (4 * ib + p < j) {
          uint16_t *t16 = FUSE ? reinterpret_cast<uint16_t *>(&sT16[p][0])
                               : reinterpret_cast<uint16_t *>(pj.totals + (slot * 4 + p) * (int64_t)kPermKB);
          const int kl = 8 * tkh + ((lane & 15) >> 1), c = lane & 1;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            t16[kl * 8 + 2 * v + c] = (uint16_t)(uint32_t)(tacc[v] + sTot[tkh][lane][v]);
        }
      }
      if constexpr (FUSE != 0) __syncthreads();  // sT16 complete
    }
    if (i >= j) continue;  // padding pivot of the last i-block: nothing to write
    if constexpr (FUSE != 0) {
      // the staging buffers are idle until the next tile's first store
      __builtin_amdgcn_s_setprio(0);
      fused_score<FUSE>(pj, acc, sT16[wave], reinterpret_cast<uint32_t *>(stage + wave * 4096), st,
                        out, i, j, kbase, slot, wave, lane, kmin, kmax);
      continue;
    }

    // ---- counts out: all-sample corner cells per triplet, case corner cells
    // per (triplet, phenotype); the finish kernel completes tables and scores.
    uint4 *cor = pj.corners + (slot * 4 + wave) * (int64_t)kPermKB * 64;
    if constexpr (!FP4) {
      uint16_t *tot16 = reinterpret_cast<uint16_t *>(pj.totals + (slot * 4 + wave) * (int64_t)kPermKB);
#pragma unroll
      for (int tt = 0; tt < kPermT; ++tt) {
        const uint32_t full = tot[tt] + __shfl_xor(tot[tt], 32);
        if (g == 0) tot16[(4 * tt + ta) * 8 + 4 * ra + 2 * rb + rc] = (uint16_t)full;
      }
    }
    // lane (q, h) holds, for each of the 4 triplets of a row tile, the 4 case
    // cells with genotype c = h at SNP k: registers 4 t + (2 a + b).  Each lane
    // writes them as 4 x uint16; halves h = 0, 1 of one (triplet, phenotype)
    // are adjacent, so the 16 bytes hold cells in the order 4 c + 2 a + b.
    uint2 *cor2 = reinterpret_cast<uint2 *>(cor);
#pragma unroll
    for (int tt = 0; tt < kPermT; ++tt)
#pragma unroll
      for (int qb = 0; qb < 2; ++qb)
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4) {
          const uint32_t c0 = Acc::get(acc[tt][qb], 4 * t4 + 0), c1 = Acc::get(acc[tt][qb], 4 * t4 + 1);
          const uint32_t c2 = Acc::get(acc[tt][qb], 4 * t4 + 2), c3 = Acc::get(acc[tt][qb], 4 * t4 + 3);
          cor2[((4 * tt + t4) * 64 + qb * 32 + r) * 2 + g] = make_uint2(c0 | (c1 << 16), c2 | (c3 << 16));
        }
  }
  if constexpr (FUSE != 0) {
    const int Q = pj.Q;
    if (lane < Q && kmax != 0u) {
      atomicMin(&sRange[lane][0], kmin);
      atomicMax(&sRange[lane][1], kmax);
    }
    __syncthreads();
    if (tid < 64 && tid < Q && sRange[tid][1] != 0u) {
      atomicMin(&st[tid].kmin, sRange[tid][0]);
      atomicMax(&st[tid].kmax, sRange[tid][1]);
    }
  }
}

// LDS: double-buffered staging, the tile slot, the FP4 totals exchange.
template <bool FP4>
__global__ void __launch_bounds__(256, 2) count_mfma_perm_kernel(
    const PermJob *__restrict__ pjp, int64_t tile_begin, int64_t n_tiles, int64_t stride,
    unsigned long long *__restrict__ queue) {
  __shared__ __attribute__((aligned(16))) unsigned char stage[2 * kStageBytes];
  __shared__ int64_t sTile[2];
  // FP4: all-sample corner counts of half the samples from the waves of the
  // second half, added by the waves of the first half
  __shared__ float sTot[2][64][4];
  const PermOut none{};
  count_perm_body<FP4, 0>(pjp, tile_begin, n_tiles, stride, queue, nullptr, nullptr, 0, none, stage,
                          sTile, sTot, nullptr, nullptr, nullptr);
}

// Dynamic LDS only, so the log-factorial table starts at LDS address 0 and a
// lookup is one ds_read at the byte offset: [table][staging][tile slot]
// [totals exchange][the tile's all-sample cells][key ranges].
template <int FUSE>
__global__ void __launch_bounds__(256, 2) count_score_perm_kernel(
    const PermJob *__restrict__ pjp, int64_t tile_begin, int64_t n_tiles, int64_t stride,
    unsigned long long *__restrict__ queue, SelState *__restrict__ st,
    const float *__restrict__ lf32, int lf_len, PermOut out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  unsigned char *stage = lds + finish_perm_table_bytes(lf_len);
  int64_t *sTile = reinterpret_cast<int64_t *>(stage + 2 * kStageBytes);
  float(*sTot)[64][4] = reinterpret_cast<float(*)[64][4]>(sTile + 2);
  uint4(*sT16)[kPermKB] = reinterpret_cast<uint4(*)[kPermKB]>(sTot + 2);
  uint32_t(*sRange)[2] = reinterpret_cast<uint32_t(*)[2]>(sT16 + 4);
  count_perm_body<true, FUSE>(pjp, tile_begin, n_tiles, stride, queue, st, lf32, lf_len, out, stage,
                              sTile, sTot, sT16, sRange, reinterpret_cast<float *>(lds));
}

// Completes the tables of one pass of tiles and scores them.  Workgroup per
// tile (persistent, round robin); wave w = pivot i = 4 ib + w.  First the
// wave's lanes 0..15 complete the all-sample tables of the tile's 16 triplets
// (one k each) and keep the cells in registers; then lane = phenotype q
// loops over the 16 k, reading lane k's cells into scalar registers
// (readlane) and their L[cell + 1] by scalar loads, and completes and scores
// its case table.  Case cells are handled as 4 x count
// (byte offsets into the table), so each lookup needs no index arithmetic.
// Per-phenotype corner cells and case pair tables are contiguous 1 KB rows;
// scores are staged per wave in LDS and written as 64-byte runs of
// consecutive ranks.  (Visiting the tiles by (i-block, k-block) instead, so
// that one XCD's L2 serves a block pair's case tables to several pivots j,
// measured slower.)
// Dynamic LDS of the finish kernel: [log-factorial table (LDS variant)] then
// the per-wave staged scores and the key ranges.  The kernel
// declares no static LDS, so the dynamic block and with it the table start at
// LDS address 0 and a lookup is one ds_read at the byte offset.
struct FinishPermLds {
  uint32_t range[64][2];
  float score[4][kPermKB][64];  // staged scores (score-plane mode only)
};
// Bytes of the block after the table: the sample and bounded modes leave the
// score staging out (more workgroups per CU).
__host__ __device__ constexpr size_t finish_perm_lds_bytes(int mode) {
  return mode == kPermOutPlane ? sizeof(FinishPermLds) : offsetof(FinishPermLds, score);
}

template <bool LDS, int MODE>
__global__ void __launch_bounds__(256) finish_perm_kernel(const PermJob *__restrict__ pjp,
                                                          int64_t tile_begin, int64_t n_tiles,
                                                          int64_t stride,
                                                          SelState *__restrict__ st,
                                                          const float *__restrict__ lf32,
                                                          int lf_len, PermOut out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  const float *sL = lf32;
  FinishPermLds &sh = *reinterpret_cast<FinishPermLds *>(lds + (LDS ? finish_perm_table_bytes(lf_len) : 0));
  if (LDS) {
    float *tab = reinterpret_cast<float *>(lds);
    for (int x = threadIdx.x; x < lf_len; x += blockDim.x) tab[x] = lf32[x];
    sL = tab;
  }
  if (threadIdx.x < 64) {
    sh.range[threadIdx.x][0] = 0xffffffffu;
    sh.range[threadIdx.x][1] = 0u;
  }
  __syncthreads();
  const PermJob pj = *pjp;
  const int q = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int M = pj.M, Mp = pj.Mp, Q = pj.Q, Qp = pj.Qp;
  const int64_t T = pj.T;
  cptr<int64_t> pre = as_const(pj.jprefix);
  const int4 *tp = reinterpret_cast<const int4 *>(pj.tot_pairs);
  typedef unsigned u4e __attribute__((ext_vector_type(4)));
  typedef unsigned u2e __attribute__((ext_vector_type(2)));
  gptr<u2e> cp = (gptr<u2e>)pj.case_pairs;
  // case pair words -> 4 x counts (byte offsets into the log-factorial table)
  auto lo4 = [](unsigned v) { return (int)((v & 0xffffu) << 2); };
  auto hi4 = [](unsigned v) { return (int)((v >> 16) << 2); };
  gptr<u4e> corners = (gptr<u4e>)pj.corners;
  const int qc = q < Q ? q : 0;  // lanes past Q compute on phenotype 0 and write nothing
  const int n1x4 = pj.n1[qc] << 2;
  // bounded: this phenotype's append bound (set before the launch)
  const float ubq = MODE == kPermOutBounded ? st[qc].ub : 0.f;
  uint32_t kmin = 0xffffffffu, kmax = 0u;
  // pivot of tile t
  auto pivot_of = [&](int64_t t) {
    int lo = 0, hi = M - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  // row of phenotype-major case pair tables for pair (x, y) (uniform)
  auto cp_row = [&](int x, int y) { return cp + ((int64_t)x * Mp + y) * Qp; };
  for (int64_t slot = blockIdx.x; slot < n_tiles; slot += gridDim.x) {
    const int64_t t = tile_begin + slot * stride;
    const int j = pivot_of(t);
    const int64_t rr = t - pre[j];
    // the quotient comes out of vector instructions: taken back to a scalar
    // register, so the row addresses below are formed by scalar arithmetic
    const int nkb_j = perm_nkb(M, j);
    int ib_, kb_;
    perm_tile_ib_kb((int)rr, j, nkb_j, ib_, kb_);
    const int ib = __builtin_amdgcn_readfirstlane(ib_);
    const int kbg = perm_kb_lo(j) + __builtin_amdgcn_readfirstlane(kb_);
    const int i = 4 * ib + wave;
    const int k0 = kbg * kPermKB;
    if (i >= j) continue;  // wave-uniform
    gptr<u4e> cor = corners + (slot * 4 + wave) * (int64_t)kPermKB * 64;
    const int64_t tbase = (slot * 4 + wave) * (int64_t)kPermKB;
    const int kk_lo = j + 1 - k0 > 0 ? j + 1 - k0 : 0;
    const int kk_hi = M - k0 < kPermKB ? M - k0 : kPermKB;
    // ---- all-sample tables, lane kk = triplet (i, j, k0 + kk) ----
    // Kept in registers, two cell counts per register (16 bits each); the
    // phenotype loop below reads lane kk's counts into scalar registers and
    // fetches L[count + 1] by scalar loads, so neither LDS bandwidth nor
    // vector instructions are spent broadcasting them.
    uint32_t pk[14];
#pragma unroll
    for (int x = 0; x < 14; ++x) pk[x] = 0u;
    if (q >= kk_lo && q < kk_hi) {
      const int k = k0 + q;
      const uint4 tq = pj.totals[tbase + q];
      const uint32_t tn[8] = {(tq.x & 0xffffu) << 2, (tq.x >> 16) << 2, (tq.y & 0xffffu) << 2,
                              (tq.y >> 16) << 2, (tq.z & 0xffffu) << 2, (tq.z >> 16) << 2,
                              (tq.w & 0xffffu) << 2, (tq.w >> 16) << 2};
      const int4 a = tp[(int64_t)i * Mp + j], b = tp[(int64_t)i * Mp + k], c = tp[(int64_t)j * Mp + k];
      const int4 ii4 = tp[(int64_t)i * Mp + i], jj4 = tp[(int64_t)j * Mp + j], kk4 = tp[(int64_t)k * Mp + k];
      const int tij[4] = {a.x << 2, a.y << 2, a.z << 2, a.w << 2};
      const int tik[4] = {b.x << 2, b.y << 2, b.z << 2, b.w << 2};
      const int tjk[4] = {c.x << 2, c.y << 2, c.z << 2, c.w << 2};
      const int mi[2] = {ii4.x << 2, ii4.w << 2}, mj[2] = {jj4.x << 2, jj4.w << 2};
      const int mk[2] = {kk4.x << 2, kk4.w << 2};
      int t4[27];
      complete_table(tn, tij, tik, tjk, mi, mj, mk, pj.N << 2, t4);
#pragma unroll
      for (int x = 0; x < 27; ++x) pk[x >> 1] |= ((uint32_t)t4[x] >> 2) << (16 * (x & 1));
    }
    // ---- case tables and scores, lane = phenotype q ----
    const u2e cij = cp_row(i, j)[qc];
    const u2e cii = cp_row(i, i)[qc], cjj = cp_row(j, j)[qc];
    const int aij[4] = {lo4(cij.x), hi4(cij.x), lo4(cij.y), hi4(cij.y)};
    const int mi[2] = {lo4(cii.x), hi4(cii.y)}, mj[2] = {lo4(cjj.x), hi4(cjj.y)};
    // loads of the next k are issued before the current k is scored; the
    // (uniform) row pointers advance by one k per step, each load being a
    // scalar base plus the lane's phenotype offset
    gptr<u4e> pq = cor + kk_lo * 64;
    gptr<u2e> pik = cp_row(i, k0 + kk_lo), pjk = cp_row(j, k0 + kk_lo);
    gptr<u2e> pkk = cp_row(k0 + kk_lo, k0 + kk_lo);
    const int64_t dkk = (int64_t)(Mp + 1) * Qp;
    u4e cq_n = pq[qc];
    u2e cik_n = pik[qc], cjk_n = pjk[qc], ckk_n = pkk[qc];
    for (int kk = kk_lo; kk < kk_hi; ++kk) {
      const u4e cq = cq_n;
      const u2e cik = cik_n, cjk = cjk_n, ckk = ckk_n;
      if (kk + 1 < kk_hi) {
        pq += 64;
        pik += Qp;
        pjk += Qp;
        pkk += dkk;
        cq_n = pq[qc];
        cik_n = pik[qc];
        cjk_n = pjk[qc];
        ckk_n = pkk[qc];
      }
      int c4[27];
      {
        // record order 4 c + 2 a + b -> corner index 4 a + 2 b + c; x 4
        const uint32_t cn[8] = {(cq.x << 2) & 0x3fffcu, (cq.z << 2) & 0x3fffcu,
                                (cq.x >> 14) & 0x3fffcu, (cq.z >> 14) & 0x3fffcu,
                                (cq.y << 2) & 0x3fffcu, (cq.w << 2) & 0x3fffcu,
                                (cq.y >> 14) & 0x3fffcu, (cq.w >> 14) & 0x3fffcu};
        const int aik[4] = {lo4(cik.x), hi4(cik.x), lo4(cik.y), hi4(cik.y)};
        const int ajk[4] = {lo4(cjk.x), hi4(cjk.x), lo4(cjk.y), hi4(cjk.y)};
        const int mk[2] = {lo4(ckk.x), hi4(ckk.y)};
        complete_table(cn, aij, aik, ajk, mi, mj, mk, n1x4, c4);
      }
      uint32_t spk[14];
#pragma unroll
      for (int x = 0; x < 14; ++x) spk[x] = __builtin_amdgcn_readlane(pk[x], kk);
      float k2 = 0.f;  // rows in order: L[r + 1] - (L[r_0] + L[r_1]), r_1 = cases
#pragma unroll
      for (int x = 0; x < 27; ++x) {
        const uint32_t nall = (spk[x >> 1] >> (16 * (x & 1))) & 0xffffu;
        const int tall = (int)(nall << 2);
        const float l1 = lf32[nall + 1];  // uniform address: a scalar load
        const int r0 = tall - c4[x];
        if (LDS)
          k2 += l1 - (lf_at_lds0(r0) + lf_at_lds0(c4[x]));
        else
          k2 += l1 - (lf_at(sL, r0) + lf_at(sL, c4[x]));
      }
      const uint32_t key = f2key(k2);
      kmin = key < kmin ? key : kmin;
      kmax = key > kmax ? key : kmax;
      if (MODE == kPermOutPlane) sh.score[wave][kk][q] = k2;
      if (MODE == kPermOutSample && q < Q)
        out.sample[(int64_t)q * out.sample_T + (out.sample_base + slot) * 64 + wave * kPermKB + kk] = k2;
      if (MODE == kPermOutBounded && q < Q && k2 <= ubq) {
        // rare (a few thousand of the C(M,3) scores per phenotype): one atomic per append
        const unsigned long long pos = atomicAdd(&st[q].cn, 1ull);
        if ((int64_t)pos < out.ccap) {
          out.ckey[(int64_t)q * out.ccap + pos] = key;
          out.crank[(int64_t)q * out.ccap + pos] = lex_base(M, i, j) + k0 + kk;
        }
      }
    }
    if (MODE != kPermOutPlane) continue;
    // scores of phenotype q at ranks base + k (this wave wrote them)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t base = lex_base(M, i, j) + k0;
#pragma unroll
    for (int e0 = 0; e0 < kPermKB * 64; e0 += 64) {
      const int e = e0 + q, qq = e / kPermKB, kk = e % kPermKB;
      if (qq < Q && kk >= kk_lo && kk < kk_hi) pj.score[(int64_t)qq * T + base + kk] = sh.score[wave][kk][qq];
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (q < Q && kmax != 0u) {
    atomicMin(&sh.range[q][0], kmin);
    atomicMax(&sh.range[q][1], kmax);
  }
  __syncthreads();
  if (threadIdx.x < 64 && threadIdx.x < Q && sh.range[threadIdx.x][1] != 0u) {
    atomicMin(&st[threadIdx.x].kmin, sh.range[threadIdx.x][0]);
    atomicMax(&st[threadIdx.x].kmax, sh.range[threadIdx.x][1]);
  }
}

hipError_t launch_perm_prefix(PermJob *pj_dev, hipStream_t s) {
  hipLaunchKernelGGL(perm_prefix_kernel, dim3(1), dim3(1024), 0, s, pj_dev);
  return hipGetLastError();
}

hipError_t launch_mask_bytes(const uint32_t *const *masks_dev, int32_t Q, int32_t Qp, int32_t N,
                             int32_t S, uint8_t *ph, int32_t *n1, bool fp4, hipStream_t s) {
  hipLaunchKernelGGL(mask_bytes_kernel, dim3(Qp), dim3(256), 0, s, masks_dev, Q, N, S, ph, n1,
                     fp4 ? 1 : 0);
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

template <bool FP4, int FUSE>
static hipError_t launch_count_t(const PermJob *pj_dev, int64_t tile_begin, int64_t n_tiles,
                                 int64_t stride, unsigned long long *queue, SelState *st,
                                 const float *lf32, int32_t lf_len, const PermOut &out,
                                 hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  if constexpr (FUSE == 0) {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, count_mfma_perm_kernel<FP4>, 256, 0);
    if (e != hipSuccess) return e;
    if (per_cu <= 0) per_cu = 1;
    int64_t blocks = (int64_t)n_cu * per_cu;
    if (blocks > n_tiles) blocks = n_tiles;
    hipLaunchKernelGGL(count_mfma_perm_kernel<FP4>, dim3((unsigned)blocks), dim3(256), 0, s, pj_dev,
                       tile_begin, n_tiles, stride, queue);
  } else {
    const size_t lds = (size_t)perm_score_lds_bytes(lf_len);
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&count_score_perm_kernel<FUSE>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, count_score_perm_kernel<FUSE>, 256, lds);
    if (e != hipSuccess) return e;
    if (per_cu <= 0) per_cu = 1;
    int64_t blocks = (int64_t)n_cu * per_cu;
    if (blocks > n_tiles) blocks = n_tiles;
    hipLaunchKernelGGL(count_score_perm_kernel<FUSE>, dim3((unsigned)blocks), dim3(256), lds, s,
                       pj_dev, tile_begin, n_tiles, stride, queue, st, lf32, lf_len, out);
  }
  return hipGetLastError();
}

// queue: 8 zeroed 64-bit counters (one per XCD part of the pass).
hipError_t launch_count_mfma_perm(const PermJob *pj_dev, int64_t tile_begin, int64_t n_tiles,
                                  int64_t stride, unsigned long long *queue, bool fp4,
                                  hipStream_t s) {
  const PermOut none{};
  return fp4 ? launch_count_t<true, 0>(pj_dev, tile_begin, n_tiles, stride, queue, nullptr, nullptr,
                                       0, none, s)
             : launch_count_t<false, 0>(pj_dev, tile_begin, n_tiles, stride, queue, nullptr,
                                        nullptr, 0, none, s);
}

bool perm_fused_ok(int32_t lf_len) {
  return lf_len > 0 && perm_score_lds_bytes(lf_len) <= 80 * 1024;  // two workgroups per CU
}

hipError_t launch_count_score_perm(const PermJob *pj_dev, int64_t tile_begin, int64_t n_tiles,
                                   int64_t stride, unsigned long long *queue, SelState *st,
                                   const float *lf32, int32_t lf_len, const PermOut &out,
                                   hipStream_t s) {
  if (!perm_fused_ok(lf_len)) return hipErrorInvalidValue;
  if (out.mode == kPermOutSample)
    return launch_count_t<true, kPermOutSample>(pj_dev, tile_begin, n_tiles, stride, queue, st, lf32,
                                                lf_len, out, s);
  if (out.mode == kPermOutBounded)
    return launch_count_t<true, kPermOutBounded>(pj_dev, tile_begin, n_tiles, stride, queue, st, lf32,
                                                 lf_len, out, s);
  return hipErrorInvalidValue;
}

template <bool LDS, int MODE>
static hipError_t launch_finish_perm_l(const PermJob *pj_dev, int64_t tile_begin, int64_t n_tiles,
                                       int64_t stride, SelState *st, const float *lf32,
                                       int32_t lf_len, const PermOut &out, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const size_t lds = (LDS ? (size_t)finish_perm_table_bytes(lf_len) : 0) + finish_perm_lds_bytes(MODE);
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(&finish_perm_kernel<LDS, MODE>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, finish_perm_kernel<LDS, MODE>, 256, lds);
  if (e != hipSuccess) return e;
  if (per_cu <= 0) per_cu = 1;
  int64_t blocks = (int64_t)n_cu * per_cu;
  if (blocks > n_tiles) blocks = n_tiles;
  hipLaunchKernelGGL((finish_perm_kernel<LDS, MODE>), dim3((unsigned)blocks), dim3(256), lds, s,
                     pj_dev, tile_begin, n_tiles, stride, st, lf32, lf_len, out);
  return hipGetLastError();
}

template <bool LDS>
static hipError_t launch_finish_perm_m(const PermJob *pj_dev, int64_t tile_begin, int64_t n_tiles,
                                       int64_t stride, SelState *st, const float *lf32,
                                       int32_t lf_len, const PermOut &out, hipStream_t s) {
  switch (out.mode) {
    case kPermOutPlane:
      return launch_finish_perm_l<LDS, kPermOutPlane>(pj_dev, tile_begin, n_tiles, stride, st, lf32,
                                                     lf_len, out, s);
    case kPermOutSample:
      return launch_finish_perm_l<LDS, kPermOutSample>(pj_dev, tile_begin, n_tiles, stride, st,
                                                      lf32, lf_len, out, s);
    case kPermOutBounded:
      return launch_finish_perm_l<LDS, kPermOutBounded>(pj_dev, tile_begin, n_tiles, stride, st,
                                                       lf32, lf_len, out, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_finish_perm(const PermJob *pj_dev, int64_t tile_begin, int64_t n_tiles,
                              int64_t stride, SelState *st, const float *lf32, int32_t lf_len,
                              const PermOut &out, hipStream_t s) {
  return lf_in_lds(lf_len)
             ? launch_finish_perm_m<true>(pj_dev, tile_begin, n_tiles, stride, st, lf32, lf_len, out, s)
             : launch_finish_perm_m<false>(pj_dev, tile_begin, n_tiles, stride, st, lf32, lf_len, out, s);
}

int64_t host_perm_sample_valid(int64_t M, int64_t stride) {
  int64_t valid = 0, pre = 0;
  for (int64_t j = 0; j < M; ++j) {
    const int64_t nt = perm_tiles_of_j(M, j);
    if (nt > 0) {
      const int nkb = perm_nkb(M, j);
      for (int64_t t = (pre + stride - 1) / stride * stride; t < pre + nt; t += stride) {
        const int64_t rr = t - pre;
        int ib_, kb_;
        perm_tile_ib_kb((int)rr, (int)j, nkb, ib_, kb_);
        const int64_t ib = ib_, kb = kb_;
        const int64_t ni = std::max<int64_t>(0, std::min<int64_t>(4, j - 4 * ib));
        const int64_t kbase = (perm_kb_lo(j) + kb) * kPermKB;
        const int64_t nk = std::max<int64_t>(
            0, std::min<int64_t>(kbase + kPermKB, M) - std::max<int64_t>(kbase, j + 1));
        valid += ni * nk;
      }
    }
    pre += nt;
  }
  return valid;
}

}  // namespace epi3
