// Count stage of the plain (two-class) scan on the matrix cores.
//
// For one class c, the corner cells of every triplet (i, j, k) are entries
// of matrix products over that class's samples:
//     C[(i, j, a, b), (k, g)] = sum_s (X_i[a][s] X_j[b][s]) X_k[g][s],
// rows (i, j, a, b), columns (k, g), K = the class's samples, 0/1 values
// (int8 bytes or FP4 nibbles) and exact accumulation.  This is the same
// integer table the paper fills with AND + POPCNT (Alg. 2); the other 19
// cells of each class follow from the pairwise tables as in the vector-ALU
// kernel.  Counting writes the 8 corner cells of both classes of every
// triplet of a pass of tiles to a scratch buffer; a second kernel completes
// the tables and scores them (Eq. 1, FP32).
//
// Workgroup tile: 16 consecutive i, JB consecutive j, 256 / JB consecutive
// k (4096 triplets), so one staged sample chunk serves 16 + JB + 256 / JB
// SNPs instead of the 161 of a (32 i, one j, 128 k) slab.  Each of the 4
// waves owns 2 i-blocks of 8 x 2 j (four 32-row A tiles: 8 i x (a, b), the
// rows X_i[a] & X_j[b] formed in registers) and two 32-column B tiles
// (16 k x g).  Operand rows are staged per chunk of 128 bytes (64 for
// JB = 2) in double-buffered LDS.
#include <algorithm>

#include "epi3_internal.h"

namespace epi3 {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

constexpr int kPI = kPlainI;   // i per workgroup tile

// Bytes per staged chunk of a row: 128 (four steps per barrier), 64 for
// JB = 2, whose 176 rows would otherwise take more than half of the LDS.
// Rows are padded by 16 bytes against bank conflicts.
__host__ __device__ constexpr int plain_chunk(int JB) { return JB == 2 ? 64 : 128; }

__host__ __device__ __forceinline__ int plain_kt(int JB) { return 256 / JB; }

// Tiles of j-block J (j in [JB J, JB J + JB)): i-blocks of 16 below the
// block's last pivot, k-blocks of 256 / JB from JB J + 1 up to M - 1.
__host__ __device__ __forceinline__ int64_t plain_tiles_of_jb(int64_t M, int64_t J, int JB) {
  const int64_t j0 = J * JB;
  int64_t jmax = j0 + JB - 1;
  if (jmax > M - 2) jmax = M - 2;
  if (jmax < 1 || j0 > M - 2) return 0;
  const int KT = plain_kt(JB);
  return ((jmax + kPI - 1) / kPI) * ((M - 1 - j0 + KT - 1) / KT);
}

__host__ __device__ __forceinline__ int64_t plain_jblocks(int64_t M, int JB) {
  return M < 3 ? 0 : (M - 1 + JB - 1) / JB;
}

// Lane n of every quad takes x from quad lane (SEL >> 2 n) & 3 (DPP
// quad_perm; the compiler folds it into the instruction that consumes it
// where it can).
template <int SEL>
__device__ __forceinline__ v4i quad_perm(v4i x) {
  v4i y;
  y.x = __builtin_amdgcn_update_dpp(0, x.x, SEL, 0xf, 0xf, true);
  y.y = __builtin_amdgcn_update_dpp(0, x.y, SEL, 0xf, 0xf, true);
  y.z = __builtin_amdgcn_update_dpp(0, x.z, SEL, 0xf, 0xf, true);
  y.w = __builtin_amdgcn_update_dpp(0, x.w, SEL, 0xf, 0xf, true);
  return y;
}

__device__ __forceinline__ int64_t rfl64q(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// jprefix[J] = tiles before j-block J; jprefix[nJ] = total.
__global__ void __launch_bounds__(1024) plain_prefix_kernel(PlainJob *pj) {
  const int64_t M = pj->M;
  const int JB = pj->JB;
  const int64_t nJ = plain_jblocks(M, JB);
  int64_t *pre = const_cast<int64_t *>(pj->jprefix);
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (nJ + 1023) / 1024;
  const int64_t a = t * chunk, b = (a + chunk < nJ) ? a + chunk : nJ;
  int64_t sum = 0;
  for (int64_t J = a; J < b; ++J) sum += plain_tiles_of_jb(M, J, JB);
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - sum;
  for (int64_t J = a; J < b; ++J) {
    pre[J] = run;
    run += plain_tiles_of_jb(M, J, JB);
  }
  if (t == 1023) pre[nJ] = part[1023];
}

template <bool FP4>
struct PlainAcc {
  typedef v16i type;
  static __device__ __forceinline__ type mma(v4i a, v4i b, type c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ uint32_t get(const type &c, int v) { return (uint32_t)c[v]; }
};
template <>
struct PlainAcc<true> {
  typedef v16f type;
  static __device__ __forceinline__ type mma(v4i a, v4i b, type c) {
    const v8i a8 = {a.x, a.y, a.z, a.w, 0, 0, 0, 0};
    const v8i b8 = {b.x, b.y, b.z, b.w, 0, 0, 0, 0};
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, c, 4, 4, 0, 127, 0, 127);
  }
  static __device__ __forceinline__ uint32_t get(const type &c, int v) { return (uint32_t)c[v]; }
};

// Decodes a tile index into its j-block through the prefix table.
struct TileDecoder {
  int J = -1;
  int64_t jlo = 0, jhi = 0;
  __device__ __forceinline__ void find(cptr<int64_t> pre, int nJ, int64_t t) {
    if (J < 0 || t < jlo || t >= jhi) {
      int lo = 0, hi = nJ - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= t) lo = mid; else hi = mid - 1;
      }
      J = lo;
      jlo = pre[J];
      jhi = pre[J + 1];
    }
  }
};

// (i0, j0, k0) of tile t of j-block J.
__device__ __forceinline__ void plain_tile_origin(const TileDecoder &dec, int64_t t, int M, int JB,
                                                  int &i0, int &j0, int &k0) {
  const int KT = 256 / JB;
  j0 = dec.J * JB;
  const int nkb = (M - 1 - j0 + KT - 1) / KT;
  const int rr = (int)(t - dec.jlo);
  const int ib = rr / nkb, kb = rr - ib * nkb;
  i0 = ib * kPI;
  k0 = j0 + 1 + kb * KT;
}

// Finds the job of global tile t: jobs own consecutive ranges of the tile
// order, job_begin[x] .. job_begin[x + 1] (uniform: scalar loads).
struct JobDecoder {
  int x = -1;
  int64_t lo = 0, hi = 0;
  __device__ __forceinline__ bool find(cptr<int64_t> job_begin, int n_jobs, int64_t t) {
    if (x >= 0 && t >= lo && t < hi) return false;
    int a = 0, b = n_jobs - 1;
    while (a < b) {
      const int mid = (a + b + 1) >> 1;
      if (job_begin[mid] <= t) a = mid; else b = mid - 1;
    }
    x = a;
    lo = job_begin[a];
    hi = job_begin[a + 1];
    return true;
  }
};

template <bool FP4, int JB>
__global__ void __launch_bounds__(256, 2) count_mfma_plain_kernel(
    const PlainJob *__restrict__ jobs, const int64_t *__restrict__ job_begin_p, int n_jobs,
    uint4 *__restrict__ corners, int64_t tile_begin, int64_t n_tiles, int64_t stride,
    unsigned long long *__restrict__ queue) {
  typedef PlainAcc<FP4> Acc;
  constexpr int KT = 256 / JB;
  constexpr int kPKC = plain_chunk(JB), kPRow = kPKC + 16;
  constexpr int kRowsI = 2 * kPI, kRowsJ = 2 * JB, kRowsK = 2 * KT;
  constexpr int kRows = kRowsI + kRowsJ + kRowsK;
  constexpr int kBuf = kRows * kPRow;
  constexpr int kChunks = kRows * (kPKC / 16);
  constexpr int kPer = (kChunks + 255) / 256;
  constexpr int NBP = KT / 32;  // pairs of B tiles; the 4 waves are (JB / 2) x NBP
  static_assert((JB / 2) * NBP == 4, "four waves per tile");
  __shared__ __attribute__((aligned(16))) unsigned char stage[2 * kBuf];
  __shared__ int64_t sTile[2];

  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wj = wave / NBP, wb = wave - wj * NBP;
  const int r = lane & 31, g = lane >> 5;
  cptr<int64_t> job_begin = as_const(job_begin_p);
  JobDecoder jd;
  int M = 0, Mp = 0, Sb = 0, Sb0 = 0, Sb1 = 0, nJ = 0;
  gptr<uint8_t> gv = nullptr;
  cptr<int64_t> pre = nullptr;
  TileDecoder dec;
  // lane roles: A row r = 4 i8 + 2 a + b; B column r = 2 k16 + g_k
  const int ri8 = r >> 2, ra = (r >> 1) & 1, rb = r & 1;
  const int ck16 = r >> 1, cpl = r & 1;
  // LDS byte offsets (within a buffer) of the rows this lane loads for its quad
  const int xi_off = (2 * (8 * rb + ri8) + ra) * kPRow;
  const int xj_off = (kRowsI + 2 * (2 * wj + ra) + rb) * kPRow;

  for (;;) {
    __syncthreads();
    if (tid == 0) sTile[0] = (int64_t)atomicAdd(queue, 1ull);
    __syncthreads();
    const int64_t slot = rfl64q(sTile[0]);  // scratch slot of this launch
    if (slot >= n_tiles) break;
    const int64_t tg = tile_begin + slot * stride;
    if (jd.find(job_begin, n_jobs, tg)) {
      const PlainJob &pj = jobs[jd.x];
      M = pj.M;
      Mp = pj.Mp;
      Sb = pj.Sb;
      Sb0 = pj.Sb0;
      Sb1 = pj.Sb1;
      nJ = (int)plain_jblocks(M, JB);
      gv = (gptr<uint8_t>)pj.vals;
      pre = as_const(pj.jprefix);
      dec.J = -1;
    }
    const int64_t t = tg - jd.lo;  // tile within its job
    dec.find(pre, nJ, t);
    int i0, j0, k0;
    plain_tile_origin(dec, t, M, JB, i0, j0, k0);

    for (int cls = 0; cls < 2; ++cls) {
      // the class's bytes rounded up to whole chunks (rows are zero-padded
      // to a multiple of 128 bytes)
      const int nch = ((cls ? Sb1 : Sb0) + kPKC - 1) / kPKC;
      const int64_t cbase = (int64_t)cls * Mp * 2;  // first row of this class
      // staging plan: rows [0, 32) X_i (i0 + x / 2, plane x % 2), then 2 JB
      // rows X_j, then 2 KT rows X_k (k0 + x / 2, plane x % 2)
      // 32-bit byte offsets of this thread's 16-byte pieces (the value planes
      // are far below 4 GB), so each load is a scalar base plus one VGPR
      constexpr int kPieces = kPKC / 16;
      uint32_t off[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int c16 = tid + 256 * u;
        const int row = c16 / kPieces < kRows ? c16 / kPieces : kRows - 1, col = (c16 % kPieces) * 16;
        int snp, pl;
        if (row < kRowsI) { snp = i0 + (row >> 1); pl = row & 1; }
        else if (row < kRowsI + kRowsJ) { const int x = row - kRowsI; snp = j0 + (x >> 1); pl = x & 1; }
        else { const int x = row - kRowsI - kRowsJ; snp = k0 + (x >> 1); pl = x & 1; }
        snp = snp < Mp ? snp : Mp - 1;  // rows past M read a zero row
        off[u] = (uint32_t)((cbase + (int64_t)snp * 2 + pl) * Sb + col);
      }
      v4i pf[kPer];
      auto fetch = [&](int ch) {
#pragma unroll
        for (int u = 0; u < kPer; ++u)
          if (tid + 256 * u < kChunks)
            pf[u] = *reinterpret_cast<gptr<v4i>>(gv + (off[u] + (uint32_t)ch * kPKC));
      };
      auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int c16 = tid + 256 * u;
          if (c16 < kChunks)
            *reinterpret_cast<v4i *>(stage + buf * kBuf + (c16 / kPieces) * kPRow + (c16 % kPieces) * 16) = pf[u];
        }
      };
      typename Acc::type acc[2][2][2];  // [i-block][j of the pair][B tile]
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[x][y][z][v] = 0;
      if (nch > 0) {
        fetch(0);
        store(0);
      }
      __syncthreads();
      const int o_xi = xi_off + 16 * g, o_xj = xj_off + 16 * g;
      const int o_b0 = (kRowsI + kRowsJ + 2 * (16 * (2 * wb) + ck16) + cpl) * kPRow + 16 * g;
      const int o_b1 = (kRowsI + kRowsJ + 2 * (16 * (2 * wb + 1) + ck16) + cpl) * kPRow + 16 * g;
#define EPI3_PLD(BB, STP, XI, XJ, B0, B1)                                           \
      XI = *reinterpret_cast<const v4i *>((BB) + o_xi + 32 * (STP));              \
      XJ = *reinterpret_cast<const v4i *>((BB) + o_xj + 32 * (STP));              \
      B0 = *reinterpret_cast<const v4i *>((BB) + o_b0 + 32 * (STP));              \
      B1 = *reinterpret_cast<const v4i *>((BB) + o_b1 + 32 * (STP));
#define EPI3_PSTEP(XI, XJ, B0, B1)                                                  \
      {                                                                           \
        const v4i xi_[2] = {quad_perm<0xA0>(XI), quad_perm<0xF5>(XI)};            \
        _Pragma("unroll") for (int x = 0; x < 2; ++x) {                           \
          const v4i a0 = xi_[x] & quad_perm<0x44>(XJ);                            \
          acc[x][0][0] = Acc::mma(a0, B0, acc[x][0][0]);                          \
          acc[x][0][1] = Acc::mma(a0, B1, acc[x][0][1]);                          \
          const v4i a1 = xi_[x] & quad_perm<0xEE>(XJ);                            \
          acc[x][1][0] = Acc::mma(a1, B0, acc[x][1][0]);                          \
          acc[x][1][1] = Acc::mma(a1, B1, acc[x][1][1]);                          \
        }                                                                         \
      }                                                                           \
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (kPKC == 128) {
        // software pipeline over the four steps of a chunk (operand sets X
        // and Y in turn; the next chunk is stored before the last step)
        v4i xiX, xjX, b0X, b1X, xiY, xjY, b0Y, b1Y;
        EPI3_PLD(stage, 0, xiX, xjX, b0X, b1X)
        for (int ch = 0; ch < nch; ++ch) {
          const bool more = ch + 1 < nch;
          if (more) fetch(ch + 1);
          const uint8_t *buf = stage + (ch & 1) * kBuf;
          const uint8_t *nbuf = stage + ((ch + 1) & 1) * kBuf;
          EPI3_PLD(buf, 1, xiY, xjY, b0Y, b1Y)
          EPI3_PSTEP(xiX, xjX, b0X, b1X)
          EPI3_PLD(buf, 2, xiX, xjX, b0X, b1X)
          EPI3_PSTEP(xiY, xjY, b0Y, b1Y)
          EPI3_PLD(buf, 3, xiY, xjY, b0Y, b1Y)
          EPI3_PSTEP(xiX, xjX, b0X, b1X)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) asm volatile("" : "+v"(acc[x][y][0]), "+v"(acc[x][y][1]));
          if (more) store((ch + 1) & 1);
          __syncthreads();
          // after the last chunk this reads the other buffer's stale
          // contents, which no product uses
          EPI3_PLD(nbuf, 0, xiX, xjX, b0X, b1X)
          EPI3_PSTEP(xiY, xjY, b0Y, b1Y)
        }
      } else {
        for (int ch = 0; ch < nch; ++ch) {
          if (ch + 1 < nch) fetch(ch + 1);
          const uint8_t *buf = stage + (ch & 1) * kBuf;
  #pragma unroll 1
          for (int stp = 0; stp < kPKC / 32; ++stp) {
            const int off = stp * 32 + 16 * g;
            // the quad (a, b) loads X_i[a] of i-block b and X_j[b] of pivot a;
            // DPP hands each lane the two rows its A rows need
            const v4i xiq = *reinterpret_cast<const v4i *>(buf + xi_off + off);
            const v4i xjq = *reinterpret_cast<const v4i *>(buf + xj_off + off);
            v4i b[2];
  #pragma unroll
            for (int x = 0; x < 2; ++x)
              b[x] = *reinterpret_cast<const v4i *>(
                  buf + (kRowsI + kRowsJ + 2 * (16 * (2 * wb + x) + ck16) + cpl) * kPRow + off);
            const v4i xi[2] = {quad_perm<0xA0>(xiq), quad_perm<0xF5>(xiq)};  // [0,0,2,2], [1,1,3,3]
  #pragma unroll
            for (int x = 0; x < 2; ++x) {
              const v4i a0 = xi[x] & quad_perm<0x44>(xjq);  // [0,1,0,1]: X_j[b] of pivot 0
              acc[x][0][0] = Acc::mma(a0, b[0], acc[x][0][0]);
              acc[x][0][1] = Acc::mma(a0, b[1], acc[x][0][1]);
              const v4i a1 = xi[x] & quad_perm<0xEE>(xjq);  // [2,3,2,3]: X_j[b] of pivot 1
              acc[x][1][0] = Acc::mma(a1, b[0], acc[x][1][0]);
              acc[x][1][1] = Acc::mma(a1, b[1], acc[x][1][1]);
            }
          }
          if (ch + 1 < nch) store((ch + 1) & 1);
          __syncthreads();
        }
      }
#undef EPI3_PLD
#undef EPI3_PSTEP
      // corners out: lane (column, g) holds rows 8 u + 4 g + w, i.e. pivot
      // i8 = 2 u + g with cells (a, b) = w, for its column (k16, plane).
      // Record (i, j, k) of class cls is 16 bytes: plane-0 cells then plane-1
      // cells, each 4 x uint16 in (a, b) order.
      uint2 *cor = reinterpret_cast<uint2 *>(corners) + ((slot * 2 + cls) * (int64_t)kPI * 256) * 2;
      // record (il, jl, kl) = (8 x + 2 u + g, 2 wj + y, 16 (2 wb + z) + ck16)
      // sits at a constant per (x, y, z, u) plus one lane offset; the offset
      // is made opaque here so the 32 addresses are formed at the stores
      // instead of being held in registers through the tile
      uint32_t lo = (uint32_t)(((g * JB + 2 * wj) * KT + 32 * wb + ck16) * 2 + cpl);
      asm volatile("" : "+v"(lo));
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int c_off = (((8 * x + 2 * u) * JB + y) * KT + 16 * z) * 2;
              const uint32_t c0 = Acc::get(acc[x][y][z], 4 * u + 0), c1 = Acc::get(acc[x][y][z], 4 * u + 1);
              const uint32_t c2 = Acc::get(acc[x][y][z], 4 * u + 2), c3 = Acc::get(acc[x][y][z], 4 * u + 3);
              (cor + c_off)[lo] = make_uint2(c0 | (c1 << 16), c2 | (c3 << 16));
            }
    }
  }
}

// Completes both tables of every triplet of a pass and scores it; workgroup
// per tile (persistent, round robin), thread per triplet of the tile.  Cells
// are carried as 4 x count (byte offsets into the FP32 log-factorial table,
// which sits at LDS address 0: the kernel declares no static LDS), so each
// of the 81 lookups per triplet needs at most one add.
// Lowest and highest key of the wave's lanes into keyrange[0..1].
__device__ __forceinline__ void flush_range(uint32_t kmin, uint32_t kmax, uint32_t *keyrange) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t a = __shfl_xor(kmin, off), b = __shfl_xor(kmax, off);
    kmin = a < kmin ? a : kmin;
    kmax = b > kmax ? b : kmax;
  }
  if ((threadIdx.x & 63) == 0 && kmax != 0u) {
    atomicMin(keyrange, kmin);
    atomicMax(keyrange + 1, kmax);
  }
}

template <int JB, bool LDS, bool COUNTS, int MODE>
__global__ void __launch_bounds__(256) finish_plain_kernel(const PlainJob *__restrict__ jobs,
                                                           const int64_t *__restrict__ job_begin_p,
                                                           int n_jobs,
                                                           const uint4 *__restrict__ corners,
                                                           int64_t tile_begin, int64_t n_tiles,
                                                           const float *__restrict__ lf32,
                                                           int lf_len, PlainOut out) {
  constexpr int KT = 256 / JB;
  constexpr int kTile = kPI * JB * KT;  // 4096 triplets
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  // after the table (its dynamic block starts at LDS address 0)
  int2(*smk)[KT] = reinterpret_cast<int2(*)[KT]>(lds + (LDS ? (lf_len * 4 + 15) / 16 * 16 : 0));
  if (LDS) {
    float *tab = reinterpret_cast<float *>(lds);
    for (int x = threadIdx.x; x < lf_len; x += blockDim.x) tab[x] = lf32[x];
  }
  __syncthreads();
  typedef int i4e __attribute__((ext_vector_type(4)));
  typedef unsigned u4e __attribute__((ext_vector_type(4)));
  cptr<int64_t> job_begin = as_const(job_begin_p);
  JobDecoder jd;
  int M = 0, Mp = 0, nJ = 0, N0x4 = 0, N1x4 = 0;
  uint32_t MpMp = 0;  // pair tables < 4 G entries
  cptr<int64_t> pre = nullptr;
  gptr<i4e> pr = nullptr;
  float *score = nullptr;
  uint32_t *counts = nullptr, *keyrange = nullptr;
  // key range of this thread's scores of the current job (flushed per job)
  uint32_t kmin = 0xffffffffu, kmax = 0u;
  TileDecoder dec;
  // bounded: this launch's append bound (set before the launch)
  const float ub = MODE == kPermOutBounded ? out.st->ub : 0.f;
  for (int64_t slot = blockIdx.x; slot < n_tiles; slot += gridDim.x) {
    const int64_t tg = tile_begin + slot * out.stride;
    if (jd.find(job_begin, n_jobs, tg)) {
      if (keyrange) flush_range(kmin, kmax, keyrange);
      kmin = 0xffffffffu;
      kmax = 0u;
      const PlainJob &pj = jobs[jd.x];
      M = pj.M;
      Mp = pj.Mp;
      nJ = (int)plain_jblocks(M, JB);
      N0x4 = pj.N0 << 2;
      N1x4 = pj.N1 << 2;
      MpMp = (uint32_t)Mp * (uint32_t)Mp;
      pre = as_const(pj.jprefix);
      pr = (gptr<i4e>)pj.pairs;
      score = pj.score;
      counts = pj.counts;
      keyrange = MODE == kPermOutSample ? out.range : pj.keyrange;
      dec.J = -1;
    }
    const int64_t t = tg - jd.lo;  // tile within its job
    dec.find(pre, nJ, t);
    int i0, j0, k0;
    plain_tile_origin(dec, t, M, JB, i0, j0, k0);
    gptr<u4e> cor = (gptr<u4e>)(corners + slot * 2 * (int64_t)kTile);
    // per-SNP counts (the pair tables' diagonals) of the tile's k range in
    // LDS, so each lane's k margin is one conflict-free LDS read instead of a
    // strided global load
    __syncthreads();  // previous tile's readers are done
    if (threadIdx.x < 2 * KT) {
      const int c = threadIdx.x / KT, kl = threadIdx.x % KT;
      const int k = k0 + kl < Mp ? k0 + kl : Mp - 1;
      const i4e v = pr[(uint32_t)c * MpMp + (uint32_t)k * Mp + k];
      smk[c][kl] = make_int2(v.x << 2, v.w << 2);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < kTile; x += blockDim.x) {
      const int il = x / (JB * KT), jl = (x / KT) % JB, kl = x % KT;
      const int i = i0 + il, j = j0 + jl, k = k0 + kl;
      if (i >= j || j >= k || k >= M) continue;
      int tab[2][27];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const u4e q = cor[c * kTile + x];
        // record order: [plane of k][a][b] -> corner index 4 a + 2 b + plane; x 4
        const uint32_t n[8] = {(q.x << 2) & 0x3fffcu, (q.z << 2) & 0x3fffcu,
                               (q.x >> 14) & 0x3fffcu, (q.z >> 14) & 0x3fffcu,
                               (q.y << 2) & 0x3fffcu, (q.w << 2) & 0x3fffcu,
                               (q.y >> 14) & 0x3fffcu, (q.w >> 14) & 0x3fffcu};
        const uint32_t cb = (uint32_t)c * MpMp;
        const i4e a4 = pr[cb + (uint32_t)i * Mp + j], b4 = pr[cb + (uint32_t)i * Mp + k];
        const i4e c4 = pr[cb + (uint32_t)j * Mp + k];
        const i4e ii = pr[cb + (uint32_t)i * Mp + i], jj = pr[cb + (uint32_t)j * Mp + j];
        const int2 kk2 = smk[c][kl];
        const int pij[4] = {a4.x << 2, a4.y << 2, a4.z << 2, a4.w << 2};
        const int pik[4] = {b4.x << 2, b4.y << 2, b4.z << 2, b4.w << 2};
        const int pjk[4] = {c4.x << 2, c4.y << 2, c4.z << 2, c4.w << 2};
        const int mi[2] = {ii.x << 2, ii.w << 2}, mj[2] = {jj.x << 2, jj.w << 2};
        const int mk[2] = {kk2.x, kk2.y};
        complete_table(n, pij, pik, pjk, mi, mj, mk, c ? N1x4 : N0x4, tab[c]);
      }
      float k2 = 0.f;  // rows in order, each L[r + 1] - (L[r_0] + L[r_1])
#pragma unroll
      for (int x2 = 0; x2 < 27; ++x2) {
        const int b0 = tab[0][x2], b1 = tab[1][x2];
        if (LDS)
          k2 += lf_at_lds0(b0 + b1 + 4) - (lf_at_lds0(b0) + lf_at_lds0(b1));
        else
          k2 += lf_at(lf32, b0 + b1 + 4) - (lf_at(lf32, b0) + lf_at(lf32, b1));
      }
      const int64_t rank = lex_base(M, i, j) + k;
      if (MODE == kPermOutPlane) score[rank] = k2;
      if (MODE == kPermOutSample) out.sample[(out.sample_base + slot) * kTile + x] = k2;
      if (MODE == kPermOutBounded && k2 <= ub) {
        // rare (a few thousand of the C(M,3) scores): one atomic per append
        const unsigned long long pos = atomicAdd(&out.st->cn, 1ull);
        if ((int64_t)pos < out.ccap) {
          out.ckey[pos] = f2key(k2);
          out.crank[pos] = rank;
        }
      }
      if (COUNTS) {
        uint32_t *o = counts + rank * 54;
        for (int x2 = 0; x2 < 27; ++x2) {
          o[x2] = (uint32_t)tab[0][x2] >> 2;
          o[27 + x2] = (uint32_t)tab[1][x2] >> 2;
        }
      }
      const uint32_t key = f2key(k2);
      kmin = key < kmin ? key : kmin;
      kmax = key > kmax ? key : kmax;
    }
  }
  if (keyrange) flush_range(kmin, kmax, keyrange);
}

__global__ void write_plainjob_kernel(PlainJob h, PlainJob *dst) { if (threadIdx.x == 0) *dst = h; }

}  // namespace

int64_t host_plain_tiles(int64_t M, int JB) {
  int64_t n = 0;
  const int64_t nJ = plain_jblocks(M, JB);
  for (int64_t J = 0; J < nJ; ++J) n += plain_tiles_of_jb(M, J, JB);
  return n;
}

hipError_t launch_write_plainjob(const PlainJob &h, PlainJob *dst_dev, hipStream_t s) {
  hipLaunchKernelGGL(write_plainjob_kernel, dim3(1), dim3(64), 0, s, h, dst_dev);
  return hipGetLastError();
}

hipError_t launch_plain_prefix(PlainJob *pj_dev, hipStream_t s) {
  hipLaunchKernelGGL(plain_prefix_kernel, dim3(1), dim3(1024), 0, s, pj_dev);
  return hipGetLastError();
}

static hipError_t cu_count(int *n_cu) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  return hipDeviceGetAttribute(n_cu, hipDeviceAttributeMultiprocessorCount, dev);
}

template <bool FP4, int JB>
static hipError_t launch_plain_count_t(const PlainJob *jobs, const int64_t *job_begin, int n_jobs,
                                       uint4 *corners, int64_t tile_begin, int64_t n,
                                       int64_t stride, unsigned long long *queue, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int n_cu = 0;
  hipError_t e = cu_count(&n_cu);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, count_mfma_plain_kernel<FP4, JB>, 256, 0);
  if (e != hipSuccess) return e;
  if (per_cu <= 0) per_cu = 1;
  int64_t blocks = (int64_t)n_cu * per_cu;
  if (blocks > n) blocks = n;
  hipLaunchKernelGGL((count_mfma_plain_kernel<FP4, JB>), dim3((unsigned)blocks), dim3(256), 0, s,
                     jobs, job_begin, n_jobs, corners, tile_begin, n, stride, queue);
  return hipGetLastError();
}

hipError_t launch_count_mfma_plain(const PlainJob *jobs, const int64_t *job_begin, int32_t n_jobs,
                                   int JB, bool fp4, uint4 *corners, int64_t tile_begin,
                                   int64_t n_tiles, int64_t stride, unsigned long long *queue,
                                   hipStream_t s) {
  if (stride < 1) return hipErrorInvalidValue;
  switch (JB) {
    case 2:
      return fp4 ? launch_plain_count_t<true, 2>(jobs, job_begin, n_jobs, corners, tile_begin, n_tiles, stride, queue, s)
                 : launch_plain_count_t<false, 2>(jobs, job_begin, n_jobs, corners, tile_begin, n_tiles, stride, queue, s);
    case 4:
      return fp4 ? launch_plain_count_t<true, 4>(jobs, job_begin, n_jobs, corners, tile_begin, n_tiles, stride, queue, s)
                 : launch_plain_count_t<false, 4>(jobs, job_begin, n_jobs, corners, tile_begin, n_tiles, stride, queue, s);
    case 8:
      return fp4 ? launch_plain_count_t<true, 8>(jobs, job_begin, n_jobs, corners, tile_begin, n_tiles, stride, queue, s)
                 : launch_plain_count_t<false, 8>(jobs, job_begin, n_jobs, corners, tile_begin, n_tiles, stride, queue, s);
  }
  return hipErrorInvalidValue;
}

template <int JB, bool LDS, bool COUNTS, int MODE>
static hipError_t launch_finish_plain_t(const PlainJob *jobs, const int64_t *job_begin, int n_jobs,
                                        const uint4 *corners, int64_t tile_begin, int64_t n,
                                        const float *lf32, int32_t lf_len, const PlainOut &out,
                                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int n_cu = 0;
  hipError_t e = cu_count(&n_cu);
  if (e != hipSuccess) return e;
  const size_t lds = (LDS ? (size_t)(lf_len * 4 + 15) / 16 * 16 : 0) +
                     2 * (256 / JB) * sizeof(int2);  // table, then the tile's k margins
  auto kern = finish_plain_kernel<JB, LDS, COUNTS, MODE>;
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds);
  if (e != hipSuccess) return e;
  if (per_cu <= 0) per_cu = 1;
  int64_t blocks = (int64_t)n_cu * per_cu;
  if (blocks > n) blocks = n;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), lds, s, jobs, job_begin, n_jobs,
                     corners, tile_begin, n, lf32, lf_len, out);
  return hipGetLastError();
}

template <int JB, bool LDS>
static hipError_t launch_finish_plain_l(const PlainJob *jobs, const int64_t *job_begin, int n_jobs,
                                        const uint4 *corners, int64_t tile_begin, int64_t n,
                                        const float *lf32, int32_t lf_len, bool counts,
                                        const PlainOut &out, hipStream_t s) {
  switch (out.mode) {
    case kPermOutPlane:
      return counts ? launch_finish_plain_t<JB, LDS, true, kPermOutPlane>(jobs, job_begin, n_jobs, corners, tile_begin, n, lf32, lf_len, out, s)
                    : launch_finish_plain_t<JB, LDS, false, kPermOutPlane>(jobs, job_begin, n_jobs, corners, tile_begin, n, lf32, lf_len, out, s);
    case kPermOutSample:
      return launch_finish_plain_t<JB, LDS, false, kPermOutSample>(jobs, job_begin, n_jobs, corners, tile_begin, n, lf32, lf_len, out, s);
    case kPermOutBounded:
      return launch_finish_plain_t<JB, LDS, false, kPermOutBounded>(jobs, job_begin, n_jobs, corners, tile_begin, n, lf32, lf_len, out, s);
  }
  return hipErrorInvalidValue;
}

template <int JB>
static hipError_t launch_finish_plain_j(const PlainJob *jobs, const int64_t *job_begin, int n_jobs,
                                        const uint4 *corners, int64_t tile_begin, int64_t n,
                                        const float *lf32, int32_t lf_len, bool counts,
                                        const PlainOut &out, hipStream_t s) {
  return lf_in_lds(lf_len)
             ? launch_finish_plain_l<JB, true>(jobs, job_begin, n_jobs, corners, tile_begin, n, lf32, lf_len, counts, out, s)
             : launch_finish_plain_l<JB, false>(jobs, job_begin, n_jobs, corners, tile_begin, n, lf32, lf_len, counts, out, s);
}

hipError_t launch_finish_plain(const PlainJob *jobs, const int64_t *job_begin, int32_t n_jobs,
                               int JB, const uint4 *corners, int64_t tile_begin, int64_t n_tiles,
                               const float *lf32, int32_t lf_len, bool counts, const PlainOut &out,
                               hipStream_t s) {
  if (out.stride < 1 || (counts && out.mode != kPermOutPlane)) return hipErrorInvalidValue;
  switch (JB) {
    case 2: return launch_finish_plain_j<2>(jobs, job_begin, n_jobs, corners, tile_begin, n_tiles, lf32, lf_len, counts, out, s);
    case 4: return launch_finish_plain_j<4>(jobs, job_begin, n_jobs, corners, tile_begin, n_tiles, lf32, lf_len, counts, out, s);
    case 8: return launch_finish_plain_j<8>(jobs, job_begin, n_jobs, corners, tile_begin, n_tiles, lf32, lf_len, counts, out, s);
  }
  return hipErrorInvalidValue;
}

int64_t host_plain_sample_valid(int64_t M, int JB, int64_t stride, int64_t *n_sample) {
  const int KT = 256 / JB;
  const int64_t nJ = plain_jblocks(M, JB);
  int64_t t0 = 0, valid = 0, ns = 0;
  for (int64_t J = 0; J < nJ; ++J) {
    const int64_t nt = plain_tiles_of_jb(M, J, JB);
    if (nt == 0) continue;
    const int64_t j0 = J * JB;
    const int64_t nkb = (M - 1 - j0 + KT - 1) / KT;
    // sampled tiles of this j-block: the multiples of stride in [t0, t0 + nt)
    for (int64_t t = (t0 + stride - 1) / stride * stride; t < t0 + nt; t += stride) {
      ++ns;
      const int64_t rr = t - t0, ib = rr / nkb, kb = rr % nkb;
      const int64_t i0 = ib * kPI, k0 = j0 + 1 + kb * KT;
      for (int64_t j = j0; j < j0 + JB && j < M; ++j) {
        const int64_t ni = std::max<int64_t>(0, std::min<int64_t>(i0 + kPI, j) - i0);
        const int64_t klo = std::max<int64_t>(k0, j + 1), khi = std::min<int64_t>(k0 + KT, M);
        valid += ni * std::max<int64_t>(0, khi - klo);
      }
    }
    t0 += nt;
  }
  if (n_sample) *n_sample = ns;
  return valid;
}

struct I64Pack {
  int64_t v[32];
};
__global__ void write_i64_kernel(I64Pack h, int n, int64_t *dst) {
  if ((int)threadIdx.x < n) dst[threadIdx.x] = h.v[threadIdx.x];
}

hipError_t launch_write_i64(const int64_t *h, int32_t n, int64_t *dst_dev, hipStream_t s) {
  for (int32_t base = 0; base < n; base += 32) {
    I64Pack pk{};
    const int m = n - base < 32 ? n - base : 32;
    for (int x = 0; x < m; ++x) pk.v[x] = h[base + x];
    hipLaunchKernelGGL(write_i64_kernel, dim3(1), dim3(64), 0, s, pk, m, dst_dev + base);
  }
  return hipGetLastError();
}

}  // namespace epi3
