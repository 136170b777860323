// Fourth-order scan with the counts on the matrix cores.
//
// Eq. 1 with I = 3^4 rows.  For one class, the 16 cells of quad (i, j, k, l)
// with all four genotypes in {0, 1} are entries of a 0/1 matrix product over
// the class's samples s:
//     C[(i, j, k, a, b, c), (l, d)] = sum_s (X_i[a] X_j[b] X_k[c])[s] X_l[d][s],
// rows = corner rows of the triplet (i, j, k), columns = the value planes of
// SNP l.  The vector-ALU quad kernel fills the same cells with AND + POPCNT
// per 32 samples (the paper's table filling, Alg. 2, with a fourth SNP); here
// they come from FP4 (E2M1) products with exact FP32 accumulation, the other
// 65 cells by inclusion-exclusion (quad_cells) from the sub-triplet corner
// table and the pairwise tables, and K2 with the expression and row order of
// the vector-ALU kernel, so both give the same FP32 score.
//
// Workgroup tile: pivot j, four pivots i (one per wave), 16 consecutive k and
// 32 consecutive l (blocks aligned to their size; combinations outside
// i < j < k < l < M are counted and dropped).  A wave's products: 4 row tiles
// (4 k x 8 corner rows each) x 2 column tiles (16 l x 2 planes each) per 64
// samples.  Per chunk of 128 bytes (256 samples) the 64 l rows, the 32 k rows
// and the 16 pair rows X_i[a] & X_j[b] are staged in LDS; the steps are
// software-pipelined as in the phenotype count kernel.
#include "epi3_internal.h"

namespace epi3 {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

constexpr int kQKB = 16;                             // k per tile
constexpr int kQLB = 32;                             // l per tile
constexpr int kQKC = 128;                            // bytes per staged chunk of a row
constexpr int kQRow = kQKC + 16;                     // padded LDS row
constexpr int kQRowsL = 2 * kQLB;                    // (l, d) rows: B operand
constexpr int kQRowsK = 2 * kQKB;                    // (k, c) rows
constexpr int kQRowsP = 16;                          // pair rows: 4 waves x (a, b)
constexpr int kQRows = kQRowsL + kQRowsK + kQRowsP;  // 112
constexpr int kQStage = kQRows * kQRow;              // one LDS buffer
static_assert(kQuadTileScratch == 2 * 4 * kQKB * 64 * 2 * 8,
              "scratch per tile: 2 classes x 4 waves x 16 k x 64 columns x 2 uint2");

// ---- tile order: pivots j; within j, (k-block, l-block) pairs, then i-blocks ----
__host__ __device__ __forceinline__ int q_kb_lo(int j) { return (j + 1) / kQKB; }
__host__ __device__ __forceinline__ int q_nkb(int M, int j) { return (M - 1) / kQKB - q_kb_lo(j) + 1; }
// first l-block of k-block kb: the block holding (smallest valid k) + 1
__host__ __device__ __forceinline__ int q_lb_lo(int j, int kb) {
  const int kmin = kb * kQKB > j + 1 ? kb * kQKB : j + 1;
  return (kmin + 1) / kQLB;
}
__host__ __device__ __forceinline__ int q_nlb(int M, int j, int kb) {
  const int kmin = kb * kQKB > j + 1 ? kb * kQKB : j + 1;
  if (kmin >= M - 1) return 0;  // no l above the block's smallest k
  return (M - 1) / kQLB - q_lb_lo(j, kb) + 1;
}
__host__ __device__ __forceinline__ int64_t q_pairs_of_j(int M, int j) {
  int64_t n = 0;
  const int nkb = q_nkb(M, j);
  for (int x = 0; x < nkb; ++x) n += q_nlb(M, j, q_kb_lo(j) + x);
  return n;
}
__host__ __device__ __forceinline__ int64_t q_tiles_of_j(int M, int j) {
  if (j < 1 || j > M - 3) return 0;
  return (int64_t)((j + 3) / 4) * q_pairs_of_j(M, j);
}
// (i-block, k-block, l-block) of tile rr of pivot j
__device__ __forceinline__ void q_decode(int M, int j, int64_t rr, int &ib, int &kb, int &lb) {
  const int nib = (j + 3) / 4;
  const int64_t u = rr / nib;
  ib = (int)(rr - u * nib);
  int64_t acc = 0;
  kb = q_kb_lo(j);
  for (;;) {
    const int n = q_nlb(M, j, kb);
    if (u < acc + n) break;
    acc += n;
    ++kb;
  }
  lb = q_lb_lo(j, kb) + (int)(u - acc);
}

__device__ __forceinline__ int64_t rfl64x(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// pre[j] = tiles before pivot j, pre[M] = all tiles (one block).
__global__ void __launch_bounds__(1024) quad_prefix_kernel(int M, int64_t *pre) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int chunk = (M + 1023) / 1024;
  const int a = t * chunk, b = a + chunk < M ? a + chunk : M;
  int64_t sum = 0;
  for (int j = a; j < b; ++j) sum += q_tiles_of_j(M, j);
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - sum;
  for (int j = a; j < b; ++j) {
    pre[j] = run;
    run += q_tiles_of_j(M, j);
  }
  if (t == 1023) pre[M] = part[1023];
}

__device__ __forceinline__ int q_pivot(cptr<int64_t> pre, int M, int64_t t) {
  int lo = 0, hi = M - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// x from quad lane TT in every lane of each quad (DPP quad_perm broadcast).
template <int TT>
__device__ __forceinline__ v4i qbcast(v4i x) {
  constexpr int sel = TT * 0x55;
  v4i y;
  y.x = __builtin_amdgcn_update_dpp(0, x.x, sel, 0xf, 0xf, true);
  y.y = __builtin_amdgcn_update_dpp(0, x.y, sel, 0xf, 0xf, true);
  y.z = __builtin_amdgcn_update_dpp(0, x.z, sel, 0xf, 0xf, true);
  y.w = __builtin_amdgcn_update_dpp(0, x.w, sel, 0xf, 0xf, true);
  return y;
}

__device__ __forceinline__ v16f qmma(v4i a, v4i b, v16f c) {
  const v8i a8 = {a.x, a.y, a.z, a.w, 0, 0, 0, 0};
  const v8i b8 = {b.x, b.y, b.z, b.w, 0, 0, 0, 0};
  // cbsz = blgp = 4: both operands FP4 (E2M1); scale exponents 127 = 2^0
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, c, 4, 4, 0, 127, 0, 127);
}

// Counts the 16 corner cells of both classes of every quad of tiles
// [tile_begin, tile_begin + n_tiles) into scratch slot t - tile_begin
// (persistent workgroups, atomic tile queue).  Fragment layout of
// v_mfma_scale_f32_32x32x64_f8f6f4: lane l supplies A row l % 32 and B column
// l % 32 with 32 consecutive samples (16 bytes) starting at 32 (l / 32); the
// result of row r, column c is in lane c + 32 ((r / 4) % 2), register
// 4 (r / 8) + r % 4.
__global__ void __launch_bounds__(256, 2) count_mfma_quad_kernel(
    const uint8_t *__restrict__ nib, const int64_t *__restrict__ pre_p, int M, int Mp, int Sb,
    int Sb0, int Sb1, int64_t tile_begin, int64_t n_tiles, uint2 *__restrict__ corners,
    unsigned long long *__restrict__ queue) {
  __shared__ __attribute__((aligned(16))) unsigned char stage[2 * kQStage];
  __shared__ int64_t sTile[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 31, g = lane >> 5;
  // A row r of a row tile = (triplet ta = r / 8, corner c = (r / 4) % 2,
  // a = (r / 2) % 2, b = r % 2); the four lanes of a quad share (ta, c), each
  // loads the k row of a different row tile and DPP broadcasts it
  const int ta = r >> 3, rc = (r >> 2) & 1, ra = (r >> 1) & 1, rb = r & 1;
  gptr<uint8_t> gv = (gptr<uint8_t>)nib;
  cptr<int64_t> pre = as_const(pre_p);
  const int prow = kQRowsL + kQRowsK + wave * 4 + (ra * 2 + rb);
  const int xrow = kQRowsL + (4 * (r & 3) + ta) * 2 + rc;
  const int o_p = prow * kQRow + 16 * g, o_x = xrow * kQRow + 16 * g;
  const int o_b0 = r * kQRow + 16 * g, o_b1 = (32 + r) * kQRow + 16 * g;
  int j = -1;
  int64_t jlo = 0, jhi = 0;
  for (;;) {
    __syncthreads();  // previous tile's readers of sTile / stage are done
    if (tid == 0) sTile[0] = (int64_t)atomicAdd(queue, 1ull);
    __syncthreads();
    const int64_t slot = rfl64x(sTile[0]);
    if (slot >= n_tiles) break;
    const int64_t t = tile_begin + slot;
    if (j < 0 || t < jlo || t >= jhi) {
      j = q_pivot(pre, M, t);
      jlo = pre[j];
      jhi = pre[j + 1];
    }
    int ib, kb, lb;
    q_decode(M, j, t - jlo, ib, kb, lb);
    const int i = 4 * ib + wave;  // may be >= j: then the wave's results are dropped
    const int kbase = kb * kQKB, lbase = lb * kQLB;
    for (int cls = 0; cls < 2; ++cls) {
      if (cls) __syncthreads();  // class 0's readers of stage are done
      const int nch = ((cls ? Sb1 : Sb0) + kQKC - 1) / kQKC;
      const int64_t crow = (int64_t)cls * Mp * 2;  // first row of the class
      // staging plan: rows [0, 64) (l, d), [64, 96) (k, c), [96, 112) pair
      // rows; main pieces c16 = tid + 256 u; threads tid < 128 also carry one
      // pair piece (both source words, ANDed when stored)
      constexpr int kPc = kQKC / 16;
      constexpr int kMainU = 96 * kPc / 256;
      constexpr int kPairPieces = kQRowsP * kPc;
      static_assert((96 * kPc) % 256 == 0 && kPairPieces <= 256, "staging plan");
      uint32_t off[kMainU], offa = 0, offb = 0;
#pragma unroll
      for (int u = 0; u < kMainU; ++u) {
        const int c16 = tid + 256 * u;
        const int row = c16 / kPc, col = (c16 % kPc) * 16;
        const int snp = row < kQRowsL ? lbase + (row >> 1) : kbase + ((row - kQRowsL) >> 1);
        off[u] = (uint32_t)((crow + (int64_t)snp * 2 + (row & 1)) * Sb + col);
      }
      if (tid < kPairPieces) {
        const int x = tid / kPc, col = (tid % kPc) * 16;  // pair row x: wave x >> 2, (a, b) = x & 3
        const int ii = 4 * ib + (x >> 2);
        offa = (uint32_t)((crow + (int64_t)ii * 2 + ((x >> 1) & 1)) * Sb + col);
        offb = (uint32_t)((crow + (int64_t)j * 2 + (x & 1)) * Sb + col);
      }
      v4i pf[kMainU], pa, pb;
      auto fetch = [&](int ch) {
        const uint32_t c0 = (uint32_t)ch * kQKC;
#pragma unroll
        for (int u = 0; u < kMainU; ++u) pf[u] = *reinterpret_cast<gptr<v4i>>(gv + (off[u] + c0));
        if (tid < kPairPieces) {
          pa = *reinterpret_cast<gptr<v4i>>(gv + (offa + c0));
          pb = *reinterpret_cast<gptr<v4i>>(gv + (offb + c0));
        }
      };
      auto store = [&](int buf) {
        uint8_t *dst = stage + buf * kQStage;
#pragma unroll
        for (int u = 0; u < kMainU; ++u) {
          const int c16 = tid + 256 * u;
          *reinterpret_cast<v4i *>(dst + (c16 / kPc) * kQRow + (c16 % kPc) * 16) = pf[u];
        }
        if (tid < kPairPieces)
          *reinterpret_cast<v4i *>(dst + (kQRowsL + kQRowsK + tid / kPc) * kQRow + (tid % kPc) * 16) = pa & pb;
      };
      v16f acc[4][2];
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[tt][0][v] = acc[tt][1][v] = 0.f;
      fetch(0);
      store(0);
      __syncthreads();
      // Software pipeline over the four steps of a chunk (operand sets X and
      // Y in turn; the next chunk is stored before the chunk's last step)
#define EPI3_QLD(BB, STP, P, X, B0, B1)                                               \
      P = *reinterpret_cast<const v4i *>((BB) + o_p + 32 * (STP));                  \
      X = *reinterpret_cast<const v4i *>((BB) + o_x + 32 * (STP));                  \
      B0 = *reinterpret_cast<const v4i *>((BB) + o_b0 + 32 * (STP));                \
      B1 = *reinterpret_cast<const v4i *>((BB) + o_b1 + 32 * (STP));
#define EPI3_QTILE(TT, P, X, B0, B1)                                                  \
      {                                                                             \
        const v4i a_ = (P) & qbcast<TT>(X);                                         \
        acc[TT][0] = qmma(a_, B0, acc[TT][0]);                                      \
        acc[TT][1] = qmma(a_, B1, acc[TT][1]);                                      \
      }
// a scheduling barrier between steps; the compiler interleaves each row
// tile's A-row ANDs with the products itself
#define EPI3_QSCHED __builtin_amdgcn_sched_barrier(0);
#define EPI3_QSTEP(P, X, B0, B1)                                                      \
      EPI3_QTILE(0, P, X, B0, B1)                                                   \
      EPI3_QTILE(1, P, X, B0, B1)                                                   \
      EPI3_QTILE(2, P, X, B0, B1)                                                   \
      EPI3_QTILE(3, P, X, B0, B1)
      static_assert(kQKC / 32 == 4, "four steps per chunk");
      v4i pX, xX, b0X, b1X, pY, xY, b0Y, b1Y;
      EPI3_QLD(stage, 0, pX, xX, b0X, b1X)
      for (int ch = 0; ch < nch; ++ch) {
        const bool more = ch + 1 < nch;
        if (more) fetch(ch + 1);
        const uint8_t *buf = stage + (ch & 1) * kQStage;
        const uint8_t *nbuf = stage + ((ch + 1) & 1) * kQStage;
        EPI3_QLD(buf, 1, pY, xY, b0Y, b1Y)
        EPI3_QSTEP(pX, xX, b0X, b1X)
        EPI3_QSCHED
        EPI3_QLD(buf, 2, pX, xX, b0X, b1X)
        EPI3_QSTEP(pY, xY, b0Y, b1Y)
        EPI3_QSCHED
        EPI3_QLD(buf, 3, pY, xY, b0Y, b1Y)
        EPI3_QSTEP(pX, xX, b0X, b1X)
        EPI3_QSCHED
        // the products above stay before the branch
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) asm volatile("" : "+v"(acc[tt][0]), "+v"(acc[tt][1]));
        if (more) store((ch + 1) & 1);
        __syncthreads();
        // after the last chunk this reads the other buffer's stale contents,
        // which no product uses
        EPI3_QLD(nbuf, 0, pX, xX, b0X, b1X)
        EPI3_QSTEP(pY, xY, b0Y, b1Y)
        EPI3_QSCHED
      }
#undef EPI3_QLD
#undef EPI3_QTILE
#undef EPI3_QSCHED
#undef EPI3_QSTEP
      if (i >= j) continue;  // padding pivot of the last i-block (wave-uniform)
      // lane (column, c) holds, for the 4 triplets of each row tile, the cells
      // (a, b) at genotype c of SNP k: registers 4 ta + 2 a + b.  Record of
      // (triplet, column) = 2 x uint2 (c = 0, 1), columns 2 l + d adjacent.
      uint2 *cor = corners + ((slot * 2 + cls) * 4 + wave) * (int64_t)(kQKB * 128);
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int t4 = 0; t4 < 4; ++t4) {
            const uint32_t c0 = (uint32_t)acc[tt][cb][4 * t4 + 0], c1 = (uint32_t)acc[tt][cb][4 * t4 + 1];
            const uint32_t c2 = (uint32_t)acc[tt][cb][4 * t4 + 2], c3 = (uint32_t)acc[tt][cb][4 * t4 + 3];
            cor[((4 * tt + t4) * 64 + cb * 32 + r) * 2 + g] = make_uint2(c0 | (c1 << 16), c2 | (c3 << 16));
          }
    }
  }
}

// the 8 corner cells of a triplet-table entry, each x 4
__device__ __forceinline__ void unpack8q(uint4 v, uint32_t *n) {
  n[0] = (v.x & 0xffffu) << 2; n[1] = (v.x >> 16) << 2; n[2] = (v.y & 0xffffu) << 2; n[3] = (v.y >> 16) << 2;
  n[4] = (v.z & 0xffffu) << 2; n[5] = (v.z >> 16) << 2; n[6] = (v.w & 0xffffu) << 2; n[7] = (v.w >> 16) << 2;
}

// Completes both 81-row tables of every quad of the pass's tiles and scores
// them (workgroup per tile, round robin; thread per quad, consecutive l).
template <bool LDS>
__global__ void __launch_bounds__(256) finish_quad_kernel(
    const uint2 *__restrict__ corners, const int64_t *__restrict__ pre_p,
    const uint4 *__restrict__ t3, const int32_t *__restrict__ pairs, int M, int Mp, int N0,
    int N1, int64_t T, int64_t tile_begin, int64_t n_tiles, const float *__restrict__ lf32,
    int lf_len, float *__restrict__ score, uint32_t *__restrict__ keyrange) {
  // the LDS table starts the kernel's dynamic LDS block, at LDS address 0
  // (no static LDS), so a lookup is one ds_read at the byte offset; the
  // per-SNP counts of the tile's l range follow it
  extern __shared__ float qtab[];
  const float *L = lf32;
  if (LDS) {
    for (int x = threadIdx.x; x < lf_len; x += blockDim.x) qtab[x] = lf32[x];
  }
  int2(*sml)[kQLB] = reinterpret_cast<int2(*)[kQLB]>(
      reinterpret_cast<unsigned char *>(qtab) + (LDS ? (lf_len * 4 + 15) / 16 * 16 : 0));
  cptr<int64_t> pre = as_const(pre_p);
  const int64_t MpMp4 = (int64_t)Mp * Mp * 4;
  uint32_t kmin = 0xffffffffu, kmax = 0u;
  int j = -1;
  int64_t jlo = 0, jhi = 0;
  for (int64_t slot = blockIdx.x; slot < n_tiles; slot += gridDim.x) {
    const int64_t t = tile_begin + slot;
    if (j < 0 || t < jlo || t >= jhi) {
      j = q_pivot(pre, M, t);
      jlo = pre[j];
      jhi = pre[j + 1];
    }
    int ib, kb, lb;
    q_decode(M, j, t - jlo, ib, kb, lb);
    // per-SNP counts of the tile's 32 l (pair-table diagonals) into LDS: one
    // conflict-free LDS read per lane instead of a strided global load
    __syncthreads();  // previous tile's readers are done (and the table is in)
    if (threadIdx.x < 2 * kQLB) {
      const int c = threadIdx.x / kQLB, ll = threadIdx.x % kQLB;
      const int l = lb * kQLB + ll < Mp ? lb * kQLB + ll : Mp - 1;
      const int4 v = reinterpret_cast<const int4 *>(pairs + c * MpMp4)[(int64_t)l * Mp + l];
      sml[c][ll] = make_int2(v.x << 2, v.w << 2);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < 4 * kQKB * kQLB; x += blockDim.x) {
      const int ll = x & (kQLB - 1), kk = (x / kQLB) & (kQKB - 1), w = x / (kQLB * kQKB);
      const int i = 4 * ib + w, k = kb * kQKB + kk, l = lb * kQLB + ll;
      if (i >= j || k <= j || l <= k || l >= M) continue;
      int tc[2][81];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const uint4 *rec = reinterpret_cast<const uint4 *>(
            corners + (((slot * 2 + c) * 4 + w) * kQKB + kk) * 128 + ll * 4);
        const uint4 v[2] = {rec[0], rec[1]};  // columns (l, d = 0) and (l, d = 1)
        uint32_t cnt[48];
        // uint2 (d, c') = (cells (0, 0) | (0, 1) << 16, (1, 0) | (1, 1) << 16) over (a, b)
#pragma unroll
        for (int d = 0; d < 2; ++d)
#pragma unroll
          for (int cc = 0; cc < 2; ++cc)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
              const uint32_t wd = a ? (cc ? v[d].w : v[d].y) : (cc ? v[d].z : v[d].x);
              cnt[8 * a + 2 * cc + d] = (wd & 0xffffu) << 2;
              cnt[8 * a + 4 + 2 * cc + d] = (wd >> 16) << 2;
            }
        const uint4 *tcl = t3 + c * T;
        unpack8q(tcl[lex_base(M, i, j) + k], cnt + 16);
        unpack8q(tcl[lex_base(M, i, j) + l], cnt + 24);
        unpack8q(tcl[lex_base(M, i, k) + l], cnt + 32);
        unpack8q(tcl[lex_base(M, j, k) + l], cnt + 40);
        // cells as byte offsets into the FP32 table (x 4)
        const int2 mlv = sml[c][ll];
        const int ml[2] = {mlv.x, mlv.y};
        quad_cells<2>(cnt, pairs + c * MpMp4, Mp, i, j, k, l, (c ? N1 : N0) << 2, tc[c], ml);
      }
      float k2 = 0.f;  // rows in order: L[r + 1] - (L[r_0] + L[r_1])
#pragma unroll
      for (int y = 0; y < 81; ++y) {
        const int b0 = tc[0][y], b1 = tc[1][y];
        if (LDS)
          k2 += lf_at_lds0(b0 + b1 + 4) - (lf_at_lds0(b0) + lf_at_lds0(b1));
        else
          k2 += lf_at(L, b0 + b1 + 4) - (lf_at(L, b0) + lf_at(L, b1));
      }
      score[quad_rank(M, i, j, k, l)] = k2;
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
hipError_t launch_finish_quad_t(const epi3_dataset &d, const uint2 *corners, const int64_t *pre,
                                const uint4 *t3, int64_t tile_begin, int64_t n_tiles,
                                float *score, uint32_t *keyrange, int n_cu, hipStream_t s) {
  const int lf_len = d.n_samples + 2;
  const int lds = (LDS ? (lf_len * 4 + 15) / 16 * 16 : 0) + 2 * kQLB * (int)sizeof(int2);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&finish_quad_kernel<LDS>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, finish_quad_kernel<LDS>, 256, lds);
  if (e != hipSuccess) return e;
  int64_t blocks = (int64_t)n_cu * (per_cu > 0 ? per_cu : 1);
  if (blocks > n_tiles) blocks = n_tiles;
  hipLaunchKernelGGL(finish_quad_kernel<LDS>, dim3((unsigned)blocks), dim3(256), lds, s, corners,
                     pre, t3, d.pairs, d.n_snps, d.snp_stride, d.n_controls, d.n_cases,
                     c3(d.n_snps), tile_begin, n_tiles, d.lf32, lf_len, score, keyrange);
  return hipGetLastError();
}

}  // namespace

int64_t host_quad_tiles(int32_t M) {
  int64_t n = 0;
  for (int j = 0; j < M; ++j) n += q_tiles_of_j(M, j);
  return n;
}

hipError_t launch_quad_prefix(int32_t M, int64_t *jprefix, hipStream_t s) {
  hipLaunchKernelGGL(quad_prefix_kernel, dim3(1), dim3(1024), 0, s, (int)M, jprefix);
  return hipGetLastError();
}

hipError_t launch_count_mfma_quad(const epi3_dataset &d, const int64_t *jprefix,
                                  unsigned long long *queue, int64_t tile_begin, int64_t n_tiles,
                                  void *scratch, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, count_mfma_quad_kernel, 256, 0);
  if (e != hipSuccess) return e;
  if (per_cu <= 0) per_cu = 1;
  int64_t blocks = (int64_t)n_cu * per_cu;
  if (blocks > n_tiles) blocks = n_tiles;
  const int Sb = d.byte_stride / 2;                 // FP4 bytes per row
  const int Sb0 = (d.n_controls + 127) / 128 * 64;  // bytes holding each class
  const int Sb1 = (d.n_cases + 127) / 128 * 64;
  hipLaunchKernelGGL(count_mfma_quad_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<const uint8_t *>(d.nibbles), jprefix, d.n_snps, d.snp_stride, Sb,
                     Sb0, Sb1, tile_begin, n_tiles, static_cast<uint2 *>(scratch), queue);
  return hipGetLastError();
}

hipError_t launch_finish_quad(const epi3_dataset &d, const void *scratch, const int64_t *jprefix,
                              const void *t3, int64_t tile_begin, int64_t n_tiles, float *score,
                              uint32_t *keyrange, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const uint2 *cor = static_cast<const uint2 *>(scratch);
  const uint4 *t = static_cast<const uint4 *>(t3);
  return lf_in_lds(d.n_samples + 2)
             ? launch_finish_quad_t<true>(d, cor, jprefix, t, tile_begin, n_tiles, score, keyrange, n_cu, s)
             : launch_finish_quad_t<false>(d, cor, jprefix, t, tile_begin, n_tiles, score, keyrange, n_cu, s);
}

}  // namespace epi3
