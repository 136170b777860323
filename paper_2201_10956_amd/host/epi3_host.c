/*
 * Host-CPU three-way scan (libepi3_host.so): the paper's fourth CPU approach
 * (CPU approaches section, Alg. 1 and the vectorization paragraph) on this
 * machine's cores, kept as a measured baseline beside the GPU library.
 *
 * Data layout.  Samples are split by class (the second CPU approach), each
 * class packed into 64-bit words per SNP and genotype (plane 0: genotype 0,
 * plane 1: genotype 1; genotype 2 is never stored), rows padded with zero
 * words to a multiple of 8 words so every vector load is whole:
 *     planes[c] = [snp][plane][Wp_c] uint64.
 * Cache blocking.  For one (i, j) the 4 pair planes X_i[a] & X_j[b] of both
 * classes (at most 16 KiB per class at 65536 samples of a class) stay in the
 * first-level cache while the k loop streams each k's two planes once; the
 * paper sizes its blocks the same way, from the L1 capacity.
 * Counting.  n(a,b,c), a,b,c in {0,1}: popcount(X_i[a] & X_j[b] & X_k[c])
 * summed over the words; the other 19 cells follow from the pair counts
 * n_xy(a,b), the single-SNP counts n_x(a) and the class size (a value 2 on
 * one axis = all - value 0 - value 1 on that axis).
 * Threads.  OpenMP over i with a dynamic schedule, per-thread top-k buffers,
 * one merge at the end.
 */
#include "epi3_host.h"

#include <immintrin.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CELLS 27
#define WALIGN 8 /* words per padded row: one 512-bit vector */

typedef void (*corner_fn)(const uint64_t *A, const uint64_t *K, int64_t Wp, uint32_t out[8]);

/* ---------------------------------------------------- counting loops ---- */
/* A = 4 rows of Wp words (pair planes, row 2a + b), K = 2 rows (planes of k).
 * out[4a + 2b + c] = sum_w popcount(A[2a + b][w] & K[c][w]). */

static void corners_scalar(const uint64_t *A, const uint64_t *K, int64_t Wp, uint32_t out[8])
{
    uint64_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t w = 0; w < Wp; ++w) {
        const uint64_t k0 = K[w], k1 = K[Wp + w];
        for (int ab = 0; ab < 4; ++ab) {
            const uint64_t x = A[ab * Wp + w];
            acc[2 * ab] += (uint64_t)__builtin_popcountll(x & k0);
            acc[2 * ab + 1] += (uint64_t)__builtin_popcountll(x & k1);
        }
    }
    for (int q = 0; q < 8; ++q) out[q] = (uint32_t)acc[q];
}

__attribute__((target("avx2"))) static inline __m256i popcnt_bytes256(__m256i v)
{
    /* per-byte popcount from two 4-bit table lookups */
    const __m256i table = _mm256_setr_epi8(0, 1, 1, 2, 1, 2, 2, 3, 1, 2, 2, 3, 2, 3, 3, 4,
                                           0, 1, 1, 2, 1, 2, 2, 3, 1, 2, 2, 3, 2, 3, 3, 4);
    const __m256i low = _mm256_set1_epi8(0x0f);
    const __m256i lo = _mm256_and_si256(v, low);
    const __m256i hi = _mm256_and_si256(_mm256_srli_epi16(v, 4), low);
    return _mm256_add_epi8(_mm256_shuffle_epi8(table, lo), _mm256_shuffle_epi8(table, hi));
}

__attribute__((target("avx2"))) static void corners_avx2(const uint64_t *A, const uint64_t *K,
                                                         int64_t Wp, uint32_t out[8])
{
    __m256i acc[8];
    for (int q = 0; q < 8; ++q) acc[q] = _mm256_setzero_si256();
    const __m256i zero = _mm256_setzero_si256();
    for (int64_t w = 0; w < Wp; w += 4) {
        const __m256i k0 = _mm256_load_si256((const __m256i *)(K + w));
        const __m256i k1 = _mm256_load_si256((const __m256i *)(K + Wp + w));
        for (int ab = 0; ab < 4; ++ab) {
            const __m256i x = _mm256_load_si256((const __m256i *)(A + ab * Wp + w));
            /* byte counts of both products summed (<= 16 per byte), then
             * widened to 64-bit lanes by a sum of absolute differences */
            acc[2 * ab] = _mm256_add_epi64(
                acc[2 * ab], _mm256_sad_epu8(popcnt_bytes256(_mm256_and_si256(x, k0)), zero));
            acc[2 * ab + 1] = _mm256_add_epi64(
                acc[2 * ab + 1], _mm256_sad_epu8(popcnt_bytes256(_mm256_and_si256(x, k1)), zero));
        }
    }
    for (int q = 0; q < 8; ++q) {
        const __m128i s = _mm_add_epi64(_mm256_castsi256_si128(acc[q]),
                                        _mm256_extracti128_si256(acc[q], 1));
        out[q] = (uint32_t)(_mm_cvtsi128_si64(s) + _mm_extract_epi64(s, 1));
    }
}

__attribute__((target("avx512f,avx512vpopcntdq"))) static void corners_avx512(
    const uint64_t *A, const uint64_t *K, int64_t Wp, uint32_t out[8])
{
    __m512i acc[8];
    for (int q = 0; q < 8; ++q) acc[q] = _mm512_setzero_si512();
    for (int64_t w = 0; w < Wp; w += 8) {
        const __m512i k0 = _mm512_load_si512((const void *)(K + w));
        const __m512i k1 = _mm512_load_si512((const void *)(K + Wp + w));
        for (int ab = 0; ab < 4; ++ab) {
            const __m512i x = _mm512_load_si512((const void *)(A + ab * Wp + w));
            acc[2 * ab] = _mm512_add_epi64(acc[2 * ab], _mm512_popcnt_epi64(_mm512_and_si512(x, k0)));
            acc[2 * ab + 1] =
                _mm512_add_epi64(acc[2 * ab + 1], _mm512_popcnt_epi64(_mm512_and_si512(x, k1)));
        }
    }
    for (int q = 0; q < 8; ++q) out[q] = (uint32_t)_mm512_reduce_add_epi64(acc[q]);
}

int epi3h_best_isa(void)
{
    __builtin_cpu_init();
    if (__builtin_cpu_supports("avx512f") && __builtin_cpu_supports("avx512vpopcntdq"))
        return EPI3H_ISA_AVX512;
    if (__builtin_cpu_supports("avx2")) return EPI3H_ISA_AVX2;
    return EPI3H_ISA_SCALAR;
}

/* ------------------------------------------------------- encoding ---- */

typedef struct {
    int32_t M, N, n[2];   /* class sizes: n[0] controls, n[1] cases */
    int64_t Wp[2];        /* padded words per plane row */
    uint64_t *planes[2];  /* [M][2][Wp[c]] */
    uint32_t *pair[2];    /* [M][M][4]: n_xy(a, b) at 2a + b, x < y filled */
    uint32_t *single[2];  /* [M][2]: n_x(a) */
    double *L;            /* L[0..N+1] */
} dataset_t;

static void *alloc64(size_t bytes)
{
    void *p = NULL;
    if (posix_memalign(&p, 64, bytes ? bytes : 64) != 0) return NULL;
    return p;
}

static void free_dataset(dataset_t *d)
{
    for (int c = 0; c < 2; ++c) {
        free(d->planes[c]);
        free(d->pair[c]);
        free(d->single[c]);
    }
    free(d->L);
}

static uint32_t popcount_rows(const uint64_t *x, const uint64_t *y, int64_t W)
{
    uint64_t s = 0;
    for (int64_t w = 0; w < W; ++w) s += (uint64_t)__builtin_popcountll(x[w] & y[w]);
    return (uint32_t)s;
}

static int build_dataset(const uint8_t *geno, int64_t ld, const uint8_t *pheno, int32_t M,
                         int32_t N, int nt, dataset_t *d)
{
    memset(d, 0, sizeof(*d));
    d->M = M;
    d->N = N;
    for (int32_t s = 0; s < N; ++s) {
        if (pheno[s] > 1) return EPI3H_E_PHENOTYPE;
        d->n[pheno[s]]++;
    }
    int bad = 0;
#pragma omp parallel for num_threads(nt) reduction(| : bad) schedule(static)
    for (int32_t m = 0; m < M; ++m)
        for (int32_t s = 0; s < N; ++s) bad |= geno[(int64_t)m * ld + s] > 2;
    if (bad) return EPI3H_E_GENOTYPE;
    /* Eq. 1's inner sums: L[n] = sum_{b=1}^{n} log b, increasing b */
    d->L = (double *)malloc(sizeof(double) * ((size_t)N + 2));
    if (!d->L) return EPI3H_E_NOMEM;
    d->L[0] = 0.0;
    for (int32_t n = 1; n <= N + 1; ++n) d->L[n] = d->L[n - 1] + log((double)n);
    /* sample -> (class, position in class), original order kept */
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!pos) return EPI3H_E_NOMEM;
    int32_t fill[2] = {0, 0};
    for (int32_t s = 0; s < N; ++s) pos[s] = fill[pheno[s]]++;
    for (int c = 0; c < 2; ++c) {
        const int64_t W = ((int64_t)d->n[c] + 63) / 64;
        d->Wp[c] = (W + WALIGN - 1) / WALIGN * WALIGN;
        d->planes[c] = (uint64_t *)alloc64(sizeof(uint64_t) * (size_t)M * 2 * (size_t)d->Wp[c]);
        d->pair[c] = (uint32_t *)calloc((size_t)M * (size_t)M * 4 + 1, sizeof(uint32_t));
        d->single[c] = (uint32_t *)calloc((size_t)M * 2 + 1, sizeof(uint32_t));
        if (!d->planes[c] || !d->pair[c] || !d->single[c]) {
            free(pos);
            return EPI3H_E_NOMEM;
        }
        memset(d->planes[c], 0, sizeof(uint64_t) * (size_t)M * 2 * (size_t)d->Wp[c]);
    }
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int32_t m = 0; m < M; ++m) {
        const uint8_t *g = geno + (int64_t)m * ld;
        for (int32_t s = 0; s < N; ++s) {
            const int c = pheno[s];
            if (g[s] == 2) continue;
            const int64_t Wp = d->Wp[c];
            uint64_t *row = d->planes[c] + ((int64_t)m * 2 + g[s]) * Wp;
            row[pos[s] >> 6] |= 1ull << (pos[s] & 63);
        }
    }
    free(pos);
    /* single-SNP and pair counts of genotypes 0/1 per class */
    for (int c = 0; c < 2; ++c) {
        const int64_t Wp = d->Wp[c];
        const uint64_t *P = d->planes[c];
        for (int32_t m = 0; m < M; ++m)
            for (int a = 0; a < 2; ++a) {
                const uint64_t *r = P + ((int64_t)m * 2 + a) * Wp;
                d->single[c][m * 2 + a] = popcount_rows(r, r, Wp);
            }
#pragma omp parallel for num_threads(nt) schedule(dynamic, 4)
        for (int32_t x = 0; x < M; ++x)
            for (int32_t y = x + 1; y < M; ++y)
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        d->pair[c][((int64_t)x * M + y) * 4 + 2 * a + b] =
                            popcount_rows(P + ((int64_t)x * 2 + a) * Wp, P + ((int64_t)y * 2 + b) * Wp, Wp);
    }
    return EPI3H_OK;
}

/* ------------------------------------------------ table and score ---- */

/* Full 27-cell table of class c for (i, j, k) from its 8 corner cells.
 * m[x][y][z] with index 2 first meaning "any genotype" on that axis; each
 * axis is then turned into genotype 2 = any - 0 - 1. */
static void complete(const dataset_t *d, int c, int32_t i, int32_t j, int32_t k,
                     const uint32_t corner[8], int32_t t[CELLS])
{
    const int32_t M = d->M;
    const uint32_t *pij = d->pair[c] + ((int64_t)i * M + j) * 4;
    const uint32_t *pik = d->pair[c] + ((int64_t)i * M + k) * 4;
    const uint32_t *pjk = d->pair[c] + ((int64_t)j * M + k) * 4;
    const uint32_t *si = d->single[c] + 2 * i, *sj = d->single[c] + 2 * j, *sk = d->single[c] + 2 * k;
    int32_t m[3][3][3];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            for (int e = 0; e < 2; ++e) m[a][b][e] = (int32_t)corner[4 * a + 2 * b + e];
            m[a][b][2] = (int32_t)pij[2 * a + b];
            m[a][2][b] = (int32_t)pik[2 * a + b];
            m[2][a][b] = (int32_t)pjk[2 * a + b];
        }
    for (int a = 0; a < 2; ++a) {
        m[a][2][2] = (int32_t)si[a];
        m[2][a][2] = (int32_t)sj[a];
        m[2][2][a] = (int32_t)sk[a];
    }
    m[2][2][2] = d->n[c];
    for (int y = 0; y < 3; ++y)
        for (int z = 0; z < 3; ++z) m[2][y][z] -= m[0][y][z] + m[1][y][z];
    for (int x = 0; x < 3; ++x)
        for (int z = 0; z < 3; ++z) m[x][2][z] -= m[x][0][z] + m[x][1][z];
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) m[x][y][2] -= m[x][y][0] + m[x][y][1];
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y)
            for (int z = 0; z < 3; ++z) t[9 * x + 3 * y + z] = m[x][y][z];
}

/* Eq. 1 of up to KB triplets, each summed over its rows in increasing index,
 * each row L[r + 1] - (L[r_0] + L[r_1]); the triplets' sums are independent
 * chains, interleaved so the adds overlap. */
#define KB 8
static void k2_fp64_block(const int32_t t0[KB][CELLS], const int32_t t1[KB][CELLS], int nk,
                          const double *L, double out[KB])
{
    double s[KB];
    for (int b = 0; b < KB; ++b) s[b] = 0.0;
    for (int r = 0; r < CELLS; ++r)
        for (int b = 0; b < KB; ++b) {
            const int32_t x = b < nk ? t0[b][r] : 0, y = b < nk ? t1[b][r] : 0;
            s[b] += L[x + y + 1] - (L[x] + L[y]);
        }
    for (int b = 0; b < nk; ++b) out[b] = s[b];
}

/* ------------------------------------------------------------ top-k ---- */

typedef struct {
    double k2;
    int32_t i, j, k;
} cand_t;

static int before(const cand_t *a, const cand_t *b)
{
    if (a->k2 < b->k2) return 1;
    if (a->k2 > b->k2) return 0;
    if (a->i != b->i) return a->i < b->i;
    if (a->j != b->j) return a->j < b->j;
    return a->k < b->k;
}

static int cand_order(const void *x, const void *y)
{
    const cand_t *a = (const cand_t *)x, *b = (const cand_t *)y;
    return before(a, b) ? -1 : before(b, a) ? 1 : 0;
}

/* Keeps the best `keep` candidates: appends into a buffer of 2 keep entries
 * and, when it fills, sorts it and cuts it back to `keep`; once cut, the
 * last kept entry is the admission bound. */
typedef struct {
    cand_t *buf;
    int64_t n, keep;
    int full;
    cand_t bound;
} topk_t;

static void topk_cut(topk_t *T)
{
    qsort(T->buf, (size_t)T->n, sizeof(cand_t), cand_order);
    if (T->n > T->keep) T->n = T->keep;
    if (T->n == T->keep) {
        T->full = 1;
        T->bound = T->buf[T->n - 1];
    }
}

static inline void topk_offer(topk_t *T, const cand_t *c)
{
    if (T->full && !before(c, &T->bound)) return;
    T->buf[T->n++] = *c;
    if (T->n == 2 * T->keep) topk_cut(T);
}

/* ------------------------------------------------------------- scan ---- */

int epi3h_scan_topk(const uint8_t *geno, int64_t ld, const uint8_t *pheno, int32_t M,
                    int32_t N, int32_t k, int32_t threads, int32_t isa, epi3h_hit *out,
                    int32_t *n_out)
{
    if (!geno || !pheno || !out || !n_out || M < 0 || N <= 0 || ld < N || k <= 0)
        return EPI3H_E_INVALID;
    if (isa < EPI3H_ISA_BEST || isa > EPI3H_ISA_AVX512) return EPI3H_E_INVALID;
    const int best = epi3h_best_isa();
    if (isa == EPI3H_ISA_BEST) isa = best;
    if (isa > best) return EPI3H_E_UNSUPPORTED;
    *n_out = 0;
    int nt = threads;
#ifdef _OPENMP
    if (nt <= 0) nt = omp_get_max_threads();
#else
    nt = 1;
#endif
    if (nt < 1) nt = 1;
    dataset_t d;
    int rc = build_dataset(geno, ld, pheno, M, N, nt, &d);
    if (rc != EPI3H_OK || M < 3) {
        free_dataset(&d);
        return rc;
    }
    const corner_fn corners = isa == EPI3H_ISA_AVX512 ? corners_avx512
                              : isa == EPI3H_ISA_AVX2 ? corners_avx2
                                                      : corners_scalar;
    const int64_t total = (int64_t)M * (M - 1) * (M - 2) / 6;
    const int64_t keep = total < k ? total : k;
    topk_t *tk = (topk_t *)calloc((size_t)nt, sizeof(topk_t));
    int nomem = tk == NULL;
    for (int t = 0; !nomem && t < nt; ++t) {
        tk[t].keep = keep;
        tk[t].buf = (cand_t *)malloc(sizeof(cand_t) * (size_t)(2 * keep));
        nomem |= tk[t].buf == NULL;
    }
    if (!nomem) {
#pragma omp parallel num_threads(nt) reduction(| : nomem)
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            topk_t *T = &tk[tid];
            uint64_t *A[2];
            A[0] = (uint64_t *)alloc64(sizeof(uint64_t) * 4 * (size_t)d.Wp[0]);
            A[1] = (uint64_t *)alloc64(sizeof(uint64_t) * 4 * (size_t)d.Wp[1]);
            if (!A[0] || !A[1]) nomem = 1;
#pragma omp for schedule(dynamic, 1)
            for (int32_t i = 0; i < M - 2; ++i) {
                if (!A[0] || !A[1]) continue;
                for (int32_t j = i + 1; j < M - 1; ++j) {
                    for (int c = 0; c < 2; ++c) {
                        const int64_t Wp = d.Wp[c];
                        const uint64_t *P = d.planes[c];
                        for (int a = 0; a < 2; ++a)
                            for (int b = 0; b < 2; ++b) {
                                const uint64_t *xi = P + ((int64_t)i * 2 + a) * Wp;
                                const uint64_t *xj = P + ((int64_t)j * 2 + b) * Wp;
                                uint64_t *y = A[c] + (2 * a + b) * Wp;
                                for (int64_t w = 0; w < Wp; ++w) y[w] = xi[w] & xj[w];
                            }
                    }
                    for (int32_t k0 = j + 1; k0 < M; k0 += KB) {
                        const int nk = M - k0 < KB ? M - k0 : KB;
                        int32_t t0[KB][CELLS], t1[KB][CELLS];
                        double k2[KB];
                        for (int b = 0; b < nk; ++b) {
                            uint32_t cor[2][8];
                            for (int c = 0; c < 2; ++c)
                                corners(A[c], d.planes[c] + (int64_t)(k0 + b) * 2 * d.Wp[c],
                                        d.Wp[c], cor[c]);
                            complete(&d, 0, i, j, k0 + b, cor[0], t0[b]);
                            complete(&d, 1, i, j, k0 + b, cor[1], t1[b]);
                        }
                        k2_fp64_block(t0, t1, nk, d.L, k2);
                        for (int b = 0; b < nk; ++b) {
                            const cand_t cd = {k2[b], i, j, k0 + b};
                            topk_offer(T, &cd);
                        }
                    }
                }
            }
            free(A[0]);
            free(A[1]);
        }
    }
    if (nomem) {
        if (tk)
            for (int t = 0; t < nt; ++t) free(tk[t].buf);
        free(tk);
        free_dataset(&d);
        return EPI3H_E_NOMEM;
    }
    /* merge: every thread's survivors, sorted, first `keep` */
    int64_t n_all = 0;
    for (int t = 0; t < nt; ++t) {
        topk_cut(&tk[t]);
        n_all += tk[t].n;
    }
    cand_t *all = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n_all > 0 ? n_all : 1));
    if (!all) {
        for (int t = 0; t < nt; ++t) free(tk[t].buf);
        free(tk);
        free_dataset(&d);
        return EPI3H_E_NOMEM;
    }
    int64_t at = 0;
    for (int t = 0; t < nt; ++t) {
        memcpy(all + at, tk[t].buf, sizeof(cand_t) * (size_t)tk[t].n);
        at += tk[t].n;
        free(tk[t].buf);
    }
    free(tk);
    qsort(all, (size_t)n_all, sizeof(cand_t), cand_order);
    const int64_t n = n_all < keep ? n_all : keep;
    for (int64_t x = 0; x < n; ++x) {
        const cand_t *c = &all[x];
        epi3h_hit *h = &out[x];
        uint32_t cor[2][8];
        int32_t t[2][CELLS];
        /* counts of the winners, recounted by the scalar loop */
        for (int cl = 0; cl < 2; ++cl) {
            const int64_t Wp = d.Wp[cl];
            const uint64_t *P = d.planes[cl];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int e = 0; e < 2; ++e) {
                        uint64_t s = 0;
                        const uint64_t *xi = P + ((int64_t)c->i * 2 + a) * Wp;
                        const uint64_t *xj = P + ((int64_t)c->j * 2 + b) * Wp;
                        const uint64_t *xk = P + ((int64_t)c->k * 2 + e) * Wp;
                        for (int64_t w = 0; w < Wp; ++w)
                            s += (uint64_t)__builtin_popcountll(xi[w] & xj[w] & xk[w]);
                        cor[cl][4 * a + 2 * b + e] = (uint32_t)s;
                    }
            complete(&d, cl, c->i, c->j, c->k, cor[cl], t[cl]);
        }
        h->i = (uint32_t)c->i;
        h->j = (uint32_t)c->j;
        h->k = (uint32_t)c->k;
        h->k2 = c->k2;
        h->k2_f32 = (float)c->k2;
        for (int r = 0; r < CELLS; ++r) {
            h->counts[0][r] = (uint32_t)t[0][r];
            h->counts[1][r] = (uint32_t)t[1][r];
        }
    }
    *n_out = (int32_t)n;
    free(all);
    free_dataset(&d);
    return EPI3H_OK;
}
