/*
 * Plain CPU oracle for the exhaustive three-way epistasis scan.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file's library.  It shares no
 * code, header, table or constant with the GPU library, and the GPU library
 * never calls it.
 *
 * What it computes, straight from the paper (no blocking, no bit-planes,
 * no inclusion-exclusion):
 *   - Problem Formulation section: a data set of M SNPs x N samples with
 *     genotypes {0,1,2} and a phenotype {0 = control, 1 = case} per sample;
 *     for a SNP combination (i, j, k) the frequency table has 3^3 = 27 rows
 *     (one per genotype combination) and 2 columns (controls, cases).  The
 *     row of genotype combination (g_i, g_j, g_k) is 9*g_i + 3*g_j + g_k.
 *   - Eq. 1: K2 = sum over the 27 rows of
 *         ( sum_{b=1}^{r+1} log b  -  sum_{class} sum_{d=1}^{r_class} log d )
 *     with r the row total and r_class the row's per-class count; natural log.
 *     Each inner sum is a log factorial, L[n] = sum_{b=1}^{n} log b, summed
 *     in increasing b as written.  The row term is taken with Eq. 1's own
 *     bracketing, L[r+1] - (L[r_0] + L[r_1]), and the rows are summed in
 *     increasing row index.
 *   - The solution is the combination with the lowest K2 (end of the
 *     Problem Formulation section); this oracle returns the k lowest under
 *     the total order (K2, i, j, k), all indices 0-based with i < j < k.
 *   - Every combination with i < j < k is evaluated (both algorithms guard
 *     on the strict order of the three SNP indices).
 *   - The same for pairs of SNPs (3^2 = 9 rows per class, row 3 g_i + g_j)
 *     and quads (3^4 = 81 rows, row 27 g_i + 9 g_j + 3 g_k + g_l), Eq. 1
 *     being stated for any number of interacting SNPs; see the second- and
 *     fourth-order sections at the end.
 *
 * Parity of the K2 values with numbers printed in the paper is unpinned: the
 * paper prints none (its worked-example figure is not available).  The tests
 * pin this file against a brute-force big-integer evaluation, closed forms
 * and table invariants instead.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ROWS 27

/* L[n] = sum_{b=1}^{n} log(b), n = 0..nmax (Eq. 1's inner sums). */
void oracle_log_factorial(int32_t nmax, double *L)
{
    L[0] = 0.0;
    for (int32_t n = 1; n <= nmax; ++n)
        L[n] = L[n - 1] + log((double)n);
}

/* Frequency table of one combination: t[class * 27 + 9 g_i + 3 g_j + g_k]. */
void oracle_table(const uint8_t *G, int64_t ld, const uint8_t *ph, int32_t N,
                  int32_t i, int32_t j, int32_t k, int32_t *t)
{
    memset(t, 0, sizeof(int32_t) * 2 * ROWS);
    const uint8_t *gi = G + (int64_t)i * ld, *gj = G + (int64_t)j * ld, *gk = G + (int64_t)k * ld;
    for (int32_t s = 0; s < N; ++s)
        t[ph[s] * ROWS + 9 * gi[s] + 3 * gj[s] + gk[s]] += 1;
}

/* Eq. 1 for one table (controls in t[0..26], cases in t[27..53]). */
double oracle_k2(const int32_t *t, const double *L)
{
    double k2 = 0.0;
    for (int c = 0; c < ROWS; ++c) {
        int32_t r0 = t[c], r1 = t[ROWS + c];
        k2 += L[r0 + r1 + 1] - (L[r0] + L[r1]);
    }
    return k2;
}

/* -------- top-k under the order (K2, i, j, k) -------- */

typedef struct { double k2; int32_t i, j, k; } cand_t;

static int cand_less(const cand_t *a, const cand_t *b)
{
    if (a->k2 != b->k2) return a->k2 < b->k2;
    if (a->i != b->i) return a->i < b->i;
    if (a->j != b->j) return a->j < b->j;
    return a->k < b->k;
}

/* Bounded max-heap holding the best `cap` candidates seen so far. */
typedef struct { cand_t *h; int n, cap; } heap_t;

static void heap_push(heap_t *H, cand_t c)
{
    if (H->n < H->cap) {
        int x = H->n++;
        H->h[x] = c;
        while (x > 0) {
            int p = (x - 1) / 2;
            if (!cand_less(&H->h[p], &H->h[x])) break;
            cand_t tmp = H->h[p]; H->h[p] = H->h[x]; H->h[x] = tmp;
            x = p;
        }
        return;
    }
    if (!cand_less(&c, &H->h[0])) return;
    H->h[0] = c;
    int x = 0;
    for (;;) {
        int l = 2 * x + 1, r = l + 1, m = x;
        if (l < H->n && cand_less(&H->h[m], &H->h[l])) m = l;
        if (r < H->n && cand_less(&H->h[m], &H->h[r])) m = r;
        if (m == x) break;
        cand_t tmp = H->h[m]; H->h[m] = H->h[x]; H->h[x] = tmp;
        x = m;
    }
}

static int cand_cmp(const void *a, const void *b)
{
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (cand_less(x, y)) return -1;
    if (cand_less(y, x)) return 1;
    return 0;
}

/*
 * Exhaustive scan: every i < j < k, table by a plain loop over samples,
 * K2 by Eq. 1, keep the `topk` lowest.  Returns the number of hits
 * (min(topk, C(M,3))) written to out_ijk [n][3], out_k2 [n] and, when
 * non-NULL, out_counts [n][54].
 */
int32_t oracle_scan_topk(const uint8_t *G, int64_t ld, const uint8_t *ph,
                         int32_t M, int32_t N, int32_t topk, int32_t nthreads,
                         int32_t *out_ijk, double *out_k2, int32_t *out_counts)
{
    if (M < 3 || topk <= 0) return 0;
    double *L = (double *)malloc(sizeof(double) * ((size_t)N + 2));
    oracle_log_factorial(N + 1, L);
    int nt = nthreads > 0 ? nthreads : 1;
#ifndef _OPENMP
    nt = 1;
#endif
    heap_t *heaps = (heap_t *)calloc((size_t)nt, sizeof(heap_t));
    for (int t = 0; t < nt; ++t) {
        heaps[t].h = (cand_t *)malloc(sizeof(cand_t) * (size_t)topk);
        heaps[t].cap = topk;
    }
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        heap_t *H = &heaps[tid];
        int32_t *row = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
        int32_t t[2 * ROWS];
#pragma omp for schedule(dynamic, 1)
        for (int32_t i = 0; i < M - 2; ++i) {
            const uint8_t *gi = G + (int64_t)i * ld;
            for (int32_t j = i + 1; j < M - 1; ++j) {
                const uint8_t *gj = G + (int64_t)j * ld;
                /* class column and the first two genotype digits of the row */
                for (int32_t s = 0; s < N; ++s)
                    row[s] = ph[s] * ROWS + 9 * gi[s] + 3 * gj[s];
                for (int32_t k = j + 1; k < M; ++k) {
                    const uint8_t *gk = G + (int64_t)k * ld;
                    memset(t, 0, sizeof(t));
                    for (int32_t s = 0; s < N; ++s)
                        t[row[s] + gk[s]] += 1;
                    cand_t c = { oracle_k2(t, L), i, j, k };
                    heap_push(H, c);
                }
            }
        }
        free(row);
    }
    /* merge the per-thread heaps */
    int64_t total = 0;
    for (int t = 0; t < nt; ++t) total += heaps[t].n;
    cand_t *all = (cand_t *)malloc(sizeof(cand_t) * (size_t)(total > 0 ? total : 1));
    int64_t pos = 0;
    for (int t = 0; t < nt; ++t) {
        memcpy(all + pos, heaps[t].h, sizeof(cand_t) * (size_t)heaps[t].n);
        pos += heaps[t].n;
        free(heaps[t].h);
    }
    free(heaps);
    qsort(all, (size_t)total, sizeof(cand_t), cand_cmp);
    int32_t n = (int32_t)(total < topk ? total : topk);
    for (int32_t x = 0; x < n; ++x) {
        out_ijk[3 * x + 0] = all[x].i;
        out_ijk[3 * x + 1] = all[x].j;
        out_ijk[3 * x + 2] = all[x].k;
        out_k2[x] = all[x].k2;
        if (out_counts)
            oracle_table(G, ld, ph, N, all[x].i, all[x].j, all[x].k, out_counts + (int64_t)54 * x);
    }
    free(all);
    free(L);
    return n;
}

/* Tables and K2 of an explicit list of combinations (ijk [n][3]). */
void oracle_score_list(const uint8_t *G, int64_t ld, const uint8_t *ph, int32_t N,
                       const int32_t *ijk, int64_t n, int32_t nthreads,
                       int32_t *out_counts, double *out_k2)
{
    double *L = (double *)malloc(sizeof(double) * ((size_t)N + 2));
    oracle_log_factorial(N + 1, L);
    int nt = nthreads > 0 ? nthreads : 1;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 64)
    for (int64_t x = 0; x < n; ++x) {
        int32_t t[2 * ROWS];
        oracle_table(G, ld, ph, N, ijk[3 * x], ijk[3 * x + 1], ijk[3 * x + 2], t);
        if (out_counts) memcpy(out_counts + 54 * x, t, sizeof(t));
        if (out_k2) out_k2[x] = oracle_k2(t, L);
    }
    free(L);
}

/* Every combination in lexicographic (i, j, k) order: K2 [C(M,3)] and,
 * when non-NULL, tables [C(M,3)][54].  For small inputs only. */
void oracle_scan_all(const uint8_t *G, int64_t ld, const uint8_t *ph, int32_t M, int32_t N,
                     int32_t nthreads, double *out_k2, int32_t *out_counts)
{
    if (M < 3) return;
    double *L = (double *)malloc(sizeof(double) * ((size_t)N + 2));
    oracle_log_factorial(N + 1, L);
    /* offset of the first combination with a given i */
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)M);
    int64_t acc = 0;
    for (int32_t i = 0; i < M; ++i) {
        off[i] = acc;
        int64_t rest = M - 1 - i;
        acc += rest * (rest - 1) / 2;
    }
    int nt = nthreads > 0 ? nthreads : 1;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int32_t i = 0; i < M - 2; ++i) {
        int64_t x = off[i];
        int32_t t[2 * ROWS];
        for (int32_t j = i + 1; j < M - 1; ++j)
            for (int32_t k = j + 1; k < M; ++k, ++x) {
                oracle_table(G, ld, ph, N, i, j, k, t);
                out_k2[x] = oracle_k2(t, L);
                if (out_counts) memcpy(out_counts + 54 * x, t, sizeof(t));
            }
    }
    free(off);
    free(L);
}

/* -------- second order: SNP pairs --------
 *
 * Eq. 1 is stated for any number of interacting SNPs: with two SNPs the
 * table has 3^2 = 9 rows per class, row 3 g_i + g_j, and K2 sums the same
 * row term over those 9 rows.  Pairs are i < j, ordered by (K2, i, j).
 */
#define ROWS2 9

/* Frequency table of one pair: t[class * 9 + 3 g_i + g_j]. */
void oracle_table2(const uint8_t *G, int64_t ld, const uint8_t *ph, int32_t N,
                   int32_t i, int32_t j, int32_t *t)
{
    memset(t, 0, sizeof(int32_t) * 2 * ROWS2);
    const uint8_t *gi = G + (int64_t)i * ld, *gj = G + (int64_t)j * ld;
    for (int32_t s = 0; s < N; ++s)
        t[ph[s] * ROWS2 + 3 * gi[s] + gj[s]] += 1;
}

/* Eq. 1 for a table of `rows` rows (controls t[0..rows), cases t[rows..2 rows)),
 * same bracketing and row order as oracle_k2. */
double oracle_k2_rows(const int32_t *t, int32_t rows, const double *L)
{
    double k2 = 0.0;
    for (int32_t c = 0; c < rows; ++c) {
        int32_t p0 = t[c], p1 = t[rows + c];
        k2 += L[p0 + p1 + 1] - (L[p0] + L[p1]);
    }
    return k2;
}

/* Every pair in lexicographic (i, j) order: K2 [C(M,2)] and, when non-NULL,
 * tables [C(M,2)][18]. */
void oracle_scan_pairs_all(const uint8_t *G, int64_t ld, const uint8_t *ph, int32_t M, int32_t N,
                           int32_t nthreads, double *out_k2, int32_t *out_counts)
{
    if (M < 2) return;
    double *L = (double *)malloc(sizeof(double) * ((size_t)N + 2));
    oracle_log_factorial(N + 1, L);
    int nt = nthreads > 0 ? nthreads : 1;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int32_t i = 0; i < M - 1; ++i) {
        /* pairs before row i: sum over i' < i of (M - 1 - i') */
        int64_t x = (int64_t)i * (M - 1) - (int64_t)i * (i - 1) / 2;
        int32_t t[2 * ROWS2];
        for (int32_t j = i + 1; j < M; ++j, ++x) {
            oracle_table2(G, ld, ph, N, i, j, t);
            out_k2[x] = oracle_k2_rows(t, ROWS2, L);
            if (out_counts) memcpy(out_counts + 2 * ROWS2 * x, t, sizeof(t));
        }
    }
    free(L);
}

/* Exhaustive pair scan keeping the `topk` lowest under (K2, i, j); returns
 * the number of hits (min(topk, C(M,2))) written to out_ij [n][2], out_k2 [n]
 * and, when non-NULL, out_counts [n][18]. */
int32_t oracle_scan_pairs_topk(const uint8_t *G, int64_t ld, const uint8_t *ph,
                               int32_t M, int32_t N, int32_t topk, int32_t nthreads,
                               int32_t *out_ij, double *out_k2, int32_t *out_counts)
{
    if (M < 2 || topk <= 0) return 0;
    double *L = (double *)malloc(sizeof(double) * ((size_t)N + 2));
    oracle_log_factorial(N + 1, L);
    int nt = nthreads > 0 ? nthreads : 1;
#ifndef _OPENMP
    nt = 1;
#endif
    heap_t *heaps = (heap_t *)calloc((size_t)nt, sizeof(heap_t));
    for (int t = 0; t < nt; ++t) {
        heaps[t].h = (cand_t *)malloc(sizeof(cand_t) * (size_t)topk);
        heaps[t].cap = topk;
    }
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        heap_t *H = &heaps[tid];
        int32_t t[2 * ROWS2];
#pragma omp for schedule(dynamic, 1)
        for (int32_t i = 0; i < M - 1; ++i)
            for (int32_t j = i + 1; j < M; ++j) {
                oracle_table2(G, ld, ph, N, i, j, t);
                cand_t c = { oracle_k2_rows(t, ROWS2, L), i, j, 0 };
                heap_push(H, c);
            }
    }
    int64_t total = 0;
    for (int t = 0; t < nt; ++t) total += heaps[t].n;
    cand_t *all = (cand_t *)malloc(sizeof(cand_t) * (size_t)(total > 0 ? total : 1));
    int64_t pos = 0;
    for (int t = 0; t < nt; ++t) {
        memcpy(all + pos, heaps[t].h, sizeof(cand_t) * (size_t)heaps[t].n);
        pos += heaps[t].n;
        free(heaps[t].h);
    }
    free(heaps);
    qsort(all, (size_t)total, sizeof(cand_t), cand_cmp);
    int32_t n = (int32_t)(total < topk ? total : topk);
    for (int32_t x = 0; x < n; ++x) {
        out_ij[2 * x + 0] = all[x].i;
        out_ij[2 * x + 1] = all[x].j;
        out_k2[x] = all[x].k2;
        if (out_counts)
            oracle_table2(G, ld, ph, N, all[x].i, all[x].j, out_counts + (int64_t)2 * ROWS2 * x);
    }
    free(all);
    free(L);
    return n;
}

/* -------- fourth order: SNP quads --------
 *
 * Four interacting SNPs: 3^4 = 81 rows per class, row 27 g_i + 9 g_j +
 * 3 g_k + g_l, i < j < k < l, ordered by (K2, i, j, k, l).
 */
#define ROWS4 81

typedef struct { double k2; int32_t i, j, k, l; } cand4_t;

static int cand4_less(const cand4_t *a, const cand4_t *b)
{
    if (a->k2 != b->k2) return a->k2 < b->k2;
    if (a->i != b->i) return a->i < b->i;
    if (a->j != b->j) return a->j < b->j;
    if (a->k != b->k) return a->k < b->k;
    return a->l < b->l;
}

static int cand4_cmp(const void *a, const void *b)
{
    const cand4_t *x = (const cand4_t *)a, *y = (const cand4_t *)b;
    if (cand4_less(x, y)) return -1;
    if (cand4_less(y, x)) return 1;
    return 0;
}

/* Frequency table of one quad: t[class * 81 + 27 g_i + 9 g_j + 3 g_k + g_l]. */
void oracle_table4(const uint8_t *G, int64_t ld, const uint8_t *ph, int32_t N,
                   int32_t i, int32_t j, int32_t k, int32_t l, int32_t *t)
{
    memset(t, 0, sizeof(int32_t) * 2 * ROWS4);
    const uint8_t *gi = G + (int64_t)i * ld, *gj = G + (int64_t)j * ld;
    const uint8_t *gk = G + (int64_t)k * ld, *gl = G + (int64_t)l * ld;
    for (int32_t s = 0; s < N; ++s)
        t[ph[s] * ROWS4 + 27 * gi[s] + 9 * gj[s] + 3 * gk[s] + gl[s]] += 1;
}

/* Every quad in lexicographic (i, j, k, l) order: K2 [C(M,4)] and, when
 * non-NULL, tables [C(M,4)][162].  For small inputs only. */
void oracle_scan_quads_all(const uint8_t *G, int64_t ld, const uint8_t *ph, int32_t M, int32_t N,
                           int32_t nthreads, double *out_k2, int32_t *out_counts)
{
    if (M < 4) return;
    double *L = (double *)malloc(sizeof(double) * ((size_t)N + 2));
    oracle_log_factorial(N + 1, L);
    /* offset of the first quad with a given i: sum over i' < i of C(M-1-i', 3) */
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)M);
    int64_t acc = 0;
    for (int32_t i = 0; i < M; ++i) {
        off[i] = acc;
        int64_t rest = M - 1 - i;
        acc += rest * (rest - 1) * (rest - 2) / 6;
    }
    int nt = nthreads > 0 ? nthreads : 1;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int32_t i = 0; i < M - 3; ++i) {
        int64_t x = off[i];
        int32_t t[2 * ROWS4];
        for (int32_t j = i + 1; j < M - 2; ++j)
            for (int32_t k = j + 1; k < M - 1; ++k)
                for (int32_t l = k + 1; l < M; ++l, ++x) {
                    oracle_table4(G, ld, ph, N, i, j, k, l, t);
                    out_k2[x] = oracle_k2_rows(t, ROWS4, L);
                    if (out_counts) memcpy(out_counts + 2 * ROWS4 * x, t, sizeof(t));
                }
    }
    free(off);
    free(L);
}

/* Exhaustive quad scan keeping the `topk` lowest under (K2, i, j, k, l):
 * returns min(topk, C(M,4)) hits in out_ijkl [n][4], out_k2 [n] and, when
 * non-NULL, out_counts [n][162]. */
int32_t oracle_scan_quads_topk(const uint8_t *G, int64_t ld, const uint8_t *ph,
                               int32_t M, int32_t N, int32_t topk, int32_t nthreads,
                               int32_t *out_ijkl, double *out_k2, int32_t *out_counts)
{
    if (M < 4 || topk <= 0) return 0;
    double *L = (double *)malloc(sizeof(double) * ((size_t)N + 2));
    oracle_log_factorial(N + 1, L);
    int nt = nthreads > 0 ? nthreads : 1;
#ifndef _OPENMP
    nt = 1;
#endif
    /* per-thread sorted arrays of the best `topk` (insertion; topk is small) */
    cand4_t *best = (cand4_t *)malloc(sizeof(cand4_t) * (size_t)topk * (size_t)nt);
    int32_t *nbest = (int32_t *)calloc((size_t)nt, sizeof(int32_t));
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        cand4_t *B = best + (size_t)tid * topk;
        int32_t nb = 0;
        int32_t t[2 * ROWS4];
#pragma omp for schedule(dynamic, 1)
        for (int32_t i = 0; i < M - 3; ++i)
            for (int32_t j = i + 1; j < M - 2; ++j)
                for (int32_t k = j + 1; k < M - 1; ++k)
                    for (int32_t l = k + 1; l < M; ++l) {
                        oracle_table4(G, ld, ph, N, i, j, k, l, t);
                        cand4_t c = { oracle_k2_rows(t, ROWS4, L), i, j, k, l };
                        if (nb == topk && !cand4_less(&c, &B[nb - 1])) continue;
                        int32_t p = nb < topk ? nb++ : topk - 1;
                        while (p > 0 && cand4_less(&c, &B[p - 1])) { B[p] = B[p - 1]; --p; }
                        B[p] = c;
                    }
        nbest[tid] = nb;
    }
    int64_t total = 0;
    for (int t = 0; t < nt; ++t) total += nbest[t];
    cand4_t *all = (cand4_t *)malloc(sizeof(cand4_t) * (size_t)(total > 0 ? total : 1));
    int64_t pos = 0;
    for (int t = 0; t < nt; ++t) {
        memcpy(all + pos, best + (size_t)t * topk, sizeof(cand4_t) * (size_t)nbest[t]);
        pos += nbest[t];
    }
    qsort(all, (size_t)total, sizeof(cand4_t), cand4_cmp);
    int32_t n = (int32_t)(total < topk ? total : topk);
    for (int32_t x = 0; x < n; ++x) {
        out_ijkl[4 * x + 0] = all[x].i;
        out_ijkl[4 * x + 1] = all[x].j;
        out_ijkl[4 * x + 2] = all[x].k;
        out_ijkl[4 * x + 3] = all[x].l;
        out_k2[x] = all[x].k2;
        if (out_counts)
            oracle_table4(G, ld, ph, N, all[x].i, all[x].j, all[x].k, all[x].l,
                          out_counts + (int64_t)2 * ROWS4 * x);
    }
    free(all);
    free(nbest);
    free(best);
    free(L);
    return n;
}
