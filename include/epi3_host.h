/*
 * epi3_host -- the same exhaustive three-way scan on the host CPU cores.
 *
 * C ABI of libepi3_host.so, a measured CPU baseline that sits beside the
 * GPU library (libepi3.so never calls it and it never calls the GPU).  It
 * follows the paper's fourth CPU approach (CPU approaches section, Alg. 1
 * and the vectorization paragraph after it): case/control-split bit planes
 * of genotypes 0 and 1, a working set held in the first cache levels, vector
 * AND + POPCNT, an OpenMP dynamic schedule with per-thread results merged at
 * the end.  Like the GPU library it counts only the 8 cells whose genotypes
 * are all 0 or 1 and completes the other 19 from pair and single-SNP counts,
 * so each (triplet, 64 samples) costs 8 AND + 8 POPCNT instead of 27.
 *
 * Conventions are those of epi3.h: 0-based triplets i < j < k < M, table row
 * 9 g_i + 3 g_j + g_k, column 0 = controls, column 1 = cases, K2 by Eq. 1
 * with natural log, results ordered by (K2, i, j, k).  K2 is evaluated in
 * FP64 for every triplet, rows in increasing index, each row as
 * L[r + 1] - (L[r_0] + L[r_1]) with L[n] = sum_{b <= n} log b summed in
 * increasing b, so the order is exact without a screen.
 *
 * All pointers are host memory owned by the caller.  Return value: 0 or a
 * negative code below.  Safe to call from several threads at once.
 */
#ifndef EPI3_HOST_H
#define EPI3_HOST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    EPI3H_OK = 0,
    EPI3H_E_INVALID = -1,     /* null pointer, M < 0, N <= 0, ld < N, k <= 0, bad isa */
    EPI3H_E_GENOTYPE = -2,    /* a genotype byte outside {0,1,2} */
    EPI3H_E_PHENOTYPE = -3,   /* a phenotype byte outside {0,1} */
    EPI3H_E_UNSUPPORTED = -7, /* the requested instruction set is not on this CPU */
    EPI3H_E_NOMEM = -8        /* a host allocation failed */
};

/* Instruction-set levels of the counting loop. */
enum {
    EPI3H_ISA_BEST = -1,      /* the highest level this CPU supports */
    EPI3H_ISA_SCALAR = 0,     /* 64-bit AND + popcount builtin */
    EPI3H_ISA_AVX2 = 1,       /* 256-bit AND, nibble-table popcount (vpshufb) + vpsadbw */
    EPI3H_ISA_AVX512 = 2      /* 512-bit AND + vpopcntq (AVX512F + AVX512_VPOPCNTDQ) */
};

/* Same layout as epi3_hit; k2_f32 is fl32(k2) here (there is no FP32 screen). */
typedef struct {
    uint32_t i, j, k;
    float k2_f32;
    double k2;
    uint32_t counts[2][27];
} epi3h_hit;

/* Highest EPI3H_ISA_* level this CPU supports. */
int epi3h_best_isa(void);

/*
 * Exhaustive scan of every triplet, k lowest K2.
 *   geno   [M][ld] bytes, genotype of SNP m and sample s at geno[m * ld + s],
 *          values 0/1/2 (number of minor alleles);
 *   pheno  [N] bytes, 0 = control, 1 = case;
 *   threads  OpenMP threads (<= 0: the OpenMP default);
 *   isa      EPI3H_ISA_*; a level this CPU lacks returns EPI3H_E_UNSUPPORTED;
 *   out      room for min(k, C(M,3)) hits, written in ascending order;
 *   n_out    number of hits written (0 when M < 3).
 */
int epi3h_scan_topk(const uint8_t *geno, int64_t ld, const uint8_t *pheno, int32_t M,
                    int32_t N, int32_t k, int32_t threads, int32_t isa, epi3h_hit *out,
                    int32_t *n_out);

#ifdef __cplusplus
}
#endif

#endif /* EPI3_HOST_H */
