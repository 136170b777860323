/*
 * epi3 -- exhaustive three-way epistasis scan (K2 score) on AMD MI355X (gfx950).
 *
 * C ABI of libepi3.so.  The library implements the hot path of
 * Marques et al., "Three-way Gene Interaction Study on modern CPUs and GPUs"
 * (arXiv 2201.10956):
 *
 *   data set D            Problem Formulation section: M SNPs x N samples,
 *                         genotype 0/1/2 per (SNP, sample), phenotype 0
 *                         (control) / 1 (case) per sample;
 *   frequency table       same section: 27 genotype rows x 2 classes per SNP
 *                         triplet, filled by AND + POPCNT over per-genotype
 *                         sample bit-planes (binarized format, Fig. 1 text);
 *   K2 score              Eq. 1 (natural log, J = 2 classes, I = 27 rows);
 *   solution              the triplet with the lowest K2; generalised here to
 *                         the k lowest under the total order (K2, i, j, k).
 *
 * Conventions shared by every call:
 *   - Indices are 0-based; a triplet is (i, j, k) with i < j < k < M.
 *   - Table row of genotype combination (g_i, g_j, g_k) is 9 g_i + 3 g_j + g_k;
 *     column 0 counts controls, column 1 counts cases.
 *   - Every `*_dev` pointer and every buffer named "device" is device memory
 *     owned by the caller; the library never allocates, frees or retains it
 *     beyond the call (except the cached graphs noted at epi3_scan_batched).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     their GPU work on it.  Calls that return host results (epi3_topk,
 *     epi3_scan_batched) and epi3_encode synchronise that stream before
 *     returning; the others are asynchronous.
 *   - Return value: EPI3_OK or a negative EPI3_E_* code; no exception crosses
 *     the ABI.  Data errors detected on the device (a genotype byte outside
 *     {0,1,2}) are reported by the next call that returns host results.
 *   - Calls on distinct streams with distinct workspaces may run concurrently
 *     (the matrix-core paths order their finish kernels with a second stream
 *     and events of their own, taken from a library pool for the duration of
 *     the call).  The tile rules, pass bytes and other process-wide settings
 *     must not change while a scan is in progress; the kernel-timing hooks
 *     sum the launches of all threads.
 *
 * K2 is screened in FP32 from a table of log factorials and the returned
 * order is decided by an FP64 re-score of every candidate that the FP32
 * error bound cannot exclude, so the hits equal the exact-order top-k of an
 * FP64 evaluation of Eq. 1; table counts are exact integers.
 */
#ifndef EPI3_H
#define EPI3_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    EPI3_OK = 0,
    EPI3_E_INVALID = -1,    /* null pointer, negative size, k <= 0, bad layout, mixed batch */
    EPI3_E_GENOTYPE = -2,   /* a genotype byte outside {0,1,2} (device-detected) */
    EPI3_E_PHENOTYPE = -3,  /* a phenotype byte outside {0,1} */
    EPI3_E_WORKSPACE = -4,  /* buffer smaller than the matching *_bytes() query */
    EPI3_E_CAPACITY = -5,   /* more FP32-screen candidates than the workspace holds */
    EPI3_E_HIP = -6,        /* a HIP runtime call failed */
    EPI3_E_UNSUPPORTED = -7 /* variant not available for this layout */
};

/* Plane layouts produced by epi3_encode. */
enum {
    /* Samples split by class (paper, CPU approaches section: controls array
     * and cases array per SNP; plane 2 is never stored because it is implied
     * by planes 0 and 1). */
    EPI3_LAYOUT_SPLIT = 0,
    /* All samples in one set of planes; the class of each sample comes from a
     * case mask supplied per job (used for phenotype permutations). */
    EPI3_LAYOUT_MASKED = 1
};

/* Flag OR'ed into the layout of epi3_encode_bytes / epi3_encode (SPLIT only):
 * encode the bit planes, pairwise tables and log-factorial tables but not the
 * 0/1 value planes (out->bytes = out->nibbles = NULL).  The pair and quad
 * scans and the vector-ALU triplet scan read bit planes only; on such a data
 * set the matrix-core variants return EPI3_E_UNSUPPORTED and
 * EPI3_VARIANT_AUTO takes the vector-ALU kernel. */
enum { EPI3_ENCODE_BITS_ONLY = 0x100 };

/* Count-stage kernels. */
enum {
    EPI3_VARIANT_AUTO = 0,  /* library choice (see epi3_tile_rule) */
    EPI3_VARIANT_VALU = 1,  /* AND + v_bcnt popcount on the vector ALU */
    EPI3_VARIANT_MFMA = 2,  /* 0/1 byte matrices on int8 matrix cores, int32 accumulation */
    EPI3_VARIANT_MFMA_FP4 = 3 /* 0/1 values as FP4 (E2M1) on the matrix cores, FP32 accumulation
                                 (exact: every count is an integer below 2^24) */
};

/* An encoded data set.  Plain data; every pointer points into the caller's
 * buffer passed to epi3_encode.  Filled by epi3_encode, read by the scans. */
typedef struct {
    int32_t n_snps;       /* M */
    int32_t n_samples;    /* N */
    int32_t n_cases;      /* N1 */
    int32_t n_controls;   /* N0 */
    int32_t words[2];     /* 32-sample words of controls, cases (MASKED: all samples in both) */
    int32_t layout;       /* EPI3_LAYOUT_* */
    int32_t snp_stride;   /* padded SNP count of the plane arrays */
    int32_t byte_stride;  /* padded sample count of the value planes (per class for SPLIT) */
    int32_t reserved;
    void *planes;         /* device: bit planes  [word][snp_stride][2] uint32 */
    void *bytes;          /* device: 0/1 value planes [class][snp_stride][2][byte_stride] bytes
                             (MASKED: one class of all samples; SPLIT: controls, cases) */
    void *nibbles;        /* device: the same as E2M1 nibbles, 0x2 = 1.0, two samples per byte
                             (low nibble first) [class][snp_stride][2][byte_stride / 2] */
    int32_t *pairs;       /* device: pairwise tables [class][snp_stride][snp_stride][4] */
    double *lf64;         /* device: log factorials L[0..N+1] in FP64 */
    float *lf32;          /* device: the same rounded to FP32 */
    int32_t *status;      /* device: status word (bit 0: bad genotype byte) */
} epi3_dataset;

/* One hit of the top-k.  counts[c][9 g_i + 3 g_j + g_k], c = 0 controls, 1 cases. */
typedef struct {
    uint32_t i, j, k;
    float k2_f32;         /* FP32 screen value computed by the scan */
    double k2;            /* FP64 value of Eq. 1 (rows summed in row order) */
    uint32_t counts[2][27];
} epi3_hit;

/* One job of a batched scan: a data set, optionally with its own case mask. */
typedef struct {
    const epi3_dataset *d;
    const uint32_t *case_mask; /* device, MASKED only: bit s of word s/32 = 1 if sample s is a case */
    int32_t k;                 /* hits wanted for this job */
    int32_t reserved;
} epi3_job;

/* ---------------------------------------------------------------------------
 * Encoding (binarized format: Problem Formulation section and Fig. 1 text;
 * reduced format: CPU approaches section -- plane 2 implied by planes 0 and 1,
 * samples split into controls and cases; 32-bit words: start of the
 * Approaches section; SNP-minor order so that lanes owning consecutive SNPs
 * read consecutive words: GPU approaches section).
 * ------------------------------------------------------------------------ */

/* Bytes of device buffer epi3_encode needs.  Returns < 0 on bad arguments. */
int64_t epi3_encode_bytes(int32_t n_snps, int32_t n_cases, int32_t n_controls, int32_t layout);

/*
 * Encode a genotype matrix.
 *   geno_dev   device uint8 [n_snps][ld], row = SNP, values {0,1,2}; ld >= n_samples.
 *   pheno_host host uint8 [n_samples], values {0,1}; read before return.
 *   buf_dev    device buffer of at least epi3_encode_bytes(...) bytes, 256-byte aligned;
 *              holds planes, pairwise tables, log-factorial tables and the status word,
 *              and must outlive every use of *out.
 *   out        host struct filled on success.
 * Also computes the pairwise tables the scans need (pairs of SNPs, per class).
 * Synchronises `stream`.  Genotype errors are flagged in out->status and returned
 * by the next epi3_topk / epi3_scan_batched.
 */
int epi3_encode(const uint8_t *geno_dev, int64_t ld, const uint8_t *pheno_host,
                int32_t n_snps, int32_t n_samples, int32_t layout,
                void *buf_dev, int64_t buf_bytes, void *stream, epi3_dataset *out);

/* ---------------------------------------------------------------------------
 * Plain scan (one data set, SPLIT layout): every triplet's table and K2
 * (Alg. 2 semantics: all i < j < k, private table per triplet, score after all
 * samples), then the k lowest.
 * ------------------------------------------------------------------------ */

/* Workspace bytes for epi3_scan + epi3_topk with count kernel `variant`.
 * cand_cap <= 0 picks a default capacity for FP32-screen candidates.  The
 * matrix-core variants add a scratch buffer for counted corner cells at the
 * end of the workspace (and, selecting by bound, a sample plane); the
 * selection state and the hits sit at the same offset for all variants.
 * The FP32 score plane (4 C(M,3) bytes) is part of it unless the scan selects
 * by bound (epi3_set_scan_select). */
int64_t epi3_workspace_bytes(const epi3_dataset *d, int32_t k, int32_t variant, int64_t cand_cap);

/* Count + score every triplet and select candidates; asynchronous.
 * variant: EPI3_VARIANT_*.  EPI3_VARIANT_MFMA and _MFMA_FP4 need class sizes
 * of at most 65535 samples, value planes of fewer than 2^32 bytes
 * (2 snp_stride 2 byte_stride) and fewer than 2^32 pair-table entries
 * (2 snp_stride^2, i.e. up to about 46000 SNPs) (EPI3_E_UNSUPPORTED
 * otherwise; AUTO then counts on the vector ALU).  Selecting by
 * bound (epi3_set_scan_select) needs a matrix-core variant
 * (EPI3_E_UNSUPPORTED for EPI3_VARIANT_VALU).
 * ws_dev: device workspace of epi3_workspace_bytes(d, k, variant, cand_cap)
 * bytes (256-byte aligned). */
int epi3_scan(const epi3_dataset *d, int32_t k, int32_t variant, int64_t cand_cap,
              void *ws_dev, int64_t ws_bytes, void *stream);

/* Re-score candidates in FP64, order them and copy min(k, C(M,3)) hits to
 * hits_host [k]; *n_out receives the count.  Synchronises `stream`.
 * EPI3_E_CAPACITY: *n_out receives the candidate count needed (selecting by
 * bound: the cand_cap whose list, 16 x cand_cap entries, holds every score
 * under the bound); retry with cand_cap >= that value. */
int epi3_topk(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
              epi3_hit *hits_host, int32_t *n_out, void *stream);

/* Device address of the FP32 score plane inside a plain-scan workspace:
 * K2_fp32 of every triplet in lexicographic (i, j, k) order, C(M,3) floats,
 * valid once the stream has run epi3_scan (and until the workspace is reused).
 * EPI3_E_UNSUPPORTED when the scan selects by bound (no plane). */
int epi3_score_plane(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                     float **plane_dev);

/* ---------------------------------------------------------------------------
 * Allocation-free plain scan, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Not a step of the paper's method: the same vector-ALU count
 * kernel and selection as epi3_scan + epi3_topk with EPI3_VARIANT_VALU, whose
 * workspace is a device array of EPI3_STATIC_SCRATCH_BYTES inside the library
 * instead of a caller buffer (each GPU the library runs on holds its own copy
 * from the first call on it, or from epi3_init, until the process ends).
 * ------------------------------------------------------------------------ */

/* Size of the library's static workspace: the FP32 score plane of the data
 * set (4 C(M,3) bytes) plus about 1 MB of selection buffers must fit, so M is
 * limited to about 580 SNPs (C(M,3) up to about 33 million triplets). */
#define EPI3_STATIC_SCRATCH_BYTES (128ll << 20)

/* epi3_scan + epi3_topk (variant EPI3_VARIANT_VALU, default candidate
 * capacity) with the static workspace: copies min(k, C(M,3)) hits to
 * hits_host [k] and their number to *n_out; synchronises `stream`.  Calls no
 * device or host allocator.  Returns EPI3_E_WORKSPACE (nothing enqueued) when
 * epi3_workspace_bytes(d, k, EPI3_VARIANT_VALU, 0) exceeds
 * EPI3_STATIC_SCRATCH_BYTES, EPI3_E_CAPACITY when more candidates pass the
 * FP32 screen than the default capacity holds (*n_out = candidates needed;
 * use epi3_scan with a larger cand_cap), and the other codes of epi3_scan /
 * epi3_topk.  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (two host threads, or two streams) race and
 * must not be made; each call initialises every part of the array it reads,
 * so what a previous call left there does not matter. */
int epi3_scan_topk_static(const epi3_dataset *d, int32_t k, epi3_hit *hits_host,
                          int32_t *n_out, void *stream);

/* ---------------------------------------------------------------------------
 * Batched scans in one persistent launch, captured into a HIP graph that is
 * cached per job signature (released by epi3_release).  Not in the paper,
 * which scans one data set per run.
 *   - SPLIT jobs: independent data sets of any shape (own phenotype).
 *   - MASKED jobs: all jobs share one data set; each job's case_mask is one
 *     phenotype (e.g. a permutation).
 * hits_host holds sum_j k_j hits, job after job; n_out_host [n_jobs].
 * ------------------------------------------------------------------------ */

/* variant: SPLIT jobs run the count kernel each would run in a plain scan
 * with that variant (AUTO follows the tile table per data set; vector-ALU
 * jobs share one persistent launch, and matrix-core jobs of one operand type
 * and tile shape share one sequence of passes over their tiles, the data
 * sets with the most samples first); MASKED jobs run on the matrix cores (AUTO = FP4; VALU is
 * EPI3_E_UNSUPPORTED) and need at most 65535 samples and value planes of
 * fewer than 2^32 bytes (snp_stride 2 byte_stride), else
 * EPI3_E_UNSUPPORTED.  The workspace depends on the variant. */
int64_t epi3_batched_workspace_bytes(const epi3_job *jobs, int32_t n_jobs, int32_t variant,
                                     int64_t cand_cap);

int epi3_scan_batched(const epi3_job *jobs, int32_t n_jobs, int32_t variant, int64_t cand_cap,
                      void *ws_dev, int64_t ws_bytes, epi3_hit *hits_host,
                      int32_t *n_out_host, void *stream);

/* Device address of job `job`'s FP32 score plane inside a batched workspace:
 * K2_fp32 of every triplet of that job's data set (and, for MASKED jobs, its
 * case mask) in lexicographic (i, j, k) order, C(M,3) floats; the arguments
 * are those of the epi3_scan_batched call that filled it, and the plane is
 * valid once the stream has run that call (until the workspace is reused);
 * the process-wide settings (tile rules, pass bytes, compacted-list size,
 * batch selection) must still be those of that call, since they lay the
 * workspace out.  A test hook: the FP32 screen values of the batched count
 * kernels.
 * EPI3_E_UNSUPPORTED when the batch keeps no plane (see
 * epi3_set_batch_select). */
int epi3_batched_score_plane(const epi3_job *jobs, int32_t n_jobs, int32_t variant,
                             int64_t cand_cap, void *ws_dev, int32_t job, float **plane_dev);

/* Test hook of a phenotype batch selected by bound (EPI3_BATCH_SELECT_BOUNDED):
 * job `job`'s list as the last epi3_scan_batched call on this workspace left
 * it.  *keys_dev / *ranks_dev: device arrays of *count entries in no
 * particular order, each the key of an FP32 score (its bit pattern with the
 * sign bit set; scores are non-negative) and the triplet's lexicographic
 * rank; *bound: the list's bound (every score <= it is listed).  Arguments
 * as for epi3_batched_score_plane; synchronises `stream`.
 * EPI3_E_UNSUPPORTED when the batch keeps a score plane instead. */
int epi3_batched_bound_list(const epi3_job *jobs, int32_t n_jobs, int32_t variant,
                            int64_t cand_cap, void *ws_dev, int32_t job, uint32_t **keys_dev,
                            int64_t **ranks_dev, int64_t *count, float *bound, void *stream);

/* Family-wise permutation p-value of an observed best score (not in the
 * paper): p = (1 + #{q : perm_min_k2[q] <= observed_k2}) / (n_perm + 1), where
 * perm_min_k2[q] is the lowest K2 of phenotype permutation q (hit 0 of job q of
 * a MASKED batched scan) and observed_k2 the lowest K2 of the real phenotype.
 * Lower K2 is stronger evidence, so a permutation counts when its best is at
 * least as low.  Host arrays; EPI3_E_INVALID for n_perm < 1 or NULL pointers
 * or a NaN score. */
int epi3_perm_pvalue(double observed_k2, const double *perm_min_k2, int32_t n_perm, double *p_out);

/* ---------------------------------------------------------------------------
 * Second-order scan: pairs of SNPs (SPLIT data sets).  Not the paper's target
 * order, but Eq. 1 is stated for any number of interacting SNPs (I = 3^k rows);
 * here I = 9.  A pair is (i, j), i < j < M; the table row of (g_i, g_j) is
 * 3 g_i + g_j.  The four cells with g_i, g_j in {0, 1} of each class are the
 * pairwise tables epi3_encode computes; the other five follow from the
 * per-SNP counts and the class size.  Hits are the k lowest under (K2, i, j)
 * with the same FP32 screen and FP64 re-score as the triplet scan (the
 * re-score recounts the table from the bit planes).
 * ------------------------------------------------------------------------ */

/* One hit of a pair scan.  counts[c][3 g_i + g_j], c = 0 controls, 1 cases. */
typedef struct {
    uint32_t i, j;
    float k2_f32;         /* FP32 screen value */
    uint32_t reserved;
    double k2;            /* FP64 value of Eq. 1 over the 9 rows, in row order */
    uint32_t counts[2][9];
} epi3_pair_hit;

/* Number of pairs C(M,2). */
int64_t epi3_n_pairs(int32_t n_snps);

/* Upper bound on |K2_fp32 - K2_fp64| of a 9-row table of N samples. */
double epi3_k2_error_bound_pairs(int32_t n_samples);

/* Workspace bytes for epi3_scan_pairs + epi3_pairs_topk (cand_cap as for
 * epi3_workspace_bytes).  EPI3_E_UNSUPPORTED for a MASKED data set. */
int64_t epi3_pairs_workspace_bytes(const epi3_dataset *d, int32_t k, int64_t cand_cap);

/* Score every pair (FP32, from the encoded pairwise tables) and select
 * candidates; asynchronous.  ws_dev: 256-byte aligned device workspace of
 * epi3_pairs_workspace_bytes(d, k, cand_cap) bytes. */
int epi3_scan_pairs(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                    int64_t ws_bytes, void *stream);

/* Copy min(k, C(M,2)) hits to hits_host [k]; *n_out receives the count.
 * Synchronises `stream`; EPI3_E_CAPACITY as for epi3_topk. */
int epi3_pairs_topk(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                    epi3_pair_hit *hits_host, int32_t *n_out, void *stream);

/* Device address of the pair scan's FP32 score plane: K2_fp32 of every pair
 * in lexicographic (i, j) order, C(M,2) floats, valid once the stream has run
 * epi3_scan_pairs. */
int epi3_pairs_score_plane(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                           float **plane_dev);

/* ---------------------------------------------------------------------------
 * Fourth-order scan: quads of SNPs (SPLIT data sets), Eq. 1 with I = 81
 * rows.  A quad is (i, j, k, l), i < j < k < l < M; the table row of
 * (g_i, g_j, g_k, g_l) is 27 g_i + 9 g_j + 3 g_k + g_l.  Per class, the 16
 * cells with all four genotypes in {0, 1} are counted on the matrix cores
 * (0/1 FP4 products, exact FP32 accumulation) when the data set has value
 * planes and classes of at most 65535 samples, else by AND + POPCNT over the
 * bit planes (a data set encoded with EPI3_ENCODE_BITS_ONLY); the corner
 * cells of the four sub-triplets are counted by AND + POPCNT once per
 * triplet, and every other cell follows by inclusion-exclusion from those,
 * the pairwise tables of epi3_encode and the class size.  Both count paths
 * give the same FP32 scores.  Hits are the k lowest under
 * (K2, i, j, k, l) with the same FP32 screen and FP64 re-score as the other
 * orders.  The score plane holds C(M,4) floats, so M is limited by memory
 * (M = 256: 0.7 GB; M = 512: 11 GB); M > 4096 is EPI3_E_UNSUPPORTED.
 * ------------------------------------------------------------------------ */

/* One hit of a quad scan.  counts[c][27 g_i + 9 g_j + 3 g_k + g_l]. */
typedef struct {
    uint32_t i, j, k, l;
    float k2_f32;         /* FP32 screen value */
    uint32_t reserved;
    double k2;            /* FP64 value of Eq. 1 over the 81 rows, in row order */
    uint32_t counts[2][81];
} epi3_quad_hit;

/* Number of quads C(M,4). */
int64_t epi3_n_quads(int32_t n_snps);

/* Upper bound on |K2_fp32 - K2_fp64| of an 81-row table of N samples. */
double epi3_k2_error_bound_quads(int32_t n_samples);

/* Workspace bytes for epi3_scan_quads + epi3_quads_topk (cand_cap as for
 * epi3_workspace_bytes).  EPI3_E_UNSUPPORTED for a MASKED data set or
 * M > 4096. */
int64_t epi3_quads_workspace_bytes(const epi3_dataset *d, int32_t k, int64_t cand_cap);

/* Count and score every quad (FP32) and select candidates; asynchronous.
 * ws_dev: 256-byte aligned device workspace of epi3_quads_workspace_bytes
 * bytes. */
int epi3_scan_quads(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                    int64_t ws_bytes, void *stream);

/* Copy min(k, C(M,4)) hits to hits_host [k]; *n_out receives the count.
 * Synchronises `stream`; EPI3_E_CAPACITY as for epi3_topk. */
int epi3_quads_topk(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                    epi3_quad_hit *hits_host, int32_t *n_out, void *stream);

/* Device address of the quad scan's FP32 score plane (lexicographic
 * (i, j, k, l) order, C(M,4) floats), valid once the stream has run
 * epi3_scan_quads. */
int epi3_quads_score_plane(const epi3_dataset *d, int32_t k, int64_t cand_cap, void *ws_dev,
                           float **plane_dev);

/* ---------------------------------------------------------------------------
 * Test hooks.
 * ------------------------------------------------------------------------ */

/* Run the count kernel of `variant` over every triplet of a SPLIT data set and
 * write each triplet's table and FP32 K2 in lexicographic (i, j, k) order:
 * counts_dev [C(M,3)][2][27] uint32 (may be NULL), k2_dev [C(M,3)] float.
 * ws_dev: a workspace of epi3_workspace_bytes(d, 1, variant, 0) bytes.  Asynchronous. */
int epi3_scan_tables(const epi3_dataset *d, int32_t variant, uint32_t *counts_dev,
                     float *k2_dev, void *ws_dev, int64_t ws_bytes, void *stream);

/* Tables and K2 of explicit triplets: ijk_dev [n][3] uint32 (i < j < k),
 * counts_dev [n][2][27] (may be NULL), k2_f32_dev [n], k2_dev [n] (FP64).
 * Asynchronous. */
int epi3_score_triplets(const epi3_dataset *d, const uint32_t *ijk_dev, int64_t n,
                        uint32_t *counts_dev, float *k2_f32_dev, double *k2_dev, void *stream);

/* Upper bound e(N) on |K2_fp32 - K2_fp64| used by the candidate screen. */
double epi3_k2_error_bound(int32_t n_samples);

/* Number of triplets C(M,3). */
int64_t epi3_n_triplets(int32_t n_snps);

/* Optional set-up on the current device: creates the library's second
 * stream and events of the matrix-core paths and the stream batched scans
 * are captured on, and looks up the device address of the static workspace
 * of epi3_scan_topk_static, which the first call that needs them would
 * otherwise do.  Returns EPI3_E_HIP if the runtime refuses. */
int epi3_init(void);

/* Release cached graphs and the library's idle streams and events.  Must not
 * run while another call of the library is in progress. */
void epi3_release(void);

/* Kernel timing for measurement: while enabled, the library records a HIP
 * event pair on the call's stream around each launch of the count stage
 * (which = 0), of the selection pipeline (which = 1), of a whole batched
 * scan (which = 2), of the table-completion/scoring kernel that follows the
 * matrix-core count of phenotype batches and of quad scans (which = 3) and of the pairwise-table
 * kernel of epi3_encode (which = 4); batched scans run without graph capture while timing is
 * enabled so that their kernels can be timed.  epi3_timing_query waits for the
 * recorded events and returns the summed milliseconds and the number of
 * launches since the last reset.  Off by default. */
void epi3_timing_enable(int enable);
int epi3_timing_query(int32_t which, double *ms, int64_t *launches);
void epi3_timing_reset(void);

/* ---------------------------------------------------------------------------
 * Tile shapes (autotuning).  Not in the paper, whose kernels fix one tile.
 * A rule applies to data sets with n_snps >= min_snps and n_samples >=
 * min_samples; among the rules of a variant that apply, the one with the
 * largest (min_snps, min_samples) wins, else the built-in default.
 *   EPI3_VARIANT_VALU: tile = pivot pairs per lane tile, 4 or 8.
 *   EPI3_VARIANT_MFMA, EPI3_VARIANT_MFMA_FP4 (plain scans): tile = JB, the
 *     pivots j per workgroup tile of 16 i x JB j x 256 / JB k: 2, 4 or 8.
 *   EPI3_VARIANT_AUTO: tile = the variant that AUTO selects for plain scans
 *     (EPI3_VARIANT_VALU, _MFMA or _MFMA_FP4; a matrix-core choice falls back
 *     to VALU for data sets it does not support).
 * Rules are process-wide; change them only between scans and size each
 * workspace after the change (the matrix-core scratch depends on the tile).
 * Returns EPI3_E_INVALID for an unknown variant or tile.
 * ------------------------------------------------------------------------ */
int epi3_tile_rule(int32_t variant, int32_t min_snps, int32_t min_samples, int32_t tile);
void epi3_tile_rules_clear(void);
/* The tile (or, for AUTO, the variant) a scan of d with `variant` uses. */
int32_t epi3_tile_for(const epi3_dataset *d, int32_t variant);
/* Scratch bytes per pass buffer of the matrix-core paths (0: default 1 GiB
 * for plain scans, 4 GiB for phenotype batches, 2 GiB for quad scans; each
 * path keeps two buffers).  Same rules as above. */
int epi3_set_pass_bytes(int64_t bytes);
/* Entries of the compacted low end of a score plane that the selection keeps
 * after its first histogram pass (0: default max(65536, 16 x candidate
 * capacity)); beyond it the later passes read the whole plane again.  Same
 * rules as above (it sizes the workspaces). */
int epi3_set_compact_cap(int64_t n);

/* How phenotype batches (MASKED jobs) find each job's k lowest, process-wide
 * (same rules as epi3_set_pass_bytes; it sizes the workspaces):
 *   PLANE    every FP32 score is written to a score plane per job (C(M,3)
 *            floats each) and the selection reads it;
 *   BOUNDED  no plane: every sample_stride-th tile of the batch is scored
 *            first, the k-th smallest score of that sample plus 2 e(N) bounds
 *            the FP32 score of every member of the exact top-k (the sample's
 *            k lowest are k real scores), and the full pass appends only the
 *            scores under that bound to a short list per job, which the
 *            selection then reads.  Workspace grows with k, not C(M,3);
 *            epi3_batched_score_plane returns EPI3_E_UNSUPPORTED.  A list that
 *            overflows ends the job with EPI3_E_CAPACITY (n_out = -(the
 *            cand_cap to retry with));
 *   AUTO     (default) BOUNDED for batches of at least 2^22 triplets.
 * EPI3_E_INVALID for another value. */
enum { EPI3_BATCH_SELECT_AUTO = 0, EPI3_BATCH_SELECT_PLANE = 1, EPI3_BATCH_SELECT_BOUNDED = 2 };
int epi3_set_batch_select(int32_t mode);

/* The same choice for plain scans (epi3_scan), process-wide (same rules as
 * epi3_set_pass_bytes; it sizes the workspaces):
 *   PLANE    every FP32 score goes to the score plane (4 C(M,3) bytes);
 *   BOUNDED  no plane (matrix-core variants): every sample_stride-th tile
 *            (about max(1024, 8 k) tiles of 4096 triplets) is scored first,
 *            the sample's k-th smallest score plus 2 e(N) bounds the FP32
 *            score of every member of the exact top-k, and the full pass
 *            appends only the scores under that bound to a list of
 *            max(16 cand_cap, 2 k sample_stride + 65536) entries.  The
 *            workspace no longer grows with C(M,3), so one GPU scans data
 *            sets whose plane would not fit in its memory;
 *   AUTO     (default) BOUNDED when the plane would take more than 16 GiB
 *            (beyond about 2900 SNPs) and the data set has value planes for
 *            the matrix cores; a vector-ALU scan of such a data set then
 *            returns EPI3_E_UNSUPPORTED unless PLANE is set.
 * EPI3_E_INVALID for another value. */
enum { EPI3_SCAN_SELECT_AUTO = 0, EPI3_SCAN_SELECT_PLANE = 1, EPI3_SCAN_SELECT_BOUNDED = 2 };
int epi3_set_scan_select(int32_t mode);

/* Library version string. */
const char *epi3_version(void);

#ifdef __cplusplus
}
#endif
#endif /* EPI3_H */
