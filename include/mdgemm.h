/*
 * mdgemm.h -- mixed-datatype general matrix multiplication on MI355X (gfx950).
 *
 *     C := beta*C + alpha*op(A)*op(B)
 *
 * where each of A, B and C is independently stored as single or double
 * precision, real or complex (s, d, c, z; and binary16 h, hc, an addition)
 * and the computation precision is chosen separately from the storage
 * precisions.  The operation and the three op() variants are those of the
 * BLAS gemm (Van Zee, Parikh, van de Geijn, "Supporting mixed-datatype matrix
 * multiplication within the BLIS framework", Section 1), plus conjugation
 * without transposition ('R', Section 3); the domain of the computation
 * follows from which operands are complex (Section 4.2, Figure "mixeddom");
 * the computation precision and the target types of A and B follow Section
 * 5.1; the scalar policies follow Section 7.
 *
 * Storage conventions (all entry points but mdgemm_strided, which takes row
 * and column strides):
 *   - matrices are column-major; complex elements are interleaved (re, im);
 *   - a leading dimension counts elements of that operand's own type and must
 *     be >= max(1, rows) of the stored matrix (rows of A are m for transa 'N'
 *     or 'R', else k; rows of B are k for transb 'N' or 'R', else n; rows of
 *     C are m);
 *   - A, B and C are device pointers owned by the caller; A and B are only
 *     read; C is updated in place and must not overlap A or B (A may equal B);
 *   - work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *     the call returns before it completes: the caller keeps every buffer alive
 *     until the stream has finished;
 *   - on any error return nothing is enqueued and C is unmodified;
 *   - device memory: a product with few output tiles (fewer than half the
 *     CUs) and a deep k splits k over workgroups and keeps their partial
 *     products in a workspace of the library, one per (device, stream):
 *     allocated with hipMallocAsync on that stream when first needed, grown
 *     on demand (the old buffer freed in stream order) and kept until the
 *     process ends, at most about 100 MB per stream.  A BF16x3 product large
 *     enough to fill the GPU with 256 x 256 tiles of its real product (at
 *     least 128 of them and k' >= 256) runs on operands cast, split into
 *     bf16 planes and packed once per call, in a second workspace of the
 *     same kind: 4 bytes per element of the real product's padded A' and B'
 *     (about 0.8 GB for m = n = k = 8192 in case 2ac), at most 8 GiB; when
 *     it cannot be had the product runs unpacked.  Calls on one stream may
 *     come from several host threads.  With MDGEMM_SPLITK=0 and
 *     MDGEMM_PACK=0 in the environment products are never split or packed
 *     and mdgemm allocates no device memory (MDGEMM_PACK=2 packs every
 *     qualifying BF16x3 product whatever its size).
 *
 * Return codes: 0 on success; -i when argument i (1-based, in mdgemm's order)
 * is invalid; positive MD_ERR_* codes otherwise (see mdgemm_strerror).
 */
#ifndef MDGEMM_H
#define MDGEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage type of one operand (domain x precision, Section 1's s/d/c/z). */
typedef enum {
    MD_S = 0, MD_D = 1, MD_C = 2, MD_Z = 3,
    /* Half precision, the next storage precision Section 5's summary names
     * (an addition of this library): IEEE 754 binary16 (MD_H) and complex
     * binary16 with interleaved re, im (MD_HC).  A half C is written by every
     * kernel; binary16 A and B together run on the fast loads under the
     * single and half precisions (each stored column a whole number of
     * 4-byte words), any other binary16 operand on the component-wise loads. */
    MD_H = 4, MD_HC = 5
} md_dt;

/* Computation precision (Section 5.1.1).  MD_COMP_DEFAULT selects the storage
 * precision of C.  MD_COMP_S_BF16X3 has single-precision semantics but forms
 * each real product from bfloat16 halves (hi*hi + hi*lo + lo*hi) on the
 * bf16 matrix cores with FP32 accumulation; it is an addition of this
 * library, not of the paper. */
typedef enum {
    MD_COMP_DEFAULT = -1,
    MD_COMP_S = 0,
    MD_COMP_D = 1,
    MD_COMP_S_BF16X3 = 2,
    /* Half computation precision (an addition of this library): each
     * element of A and B is rounded to binary16 (nearest even) as it is
     * staged and the products run on the fp16 matrix cores with FP32
     * accumulation; alpha, beta and the update follow the single rules.  The
     * default for a half-precision C. */
    MD_COMP_H = 3,
    /* Flag, OR'ed into MD_COMP_S, MD_COMP_D or MD_COMP_S_BF16X3 (not into
     * MD_COMP_DEFAULT): a complex alpha is applied as given in the six mixed
     * cases too, under the literal interpretation Section 7.2 describes (all
     * five operands in their own domains), instead of being refused.  With C
     * real (cases 1a, 1b, 2ab) alpha is folded into the complex operand as it
     * is staged (Re(alpha*A), Re(alpha*B), alpha*A: the packing the paper
     * suggests in a footnote to Section 7.2), so the flop count stays the
     * case's minimum; with C complex (1c, 2ac, 2bc) the epilogue multiplies
     * by the complex alpha.  An extension of the paper's policy. */
    MD_COMP_LITERAL_ALPHA = 0x100
} md_comp;

/* alpha and beta are always passed as complex double; see Section 7 for how
 * each case uses them. */
typedef struct { double re, im; } md_scalar;

/* Domain cases of Figure "mixeddom" (C, A, B domains). */
typedef enum {
    MD_CASE_0 = 0,   /* R R R : C += AB                       2mnk */
    MD_CASE_1A = 1,  /* R C R : C += Re(A) B                  2mnk */
    MD_CASE_1B = 2,  /* R R C : C += A Re(B)                  2mnk */
    MD_CASE_1C = 3,  /* C R R : Re(C) += AB                   2mnk */
    MD_CASE_2AB = 4, /* R C C : C += Re(AB)                   4mnk */
    MD_CASE_2AC = 5, /* C C R : C += AB, Im(B) = 0 skipped    4mnk */
    MD_CASE_2BC = 6, /* C R C : C += AB, Im(A) = 0 skipped    4mnk */
    MD_CASE_3 = 7    /* C C C : C += AB                       8mnk */
} md_case;

/* Status codes. */
#define MD_OK 0
#define MD_ERR_ALPHA_IMAG 1  /* Im(alpha) != 0 in case 1a, 1b, 1c, 2ab, 2ac or 2bc (Section 7.2) */
#define MD_ERR_HIP 2         /* HIP launch or runtime failure */
#define MD_ERR_BUDGET 3      /* a serving request exceeds the memory budget */
#define MD_ERR_STATE 4       /* call not valid in the object's current state */
#define MD_ERR_UNSUPPORTED 5 /* valid request that this build cannot run */
#define MD_ERR_SCRATCH 6     /* mdgemm_grouped_noalloc: work table larger than its fixed scratch */

/*
 * mdgemm -- one mixed-datatype product.
 *
 * Arguments (position in parentheses is the one reported as -i on error):
 *  (1) transa, (2) transb : 'N', 'T', 'C' (the BLAS) or 'R' (conjugate
 *        without transposing, the fourth value of the paper's hypothetical
 *        API, Section 3); lower case accepted.  On a real operand 'C' equals
 *        'T' and 'R' equals 'N'.
 *  (3) m, (4) n, (5) k     : op(A) is m x k, op(B) is k x n, C is m x n; >= 0.
 *  (6) alpha               : cast to the computation precision (Section 7.1,
 *        option 1).  Im(alpha) is ignored in case 0 and used in case 3; in the
 *        other six cases a non-zero Im(alpha) returns MD_ERR_ALPHA_IMAG unless
 *        comp carries MD_COMP_LITERAL_ALPHA.
 *  (7) A, (8) dta, (9) lda : operand A, its storage type, leading dimension.
 *  (10) B, (11) dtb, (12) ldb : operand B likewise.
 *  (13) beta               : cast to C's storage precision (Section 7.1,
 *        option 1); Im(beta) is ignored when C is real.  beta == 0 means C is
 *        not read (NaN in C does not propagate).
 *  (14) C, (15) dtc, (16) ldc : operand C likewise; updated in place.
 *  (17) comp               : computation precision (md_comp).
 *  (18) stream             : hipStream_t to enqueue on.
 *
 * The result is beta*C + alpha*op(A)*op(B) computed with the product in the
 * computation precision and the update in the wider of the computation and C
 * precisions, rounded once to C's storage type.  m == 0 or n == 0 is a
 * no-op; alpha == 0 or k == 0 only scales C by beta (A and B are not read).
 */
int mdgemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
           md_scalar alpha,
           const void *A, md_dt dta, int64_t lda,
           const void *B, md_dt dtb, int64_t ldb,
           md_scalar beta,
           void *C, md_dt dtc, int64_t ldc,
           md_comp comp, void *stream);

/*
 * mdgemm_strided -- the same product with every operand addressed by its row
 * and column strides (element (i, j) of a stored operand at i*rs + j*cs
 * elements of its type), the storage description of the paper's hypothetical
 * API (Section 3; Section 2.2.1 for BLIS's row and column strides).  Strides are
 * >= 1 and an operand's elements must not overlap: its columns lie apart
 * (cs >= rs*rows; column-major storage is rs == 1) or its rows do
 * (rs >= cs*cols; row-major storage is cs == 1); a stride along an extent of
 * one element is not used.  Each operand is laid out independently:
 *   - column-major and row-major operands run on the same kernels as mdgemm:
 *     a row-major operand is its transpose stored column-major (its op flips
 *     N <-> T, R <-> C), and a row-major C is computed as
 *     C^T = op(B)^T op(A)^T;
 *   - general storage (neither stride 1) takes the component-wise loads,
 *     which read each element where its strides put it (slower: no 16-byte
 *     chunks).
 * Results follow mdgemm's rules.  Argument positions for errors: (1) transa
 * (2) transb (3) m (4) n (5) k (6) alpha (7) A (8) dta (9) rsa (10) csa
 * (11) B (12) dtb (13) rsb (14) csb (15) beta (16) C (17) dtc (18) rsc
 * (19) csc (20) comp (21) stream; overlapping strides name the column stride
 * when rs <= cs, else the row stride.
 */
int mdgemm_strided(char transa, char transb, int64_t m, int64_t n, int64_t k, md_scalar alpha,
                   const void *A, md_dt dta, int64_t rsa, int64_t csa,
                   const void *B, md_dt dtb, int64_t rsb, int64_t csb,
                   md_scalar beta, void *C, md_dt dtc, int64_t rsc, int64_t csc,
                   md_comp comp, void *stream);

/* What mdgemm would do with the same arguments, computed on the host only
 * (no device call, usable without a GPU). */
typedef struct {
    int status;        /* the value mdgemm would return */
    int domain_case;   /* md_case */
    int comp;          /* resolved computation precision (MD_COMP_S/D/S_BF16X3) */
    int quick;         /* 0: full product; 1: nothing to do; 2: C := beta*C only */
    double flops;      /* algorithmic flops of Figure "mixeddom" (0 if quick) */
    int64_t m_real;    /* rows of the real product the case is lowered to */
    int64_t n_real;    /* columns of that real product */
    int64_t k_real;    /* inner dimension of that real product */
    int a_parts;       /* parts of A that reach C: 1 = real or Re only, 2 = Re and Im */
    int b_parts;       /* parts of B that reach C */
    int tile_m, tile_n, tile_k; /* workgroup tile of the real product */
    int64_t workgroups;         /* workgroups launched */
    char kernel[48];            /* kernel variant name */
} md_plan;

int mdgemm_plan(char transa, char transb, int64_t m, int64_t n, int64_t k,
                md_scalar alpha,
                const void *A, md_dt dta, int64_t lda,
                const void *B, md_dt dtb, int64_t ldb,
                md_scalar beta,
                void *C, md_dt dtc, int64_t ldc,
                md_comp comp, md_plan *out);

/*
 * Grouped form: `count` independent products enqueued as ONE persistent
 * kernel launch on `stream`.  Each descriptor holds exactly mdgemm's
 * arguments (1)-(17); products may differ in shape, storage types and
 * computation precision.  Every descriptor is validated first; if any is
 * invalid the call returns -(1000*index + i) for the first bad argument i of
 * descriptor `index` (or MD_ERR_ALPHA_IMAG) and enqueues nothing.  The C
 * operands must be pairwise disjoint and must not overlap any A or B.  The
 * work table (one entry per product and per output tile, largest work first)
 * is uploaded through page-locked staging into a device table that the
 * library keeps per (device, stream): allocated on first use, grown on
 * demand, kept until the process ends (the staging is reused once the
 * previous upload from it has been read; calls on one stream may come from
 * several host threads).  Products that take the plain kernels inside the
 * call (see mdgemm_grouped_noalloc) follow mdgemm's allocation rules.  The
 * tile shape of each product comes from the tile-shape table below.
 */
typedef struct {
    char transa, transb;
    int64_t m, n, k;
    md_scalar alpha;
    const void *A; md_dt dta; int64_t lda;
    const void *B; md_dt dtb; int64_t ldb;
    md_scalar beta;
    void *C; md_dt dtc; int64_t ldc;
    md_comp comp;
} md_gemm_desc;

int mdgemm_grouped(int64_t count, const md_gemm_desc *descs, void *stream);

/*
 * mdgemm_grouped_noalloc -- mdgemm_grouped for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, validation, kernels and results,
 * except:
 *   - the work table (a 256-byte header holding the tile counter, one
 *     descriptor per product, 16 bytes per output tile) is uploaded into a
 *     fixed array of MD_GROUPED_NOALLOC_BYTES that the library holds on each
 *     GPU it runs on until the process ends, instead of a stream-ordered
 *     allocation; a table that does not fit returns MD_ERR_SCRATCH and
 *     enqueues nothing;
 *   - products that mdgemm_grouped hands to the plain kernels (large leading
 *     dimensions, binary16, a complex alpha staged into an operand) run
 *     unsplit and unpacked, so no split-k or packing workspace is taken.
 * It calls no hipMalloc, hipFree or other allocating routine (the host copy
 * of the table is ordinary host memory, consumed by the upload).  Every call
 * on one GPU shares that GPU's array, which keeps the last call's table:
 * calls on one stream from one host thread run in order, but calls that
 * overlap on one GPU (other streams, or host threads sharing a stream) race
 * on it -- serialise them.
 */
#define MD_GROUPED_NOALLOC_BYTES (8u << 20)
int mdgemm_grouped_noalloc(int64_t count, const md_gemm_desc *descs, void *stream);

/*
 * Tile configurations of the grouped kernel: the workgroup tile of the real
 * product (m' x n') and its k-tile depth (double / single computation
 * precision), each run by 8 waves.
 */
enum md_gtile {
    MD_GTILE_64x64 = 0,       /* 64 x 64, k-tile 16 / 32, 2 x 2 waves in two k-groups */
    MD_GTILE_128x128 = 1,     /* 128 x 128, k-tile 8 / 16, 2 x 4 waves */
    MD_GTILE_128x64 = 2,      /* 128 x 64, k-tile 16 / 32, 4 x 2 waves */
    MD_GTILE_64x128 = 3,      /* 64 x 128, k-tile 16 / 32, 2 x 4 waves */
    MD_GTILE_64x64_DEEPK = 4, /* 64 x 64, k-tile 32 / 64, 2 x 2 waves in two k-groups */
    MD_GTILE_COUNT = 5
};

/*
 * Tile table of the grouped kernel: for each computation precision (md_comp
 * S, D or S_BF16X3), domain case (md_case) and pair of size buckets of the
 * real product the case lowers to (m' and n' each: 0: <=64, 1: <=128,
 * 2: <=256, 3: <=512, 4: larger) the md_gtile configuration.  BF16x3 products
 * always use MD_GTILE_64x64.  Built-in default: per dimension, a 64-wide tile
 * up to bucket 2 and a 128-wide one above.  The autotuner measures the
 * configurations in context and writes a text table, one entry per line:
 * "comp case bucket_m bucket_n config" (comp s|d|bf16x3, case
 * 0|1a|1b|1c|2ab|2ac|2bc|3, config 64x64|128x128|128x64|64x128|64x64k), '#'
 * comments.
 *
 * mdgemm_tune_load: the built-in defaults with the entries of the file at
 *   `path` applied become the table (NULL: the defaults alone).  Returns 0,
 *   or MD_ERR_STATE with the table unchanged if the file is missing or
 *   malformed.
 * mdgemm_tune_set: set one entry to an md_gtile value; returns 0 or
 *   MD_ERR_STATE for an invalid entry.
 * mdgemm_tune_get: the md_gtile value of one entry, or -1 if invalid.
 * The table is process-wide and guarded by a lock.
 */
#define MD_TUNE_BUCKETS 5
int mdgemm_tune_load(const char *path);
int mdgemm_tune_set(int comp, int domain_case, int bucket_m, int bucket_n, int config);
int mdgemm_tune_get(int comp, int domain_case, int bucket_m, int bucket_n);

/* Human-readable text for a status code. */
const char *mdgemm_strerror(int status);

/* Library version string. */
const char *mdgemm_version(void);

#ifdef __cplusplus
}
#endif
#endif
