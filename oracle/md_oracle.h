/*
 * md_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow CPU reference for mixed-datatype matrix multiplication
 *     C := beta*C + alpha*op(A)*op(B)
 * as stated in Van Zee, Parikh, van de Geijn, "Supporting mixed-datatype matrix
 * multiplication within the BLIS framework" (Section 1 for the operation and the
 * op() variants; Section 4.2 / Figure "mixeddom" for the eight domain cases;
 * Section 5 for precision; Section 7 for the scalar policies).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * call this.  It shares no code, header, table or helper with the GPU library.
 *
 * Storage tags: 0 = s (float), 1 = d (double), 2 = c (float complex,
 * interleaved re,im), 3 = z (double complex, interleaved), 4 = h (IEEE
 * binary16), 5 = hc (binary16 complex, interleaved): the half precision the
 * paper's Section 5 summary names as the next storage precision.  Matrices are
 * column-major unless strides are given (md_oracle_gemm_gs); a leading
 * dimension or stride counts elements of the operand's own type.  Trans
 * letters: N, T, C (the BLAS) and R (conjugate without transposing).
 */
#ifndef MD_ORACLE_H
#define MD_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_OK 0
#define ORACLE_ERR_ALPHA_IMAG 1   /* Section 7.2: Im(alpha) != 0 in cases 1a,1b,1c,2ab,2ac,2bc */
#define ORACLE_ERR_ARG (-1)       /* malformed arguments (trans letter, dims, tags, ld) */

/* Domain case of Figure "mixeddom", encoded 0..7 as
 * 0:"0" 1:"1b" 2:"1a" 3:"2ab" 4:"1c" 5:"2bc" 6:"2ac" 7:"3"
 * (the figure's row order). */
int md_oracle_case(int dtc, int dta, int dtb);

/* Minimum flop count of the case, Figure "mixeddom": 2mnk, 4mnk or 8mnk. */
double md_oracle_flops(int dtc, int dta, int dtb, int64_t m, int64_t n, int64_t k);

/*
 * Full reference.  Writes, for every 0<=i<m, 0<=j<n,
 *   cref[2*(i+j*m)], cref[2*(i+j*m)+1] : the exact-input FP64 result (re, im);
 *                                         im is 0 when C is real-stored
 *   g[i+j*m] (if g != NULL)            : sum_p |op(A)_ip| * |op(B)_pj|
 *                                         (complex modulus), the bound term.
 * C itself is read, never written.  Returns ORACLE_OK, ORACLE_ERR_ALPHA_IMAG
 * (cref untouched) or ORACLE_ERR_ARG.
 */
int md_oracle_gemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
                   double alpha_re, double alpha_im,
                   const void *A, int dta, int64_t lda,
                   const void *B, int dtb, int64_t ldb,
                   double beta_re, double beta_im,
                   const void *C, int dtc, int64_t ldc,
                   double *cref, double *g);

/* The same under the literal interpretation of Section 7.2: a complex alpha
 * is applied as given in every case, so the six mixed cases accept
 * Im(alpha) != 0 (never returns ORACLE_ERR_ALPHA_IMAG). */
int md_oracle_gemm_literal(char transa, char transb, int64_t m, int64_t n, int64_t k,
                           double alpha_re, double alpha_im,
                           const void *A, int dta, int64_t lda,
                           const void *B, int dtb, int64_t ldb,
                           double beta_re, double beta_im,
                           const void *C, int dtc, int64_t ldc,
                           double *cref, double *g);

/* The same definition evaluated only at `count` entries (rows[t], cols[t]);
 * cref has 2*count doubles, g (optional) count doubles. */
int md_oracle_gemm_at(char transa, char transb, int64_t m, int64_t n, int64_t k,
                      double alpha_re, double alpha_im,
                      const void *A, int dta, int64_t lda,
                      const void *B, int dtb, int64_t ldb,
                      double beta_re, double beta_im,
                      const void *C, int dtc, int64_t ldc,
                      int64_t count, const int64_t *rows, const int64_t *cols,
                      double *cref, double *g);

/* The same definition with every operand addressed by its row and column
 * strides (element (r, c) at r*rs + c*cs elements; the hypothetical API of
 * Section 3: column-major, row-major or general storage), and trans letters
 * N, T, C or R (conjugate without transposing).  cref and g are column-major
 * m x n as in md_oracle_gemm.  Strides must be positive. */
int md_oracle_gemm_gs(char transa, char transb, int64_t m, int64_t n, int64_t k,
                      double alpha_re, double alpha_im,
                      const void *A, int dta, int64_t rsa, int64_t csa,
                      const void *B, int dtb, int64_t rsb, int64_t csb,
                      double beta_re, double beta_im,
                      const void *C, int dtc, int64_t rsc, int64_t csc,
                      double *cref, double *g);

#ifdef __cplusplus
}
#endif
#endif
