/*
 * md_oracle.c -- TEST INFRASTRUCTURE ONLY (see md_oracle.h).
 *
 * The method (domain-case lowering plus typecasting while packing) reaches the
 * plain mathematical definition of the product exactly, up to rounding, so this
 * file is that definition written out, with no blocking, packing or reordering:
 *
 *   1. every stored element is promoted exactly to complex double (a real
 *      operand has imaginary part 0; float -> double is exact);
 *   2. op(X) is X, X^T, X^H (Section 1, the nine BLAS variants) or conj(X),
 *      the conjugation without transposition of the paper's hypothetical
 *      API (Section 3); an element (r, c) of a stored operand lies at
 *      r * rstride + c * cstride elements from its origin, the row and
 *      column strides of that API (column-major: rstride 1, cstride = ld);
 *   3. for every (i, j) the sum over p runs in ascending order with the
 *      complex product written out in real arithmetic;
 *   4. the scalars follow Section 7: alpha is used as given (a complex alpha
 *      with a non-zero imaginary part is refused in the six mixed cases of
 *      Section 7.2, except by md_oracle_gemm_literal, which computes those
 *      cases under the literal interpretation Section 7.2 describes, all
 *      five operands taken in their own domains; in case 0 the product is
 *      real so Re(alpha*AB) equals Re(alpha)*AB, the projection the paper
 *      describes); beta is reduced to Re(beta) when C is real (Section 7.2);
 *   5. a real C keeps Re of the result.  Figure "mixeddom"'s interpretations
 *      (A Re(B), Re(A) B, Re(AB), AB into Re(C), complex products with an
 *      implicit zero imaginary part) are all what steps 1-5 give.
 *
 * The result is returned in FP64 without rounding to C's storage type.
 * Quick-return conventions (the paper is silent; BLAS usage): alpha == 0 or
 * k == 0 means A and B are not read; beta == 0 means C is not read.
 */
#include "md_oracle.h"
#include <math.h>
#include <stddef.h>

/* storage tags */
#define T_S 0
#define T_D 1
#define T_C 2
#define T_Z 3
#define T_H 4   /* IEEE 754 binary16 */
#define T_HC 5  /* complex binary16, interleaved re, im */

static int tag_ok(int dt) { return dt >= T_S && dt <= T_HC; }
static int tag_complex(int dt) { return dt == T_C || dt == T_Z || dt == T_HC; }

/* The value of a binary16 bit pattern (1 sign, 5 exponent bits biased by 15,
 * 10 fraction bits; exponent 0 = subnormal, 31 = infinity or NaN), exactly in
 * double: the additional precision the paper's Section 5 discussion leaves
 * room for. */
static double half_value(uint16_t h)
{
    int sign = h >> 15, e = (h >> 10) & 31, f = h & 1023;
    double v;
    if (e == 0)
        v = ldexp((double)f, -24);
    else if (e == 31)
        v = f ? NAN : INFINITY;
    else
        v = ldexp((double)(1024 + f), e - 25);
    return sign ? -v : v;
}

/* Promote stored element (r, c) exactly to (re, im); (rs, cs) are the row and
 * column strides in elements of the operand's own type. */
static void fetch(const void *X, int dt, int64_t rs, int64_t cs, int64_t r, int64_t c,
                  double *re, double *im)
{
    int64_t idx = r * rs + c * cs;
    if (dt == T_S) {
        *re = (double)((const float *)X)[idx];
        *im = 0.0;
    } else if (dt == T_D) {
        *re = ((const double *)X)[idx];
        *im = 0.0;
    } else if (dt == T_C) {
        *re = (double)((const float *)X)[2 * idx];
        *im = (double)((const float *)X)[2 * idx + 1];
    } else if (dt == T_H) {
        *re = half_value(((const uint16_t *)X)[idx]);
        *im = 0.0;
    } else if (dt == T_HC) {
        *re = half_value(((const uint16_t *)X)[2 * idx]);
        *im = half_value(((const uint16_t *)X)[2 * idx + 1]);
    } else {
        *re = ((const double *)X)[2 * idx];
        *im = ((const double *)X)[2 * idx + 1];
    }
}

/* Element (i, p) of op(X): 'N' -> X(i,p); 'R' -> conj(X(i,p));
 * 'T' -> X(p,i); 'C' -> conj(X(p,i)). */
static void fetch_op(char tr, const void *X, int dt, int64_t rs, int64_t cs, int64_t i, int64_t p,
                     double *re, double *im)
{
    if (tr == 'N' || tr == 'R')
        fetch(X, dt, rs, cs, i, p, re, im);
    else
        fetch(X, dt, rs, cs, p, i, re, im);
    if (tr == 'C' || tr == 'R')
        *im = -*im;
}

static char norm_trans(char t)
{
    if (t == 'n') return 'N';
    if (t == 't') return 'T';
    if (t == 'c') return 'C';
    if (t == 'r') return 'R';
    return t;
}

static int trans_ok(char t) { return t == 'N' || t == 'T' || t == 'C' || t == 'R'; }

int md_oracle_case(int dtc, int dta, int dtb)
{
    /* Figure "mixeddom" rows, in order: (C,A,B) domains
     * RRR=0  RRC=1b  RCR=1a  RCC=2ab  CRR=1c  CRC=2bc  CCR=2ac  CCC=3 */
    return (tag_complex(dtc) ? 4 : 0) | (tag_complex(dta) ? 2 : 0) | (tag_complex(dtb) ? 1 : 0);
}

double md_oracle_flops(int dtc, int dta, int dtb, int64_t m, int64_t n, int64_t k)
{
    /* Figure "mixeddom": 0,1a,1b,1c -> 2mnk; 2ab,2ac,2bc -> 4mnk; 3 -> 8mnk. */
    int ncomplex = tag_complex(dtc) + tag_complex(dta) + tag_complex(dtb);
    double f = (ncomplex <= 1) ? 2.0 : (ncomplex == 2 ? 4.0 : 8.0);
    return f * (double)m * (double)n * (double)k;
}

/* Validate arguments as a plain BLAS-style routine would. */
static int check_args(char ta, char tb, int64_t m, int64_t n, int64_t k,
                      int dta, int64_t lda, int dtb, int64_t ldb, int dtc, int64_t ldc)
{
    if (!trans_ok(ta) || !trans_ok(tb)) return ORACLE_ERR_ARG;
    if (m < 0 || n < 0 || k < 0) return ORACLE_ERR_ARG;
    if (!tag_ok(dta) || !tag_ok(dtb) || !tag_ok(dtc)) return ORACLE_ERR_ARG;
    int64_t arows = (ta == 'N' || ta == 'R') ? m : k;
    int64_t brows = (tb == 'N' || tb == 'R') ? k : n;
    if (lda < (arows > 1 ? arows : 1)) return ORACLE_ERR_ARG;
    if (ldb < (brows > 1 ? brows : 1)) return ORACLE_ERR_ARG;
    if (ldc < (m > 1 ? m : 1)) return ORACLE_ERR_ARG;
    return ORACLE_OK;
}

/* Section 7.2: a non-zero Im(alpha) is refused in cases 1a,1b,1c,2ab,2ac,2bc. */
static int alpha_refused(int dtc, int dta, int dtb, double alpha_im)
{
    int cs = md_oracle_case(dtc, dta, dtb);
    return alpha_im != 0.0 && cs != 0 && cs != 7;
}

/* One entry of the result: the definition, for C(i, j). */
static void entry(char ta, char tb, int64_t k,
                  double alpha_re, double alpha_im,
                  const void *A, int dta, int64_t rsa, int64_t csa,
                  const void *B, int dtb, int64_t rsb, int64_t csb,
                  double beta_re, double beta_im,
                  const void *C, int dtc, int64_t rsc, int64_t csc,
                  int64_t i, int64_t j, double *out_re, double *out_im, double *out_g)
{
    double sr = 0.0, si = 0.0, g = 0.0;
    /* Section 7.2: in case 0 a complex alpha is projected onto the real domain */
    if (md_oracle_case(dtc, dta, dtb) == 0)
        alpha_im = 0.0;
    int use_ab = (k > 0) && (alpha_re != 0.0 || alpha_im != 0.0);
    if (use_ab) {
        for (int64_t p = 0; p < k; ++p) {
            double ar, ai, br, bi;
            fetch_op(ta, A, dta, rsa, csa, i, p, &ar, &ai);
            fetch_op(tb, B, dtb, rsb, csb, p, j, &br, &bi);
            sr += ar * br - ai * bi;
            si += ar * bi + ai * br;
            g += sqrt(ar * ar + ai * ai) * sqrt(br * br + bi * bi);
        }
    }
    /* t = alpha * (sr + i si) */
    double tr = use_ab ? alpha_re * sr - alpha_im * si : 0.0;
    double ti = use_ab ? alpha_re * si + alpha_im * sr : 0.0;

    /* beta: only its real part matters for a real C */
    double bre = beta_re;
    double bim = tag_complex(dtc) ? beta_im : 0.0;
    double rr = tr, ri = ti;
    if (bre != 0.0 || bim != 0.0) {
        double cr, ci;
        fetch(C, dtc, rsc, csc, i, j, &cr, &ci);
        rr = bre * cr - bim * ci + tr;
        ri = bre * ci + bim * cr + ti;
    }
    *out_re = rr;
    *out_im = tag_complex(dtc) ? ri : 0.0; /* a real C keeps only Re */
    if (out_g) *out_g = g;
}

static int gemm_colmajor(char transa, char transb, int64_t m, int64_t n, int64_t k,
                         double alpha_re, double alpha_im,
                         const void *A, int dta, int64_t lda,
                         const void *B, int dtb, int64_t ldb,
                         double beta_re, double beta_im,
                         const void *C, int dtc, int64_t ldc,
                         double *cref, double *g, int literal)
{
    char ta = norm_trans(transa), tb = norm_trans(transb);
    int st = check_args(ta, tb, m, n, k, dta, lda, dtb, ldb, dtc, ldc);
    if (st != ORACLE_OK) return st;
    if (!literal && alpha_refused(dtc, dta, dtb, alpha_im)) return ORACLE_ERR_ALPHA_IMAG;
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            int64_t o = i + j * m;
            entry(ta, tb, k, alpha_re, alpha_im, A, dta, 1, lda, B, dtb, 1, ldb,
                  beta_re, beta_im, C, dtc, 1, ldc, i, j,
                  &cref[2 * o], &cref[2 * o + 1], g ? &g[o] : NULL);
        }
    }
    return ORACLE_OK;
}

int md_oracle_gemm(char transa, char transb, int64_t m, int64_t n, int64_t k,
                   double alpha_re, double alpha_im,
                   const void *A, int dta, int64_t lda,
                   const void *B, int dtb, int64_t ldb,
                   double beta_re, double beta_im,
                   const void *C, int dtc, int64_t ldc,
                   double *cref, double *g)
{
    return gemm_colmajor(transa, transb, m, n, k, alpha_re, alpha_im, A, dta, lda, B, dtb, ldb,
                         beta_re, beta_im, C, dtc, ldc, cref, g, 0);
}

int md_oracle_gemm_literal(char transa, char transb, int64_t m, int64_t n, int64_t k,
                           double alpha_re, double alpha_im,
                           const void *A, int dta, int64_t lda,
                           const void *B, int dtb, int64_t ldb,
                           double beta_re, double beta_im,
                           const void *C, int dtc, int64_t ldc,
                           double *cref, double *g)
{
    return gemm_colmajor(transa, transb, m, n, k, alpha_re, alpha_im, A, dta, lda, B, dtb, ldb,
                         beta_re, beta_im, C, dtc, ldc, cref, g, 1);
}

int md_oracle_gemm_at(char transa, char transb, int64_t m, int64_t n, int64_t k,
                      double alpha_re, double alpha_im,
                      const void *A, int dta, int64_t lda,
                      const void *B, int dtb, int64_t ldb,
                      double beta_re, double beta_im,
                      const void *C, int dtc, int64_t ldc,
                      int64_t count, const int64_t *rows, const int64_t *cols,
                      double *cref, double *g)
{
    char ta = norm_trans(transa), tb = norm_trans(transb);
    int st = check_args(ta, tb, m, n, k, dta, lda, dtb, ldb, dtc, ldc);
    if (st != ORACLE_OK) return st;
    if (alpha_refused(dtc, dta, dtb, alpha_im)) return ORACLE_ERR_ALPHA_IMAG;
    for (int64_t t = 0; t < count; ++t) {
        if (rows[t] < 0 || rows[t] >= m || cols[t] < 0 || cols[t] >= n) return ORACLE_ERR_ARG;
        entry(ta, tb, k, alpha_re, alpha_im, A, dta, 1, lda, B, dtb, 1, ldb,
              beta_re, beta_im, C, dtc, 1, ldc, rows[t], cols[t],
              &cref[2 * t], &cref[2 * t + 1], g ? &g[t] : NULL);
    }
    return ORACLE_OK;
}

int md_oracle_gemm_gs(char transa, char transb, int64_t m, int64_t n, int64_t k,
                      double alpha_re, double alpha_im,
                      const void *A, int dta, int64_t rsa, int64_t csa,
                      const void *B, int dtb, int64_t rsb, int64_t csb,
                      double beta_re, double beta_im,
                      const void *C, int dtc, int64_t rsc, int64_t csc,
                      double *cref, double *g)
{
    char ta = norm_trans(transa), tb = norm_trans(transb);
    if (!trans_ok(ta) || !trans_ok(tb)) return ORACLE_ERR_ARG;
    if (m < 0 || n < 0 || k < 0) return ORACLE_ERR_ARG;
    if (!tag_ok(dta) || !tag_ok(dtb) || !tag_ok(dtc)) return ORACLE_ERR_ARG;
    if (rsa < 1 || csa < 1 || rsb < 1 || csb < 1 || rsc < 1 || csc < 1) return ORACLE_ERR_ARG;
    if (alpha_refused(dtc, dta, dtb, alpha_im)) return ORACLE_ERR_ALPHA_IMAG;
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            int64_t o = i + j * m;
            entry(ta, tb, k, alpha_re, alpha_im, A, dta, rsa, csa, B, dtb, rsb, csb,
                  beta_re, beta_im, C, dtc, rsc, csc, i, j,
                  &cref[2 * o], &cref[2 * o + 1], g ? &g[o] : NULL);
        }
    }
    return ORACLE_OK;
}
