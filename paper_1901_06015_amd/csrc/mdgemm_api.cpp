// mdgemm_api.cpp -- the C ABI of libmdgemm: argument validation, domain-case
// classification (Figure "mixeddom"), the computation-precision and scalar
// policies (Sections 5.1 and 7), quick returns, and dispatch to the kernels.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "md_internal.h"

using namespace md;

namespace {

int norm_trans(char t) {
    switch (t) {
    case 'N': case 'n': return 0;
    case 'T': case 't': return 1;
    case 'C': case 'c': return 2;
    case 'R': case 'r': return 3;  // conjugate without transposing (Section 3's hypothetical API)
    }
    return -1;
}

bool dt_ok(int dt) { return dt >= MD_S && dt <= MD_HC; }

// A computation precision, optionally with MD_COMP_LITERAL_ALPHA OR'ed into an
// explicit one.
bool comp_ok(int comp) {
    if (comp == MD_COMP_DEFAULT) return true;
    if (comp < 0) return false;
    const int base = comp & ~MD_COMP_LITERAL_ALPHA;
    return base == MD_COMP_S || base == MD_COMP_D || base == MD_COMP_S_BF16X3 || base == MD_COMP_H;
}

// The op of an operand after swapping its row and column strides (its
// transpose): N <-> T, R <-> C.
char flip_op(char t) {
    switch (t) {
    case 'N': case 'n': return 'T';
    case 'T': case 't': return 'N';
    case 'C': case 'c': return 'R';
    case 'R': case 'r': return 'C';
    }
    return t;
}

// A stored rows x cols block with row stride rs and column stride cs (in
// elements), seen as a column-major matrix with leading dimension ld and
// element stride rs along its columns: the block itself, or its transpose
// (then the operand's op flips).  Its elements must not overlap, so either its
// columns lie apart (cs >= rs*rows) or its rows do (rs >= cs*cols); the view
// keeps columns (rows) as stored columns accordingly.  Returns 0, 1 (bad row
// stride) or 2 (bad column stride).
struct View {
    int64_t ld, rs;
    bool transposed;
};
int storage_view(int64_t rows, int64_t cols, int64_t rs, int64_t cs, View *v) {
    if (rs < 1) return 1;
    if (cs < 1) return 2;
    if (rows <= 1) {  // one row: cols elements at stride cs
        *v = View{cols > 1 ? cs : 1, 1, false};
        return 0;
    }
    if (cols <= 1) {  // one column: rows elements at stride rs, read as one stored row
        *v = View{rs, 1, true};
        return 0;
    }
    const bool cols_apart = cs / rows >= rs, rows_apart = rs / cols >= cs;
    if (cols_apart) *v = View{cs, rs, false};
    else if (rows_apart) *v = View{rs, cs, true};
    else return rs <= cs ? 2 : 1;
    return 0;
}
bool dt_cplx(int dt) { return dt == MD_C || dt == MD_Z || dt == MD_HC; }
bool dt_dbl(int dt) { return dt == MD_D || dt == MD_Z; }
bool dt_half(int dt) { return dt == MD_H || dt == MD_HC; }
// bytes of one stored element
int64_t dt_bytes(int dt) {
    return dt == MD_Z ? 16 : (dt == MD_D || dt == MD_C) ? 8 : dt == MD_S ? 4 : dt == MD_HC ? 4 : 2;
}
int64_t max1(int64_t v) { return v > 1 ? v : 1; }

}  // namespace

namespace {

}  // namespace

namespace md {

Decision decide(char transa, char transb, int64_t m, int64_t n, int64_t k, md_scalar alpha,
                const void *A, int dta, int64_t lda, const void *B, int dtb, int64_t ldb,
                md_scalar beta, void *C, int dtc, int64_t ldc, int comp,
                int64_t rsa, int64_t rsb, int64_t rsc) {
    Decision d;
    const int ta = norm_trans(transa), tb = norm_trans(transb);
    if (ta < 0) { d.status = -1; return d; }
    if (tb < 0) { d.status = -2; return d; }
    if (m < 0) { d.status = -3; return d; }
    if (n < 0) { d.status = -4; return d; }
    if (k < 0) { d.status = -5; return d; }
    const bool uses_ab = m > 0 && n > 0 && k > 0 && (alpha.re != 0.0 || alpha.im != 0.0);
    if (uses_ab && A == nullptr) { d.status = -7; return d; }
    if (!dt_ok(dta)) { d.status = -8; return d; }
    // a column of r elements at element stride rs spans rs*r elements
    if (lda / rsa < max1((ta == 0 || ta == 3) ? m : k)) { d.status = -9; return d; }
    if (uses_ab && B == nullptr) { d.status = -10; return d; }
    if (!dt_ok(dtb)) { d.status = -11; return d; }
    if (ldb / rsb < max1((tb == 0 || tb == 3) ? k : n)) { d.status = -12; return d; }
    if (m > 0 && n > 0 && C == nullptr) { d.status = -14; return d; }
    if (!dt_ok(dtc)) { d.status = -15; return d; }
    if (ldc / rsc < max1(m)) { d.status = -16; return d; }
    if (!comp_ok(comp)) { d.status = -17; return d; }
    const bool literal = comp != MD_COMP_DEFAULT && (comp & MD_COMP_LITERAL_ALPHA);
    if (literal) comp &= ~MD_COMP_LITERAL_ALPHA;

    // Section 5.1.1: the computation precision defaults to C's storage precision.
    if (comp == MD_COMP_DEFAULT) comp = dt_dbl(dtc) ? MD_COMP_D : (dt_half(dtc) ? MD_COMP_H : MD_COMP_S);
    d.prec = comp == MD_COMP_D ? PREC_D
           : comp == MD_COMP_S ? PREC_S
           : comp == MD_COMP_H ? PREC_H : PREC_BF16X3;
    d.cs = classify(dtc, dta, dtb);

    // Section 7.2: Im(alpha) is projected away in case 0, used in case 3 and
    // refused in the six mixed cases -- unless the caller asks for the literal
    // interpretation: then a complex C takes the complex alpha in the epilogue,
    // and for a real C the complex operand is staged as alpha times itself
    // (Re(alpha A) B, A Re(alpha B), Re((alpha A) B)) with the epilogue's alpha 1.
    double are = alpha.re, aim = alpha.im;
    int a_scale = 0, b_scale = 0;
    double sre = 0.0, sim = 0.0;
    if (d.cs == MD_CASE_0) aim = 0.0;
    else if (d.cs != MD_CASE_3 && aim != 0.0) {
        if (!literal) { d.status = MD_ERR_ALPHA_IMAG; return d; }
        if (d.cs == MD_CASE_1A || d.cs == MD_CASE_1B || d.cs == MD_CASE_2AB) {
            a_scale = d.cs != MD_CASE_1B;
            b_scale = d.cs == MD_CASE_1B;
            sre = are; sim = aim;
            are = 1.0; aim = 0.0;
        }
    }
    // Section 7.2: Im(beta) cannot change a real C.
    double bre = beta.re, bim = dt_cplx(dtc) ? beta.im : 0.0;
    // Section 7.1 option (1): beta takes C's storage precision.
    if (dt_half(dtc)) { bre = (double)(_Float16)bre; bim = (double)(_Float16)bim; }
    else if (!dt_dbl(dtc)) { bre = (double)(float)bre; bim = (double)(float)bim; }

    GemmArgs &g = d.g;
    g.A = A; g.B = B; g.C = C; g.Cin = C;
    g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.rsa = rsa; g.rsb = rsb; g.rsc = rsc;
    g.m = m; g.n = n; g.k = k;
    g.a_dbl = dt_dbl(dta); g.b_dbl = dt_dbl(dtb); g.c_dbl = dt_dbl(dtc);
    g.a_half = dt_half(dta); g.b_half = dt_half(dtb); g.c_half = dt_half(dtc);
    g.c_cplx = dt_cplx(dtc);
    g.ta = ta; g.tb = tb;
    // The fast kernels stage 16-byte chunks with buffer loads, which need only
    // the 4-byte alignment every s/d/c/z array has.  An operand stored
    // contiguous along k whose columns are not a whole number of chunks is
    // "ragged": the components a chunk reads past a column's end are zeroed
    // after the load (Stage::load_fast).
    const int wa = dt_cplx(dta) ? 2 : 1, wb = dt_cplx(dtb) ? 2 : 1;
    // components per 16-byte chunk
    const int cwa = dt_dbl(dta) ? 2 : (dt_half(dta) ? 8 : 4), cwb = dt_dbl(dtb) ? 2 : (dt_half(dtb) ? 8 : 4);
    // They address an operand tile with 32-bit byte offsets from its origin:
    // the stored columns the fast tile spans (its k extent for an operand
    // stored along m or n, its m or n extent for one stored along k), ld
    // elements apart, plus the reach of a chunk inside its column, must stay
    // below 2 GiB.  The tile is the one the fast kernel of this precision and
    // case would run, so a wider tile lowers the limit.
    int fbm, fbn, fbk;
    tile_shape(d.prec, d.cs, true, &fbm, &fbn, &fbk);
    const Lowering L0 = lower_case(d.cs);
    auto fast_ld_ok = [&](bool is_a, int dt, int tr, int64_t ld) {
        const bool mn_contig = is_a ? (tr == 0 || tr == 3) : (tr == 1 || tr == 2);
        const int64_t tmn = is_a ? fbm / (L0.mdbl ? 2 : 1) : fbn / (L0.ndbl ? 2 : 1);
        const int64_t tk = fbk / (L0.kdbl ? 2 : 1);
        const int64_t cols = mn_contig ? tk : tmn;
        const int64_t reach = 4096;  // a chunk's offset inside its column: < 256 elements of 16 bytes
        return ld < ((((int64_t)1 << 31) - reach) / (cols * dt_bytes(dt)));
    };
    // General storage (an element stride along the column, for any operand)
    // takes the component-wise path.  Binary16 operands have fast kernels when
    // both A and B are binary16 and the precision is single or half, with
    // every stored column a whole number of 4-byte words; otherwise they take
    // the component-wise path too.
    const bool plain_c = rsc == 1;
    const bool half_pair = dt_half(dta) && dt_half(dtb) && (d.prec == PREC_S || d.prec == PREC_H) &&
                           (lda * wa) % 2 == 0 && (ldb * wb) % 2 == 0;
    const bool ha_ok = !dt_half(dta) || half_pair, hb_ok = !dt_half(dtb) || half_pair;
    g.a_vec = ((uintptr_t)A % 4 == 0) && fast_ld_ok(true, dta, ta, lda) && rsa == 1 && plain_c && ha_ok;
    g.b_vec = ((uintptr_t)B % 4 == 0) && fast_ld_ok(false, dtb, tb, ldb) && rsb == 1 && plain_c && hb_ok;
    g.a_ragged = (ta == 1 || ta == 2) && (k * wa) % cwa != 0;
    g.b_ragged = (tb == 0 || tb == 3) && (k * wb) % cwb != 0;
    g.alpha_re = are; g.alpha_im = aim;
    g.a_scale = a_scale; g.b_scale = b_scale;
    g.scale_re = sre; g.scale_im = sim;
    g.beta_re = bre; g.beta_im = bim;
    g.beta_zero = (bre == 0.0 && bim == 0.0);

    if (m == 0 || n == 0) { d.quick = 1; return d; }
    if (k == 0 || (are == 0.0 && aim == 0.0)) { d.quick = 2; return d; }

    const Lowering L = lower_case(d.cs);
    int bm, bn, bk;
    tile_shape(d.prec, d.cs, g.a_vec && g.b_vec, &bm, &bn, &bk);
    int64_t tmn_a = bm / (L.mdbl ? 2 : 1), tmn_b = bn / (L.ndbl ? 2 : 1);
    // few tiles: the small kernel (single and double precision, BLAS storage,
    // no binary16 operand, no operand staged with alpha)
    const int64_t tiles = ((m + tmn_a - 1) / tmn_a) * ((n + tmn_b - 1) / tmn_b);
    const char *sm = getenv("MDGEMM_SMALL");
    if ((d.prec == PREC_S || d.prec == PREC_D) && !(sm && sm[0] == '0') && tiles <= SMALL_MAX_TILES &&
        k * (L.kdbl ? 2 : 1) <= SMALL_MAX_K && rsa == 1 && rsb == 1 && plain_c && !g.a_half && !g.b_half &&
        !a_scale && !b_scale) {
        g.small = 1;
        tmn_a = SMALL_TILE / (L.mdbl ? 2 : 1);
        tmn_b = SMALL_TILE / (L.ndbl ? 2 : 1);
    }
    // BF16x3 large enough to fill the GPU with 256 x 256 tiles: packed
    // operands (BLAS or row-major storage, no binary16 operand, no operand
    // staged with alpha)
    const char *pk = getenv("MDGEMM_PACK");
    const int pmode = pk ? atoi(pk) : 1;
    if (d.prec == PREC_BF16X3 && pmode != 0 && rsa == 1 && rsb == 1 && plain_c && !g.a_half && !g.b_half &&
        !a_scale && !b_scale) {
        const int64_t pa = PACK_TILE / (L.mdbl ? 2 : 1), pb = PACK_TILE / (L.ndbl ? 2 : 1);
        const int64_t ptiles = ((m + pa - 1) / pa) * ((n + pb - 1) / pb);
        if (pmode == 2 || (ptiles >= PACK_MIN_TILES && k * (L.kdbl ? 2 : 1) >= 256)) {
            g.packed = 1;
            tmn_a = pa;
            tmn_b = pb;
        }
    }
    g.tiles_m = (int)((m + tmn_a - 1) / tmn_a);
    g.tiles_n = (int)((n + tmn_b - 1) / tmn_b);
    return d;
}

}  // namespace md

namespace {

int run_decision(const Decision &d, void *stream, bool may_split = true) {
    if (d.status != MD_OK) return d.status;
    if (d.quick == 1) return MD_OK;
    if (d.quick == 2) return launch_scale(d.g, stream);
    if ((int64_t)d.g.tiles_m * d.g.tiles_n > 0x7fffffffLL) return MD_ERR_UNSUPPORTED;
    return launch_gemm(d.prec, d.cs, d.g, stream, nullptr, may_split);
}

}  // namespace

namespace md {

int gemm_enqueue(const md_gemm_desc &x, const void *c_in, void *stream, bool may_split) {
    Decision d = decide(x.transa, x.transb, x.m, x.n, x.k, x.alpha, x.A, x.dta, x.lda, x.B, x.dtb, x.ldb,
                        x.beta, x.C, x.dtc, x.ldc, x.comp);
    if (c_in) d.g.Cin = c_in;
    return run_decision(d, stream, may_split);
}

}  // namespace md

extern "C" {

int mdgemm(char transa, char transb, int64_t m, int64_t n, int64_t k, md_scalar alpha,
           const void *A, md_dt dta, int64_t lda, const void *B, md_dt dtb, int64_t ldb,
           md_scalar beta, void *C, md_dt dtc, int64_t ldc, md_comp comp, void *stream) {
    const Decision d = decide(transa, transb, m, n, k, alpha, A, dta, lda, B, dtb, ldb, beta, C, dtc,
                              ldc, comp);
    return run_decision(d, stream);
}

int mdgemm_strided(char transa, char transb, int64_t m, int64_t n, int64_t k, md_scalar alpha,
                   const void *A, md_dt dta, int64_t rsa, int64_t csa,
                   const void *B, md_dt dtb, int64_t rsb, int64_t csb,
                   md_scalar beta, void *C, md_dt dtc, int64_t rsc, int64_t csc,
                   md_comp comp, void *stream) {
    const int ta = norm_trans(transa), tb = norm_trans(transb);
    if (ta < 0) return -1;
    if (tb < 0) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    const bool uses_ab = m > 0 && n > 0 && k > 0 && (alpha.re != 0.0 || alpha.im != 0.0);
    if (uses_ab && A == nullptr) return -7;
    if (!dt_ok(dta)) return -8;
    if (uses_ab && B == nullptr) return -11;
    if (!dt_ok(dtb)) return -12;
    if (m > 0 && n > 0 && C == nullptr) return -16;
    if (!dt_ok(dtc)) return -17;
    if (!comp_ok(comp)) return -20;
    // each operand as a column-major view: its stored block (rows x cols),
    // or its transpose when its rows lie apart
    const bool an = ta == 0 || ta == 3, bn = tb == 0 || tb == 3;
    View va, vb, vc;
    int st = storage_view(an ? m : k, an ? k : m, rsa, csa, &va);
    if (st != 0) return st == 1 ? -9 : -10;
    st = storage_view(bn ? k : n, bn ? n : k, rsb, csb, &vb);
    if (st != 0) return st == 1 ? -13 : -14;
    st = storage_view(m, n, rsc, csc, &vc);
    if (st != 0) return st == 1 ? -18 : -19;
    // an operand seen transposed flips its op
    const char oa = va.transposed ? flip_op(transa) : transa;
    const char ob = vb.transposed ? flip_op(transb) : transb;
    if (!vc.transposed)
        return run_decision(decide(oa, ob, m, n, k, alpha, A, dta, va.ld, B, dtb, vb.ld, beta, C, dtc, vc.ld,
                                   comp, va.rs, vb.rs, vc.rs),
                            stream);
    // C seen transposed: C^T := beta C^T + alpha op(B)^T op(A)^T
    return run_decision(decide(flip_op(ob), flip_op(oa), n, m, k, alpha, B, dtb, vb.ld, A, dta, va.ld, beta, C,
                               dtc, vc.ld, comp, vb.rs, va.rs, vc.rs),
                        stream);
}

int mdgemm_plan(char transa, char transb, int64_t m, int64_t n, int64_t k, md_scalar alpha,
                const void *A, md_dt dta, int64_t lda, const void *B, md_dt dtb, int64_t ldb,
                md_scalar beta, void *C, md_dt dtc, int64_t ldc, md_comp comp, md_plan *out) {
    if (!out) return MD_ERR_STATE;
    memset(out, 0, sizeof(*out));
    Decision d = decide(transa, transb, m, n, k, alpha, A, dta, lda, B, dtb, ldb, beta, C, dtc,
                        ldc, comp);
    out->status = d.status;
    if (d.status < 0) return d.status;
    out->domain_case = d.cs;
    out->comp = d.prec == PREC_D ? MD_COMP_D
              : d.prec == PREC_S ? MD_COMP_S
              : d.prec == PREC_H ? MD_COMP_H : MD_COMP_S_BF16X3;
    if (d.status != MD_OK) return d.status;
    out->quick = d.quick;
    const Lowering L = lower_case(d.cs);
    out->a_parts = (L.mdbl || L.kdbl) ? 2 : 1;
    out->b_parts = (L.ndbl || L.kdbl) ? 2 : 1;
    out->m_real = m * (L.mdbl ? 2 : 1);
    out->n_real = n * (L.ndbl ? 2 : 1);
    out->k_real = k * (L.kdbl ? 2 : 1);
    if (d.quick == 0) {
        out->flops = (double)L.flop_factor * (double)m * (double)n * (double)k;
        int bm, bn, bk;
        tile_shape(d.prec, d.cs, d.g.a_vec && d.g.b_vec, &bm, &bn, &bk);
        if (d.g.small) bm = bn = SMALL_TILE, bk = 4;
        if (d.g.packed) bm = bn = PACK_TILE, bk = 32;
        out->tile_m = bm; out->tile_n = bn; out->tile_k = bk;
        out->workgroups = (int64_t)d.g.tiles_m * d.g.tiles_n;
        kernel_name(d.prec, d.cs, d.g, out->kernel, (int)sizeof(out->kernel));
    } else if (d.quick == 2) {
        snprintf(out->kernel, sizeof(out->kernel), "md_scale_kernel");
    }
    return d.status;
}

const char *mdgemm_strerror(int status) {
    if (status == MD_OK) return "success";
    if (status < 0) {
        static const char *args[] = {"?", "transa", "transb", "m", "n", "k", "alpha", "A", "dta",
                                     "lda", "B", "dtb", "ldb", "beta", "C", "dtc", "ldc", "comp",
                                     "stream"};
        int i = -status;
        if (i <= 18) return args[i];
        return "invalid argument in a grouped descriptor";
    }
    switch (status) {
    case MD_ERR_ALPHA_IMAG: return "Im(alpha) != 0 is not supported in cases 1a, 1b, 1c, 2ab, 2ac, 2bc";
    case MD_ERR_HIP: return "HIP launch or runtime error";
    case MD_ERR_BUDGET: return "request exceeds the memory budget";
    case MD_ERR_STATE: return "invalid state";
    case MD_ERR_UNSUPPORTED: return "not supported by this build";
    case MD_ERR_SCRATCH:
        return "the work table exceeds the fixed scratch of mdgemm_grouped_noalloc (MD_GROUPED_NOALLOC_BYTES)";
    }
    return "unknown status";
}

const char *mdgemm_version(void) { return "mdgemm 0.1 gfx950"; }

}  // extern "C"

