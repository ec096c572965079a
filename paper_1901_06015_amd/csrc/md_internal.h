// md_internal.h -- shared between the host planner and the device kernels of
// libmdgemm (never installed, never seen by callers).
#pragma once
#include <stdint.h>

#include "../../include/mdgemm.h"

namespace md {

// Lowering of a domain case onto one real product (Figure "mixeddom",
// Section 4.2).  The real product is C' (M' x N') += A' (M' x K') B' (K' x N'):
//   mdbl: M' = 2m -- C and A complex: Re/Im of A and C become separate rows
//         (case 2ac; in case 3 together with kdbl this is the 1e/1r pairing
//         of Eq. 1mc);
//   ndbl: N' = 2n -- C and B complex, A real: Re/Im of B and C become
//         separate columns (case 2bc);
//   kdbl: K' = 2k -- A and B complex: Re/Im of A and B interleave along the
//         inner dimension (case 2ab, and case 3).
// Operand parts that cannot reach C (Im(A) in 1a, Im(B) in 1b) are never
// staged; operand parts that are implicitly zero (Im(B) in 2ac, Im(A) in 2bc)
// generate no work.
struct Lowering {
    bool c_cplx, a_cplx, b_cplx;
    bool mdbl, ndbl, kdbl;
    int flop_factor;  // 2, 4 or 8 (x mnk)
};

inline Lowering lower_case(int cs) {
    Lowering L{};
    L.c_cplx = (cs == MD_CASE_1C || cs == MD_CASE_2AC || cs == MD_CASE_2BC || cs == MD_CASE_3);
    L.a_cplx = (cs == MD_CASE_1A || cs == MD_CASE_2AB || cs == MD_CASE_2AC || cs == MD_CASE_3);
    L.b_cplx = (cs == MD_CASE_1B || cs == MD_CASE_2AB || cs == MD_CASE_2BC || cs == MD_CASE_3);
    L.mdbl = (cs == MD_CASE_2AC || cs == MD_CASE_3);
    L.ndbl = (cs == MD_CASE_2BC);
    L.kdbl = (cs == MD_CASE_2AB || cs == MD_CASE_3);
    L.flop_factor = (cs == MD_CASE_3) ? 8 : ((cs == MD_CASE_2AB || cs == MD_CASE_2AC || cs == MD_CASE_2BC) ? 4 : 2);
    return L;
}

inline int classify(int dtc, int dta, int dtb) {
    auto cplx = [](int dt) { return dt == MD_C || dt == MD_Z || dt == MD_HC; };
    const bool c = cplx(dtc), a = cplx(dta), b = cplx(dtb);
    if (!c && !a && !b) return MD_CASE_0;
    if (!c && a && !b) return MD_CASE_1A;
    if (!c && !a && b) return MD_CASE_1B;
    if (c && !a && !b) return MD_CASE_1C;
    if (!c && a && b) return MD_CASE_2AB;
    if (c && a && !b) return MD_CASE_2AC;
    if (c && !a && b) return MD_CASE_2BC;
    return MD_CASE_3;
}

// Arguments of one product as the kernels see them (all operands already
// validated; alpha and beta already follow the scalar policies).
struct GemmArgs {
    const void *A;
    const void *B;
    void *C;
    const void *Cin;        // where beta*C is read from: C itself for the in-place
                            // operation, another m x n array of C's type and ldc otherwise
    int64_t lda, ldb, ldc;  // in elements of each operand's own type
    int64_t rsa, rsb, rsc;  // element stride along a stored column: 1, except for general
                            // storage (Section 3 row and column strides), which only the
                            // component-wise loads and their epilogue take
    int64_t m, n, k;
    int a_dbl, b_dbl, c_dbl;  // storage precision is double
    int a_half, b_half, c_half;  // storage precision is binary16 (component-wise path only)
    int c_cplx;               // C is complex
    int ta, tb;               // 0 = 'N', 1 = 'T', 2 = 'C', 3 = 'R' (conjugate, not transposed)
    int a_vec, b_vec;         // the operand can be staged in 16-byte chunks
    int a_ragged, b_ragged;   // stored along k, its columns end inside a chunk (Stage::load_fast)
    int beta_zero;            // C is not read
    double alpha_re, alpha_im;
    double beta_re, beta_im;
    int a_scale, b_scale;       // stage A (B) as (scale_re + i scale_im) times itself: a complex
    double scale_re, scale_im;  // alpha under the literal interpretation with C real
    int tiles_m, tiles_n;     // workgroup tiles of the real product
    int small;                // runs on md_small_kernel: 32 x 32 real-product tiles (md_small.h)
    int packed;               // BF16x3 on packed operands: 256 x 256 real-product tiles (md_pack.h)
    int splits;               // > 1: k split over this many workgroups per tile (plain kernels)
    void *part;               // their partial products: splits x n x m pairs (re, im) of the
                              // computation type, summed and finished by md_split_reduce
};

enum Prec { PREC_S = 0, PREC_D = 1, PREC_BF16X3 = 2, PREC_H = 3 };

// Tile configuration of the plain product kernel for (computation precision,
// case, fast load path): 0 = 128 x 128 tiles of 4 waves, 1 = 128 x 256 and
// 2 = 256 x 128 tiles of 8 waves, 3 = 128 x 128 tiles of 8 waves, 4 = 256 x
// 256 tiles of 8 waves (half precision only).  The host's
// tile counts and the device's kernel choice both come from here.  MD_WIDE
// selects them at build time: bits 0/1 FP64/FP32 -> 128 x 256, bits 2/3 ->
// 256 x 128, bits 4/5 -> 8-wave 128 x 128.  Default: 8-wave 128 x 128 for
// both (measured at m=n=k=4096 against the 4-wave tile: FP32 1.00-1.11x,
// 1.047x on average; FP64 0.99-1.05x, 1.028x on average).
#ifndef MD_WIDE
#define MD_WIDE 48
#endif
// BF16x3 keeps 4 waves per 128 x 128 tile: 8 waves measured 0.95x at 8192.
#ifndef MD_BF16X3_DEEP
#define MD_BF16X3_DEEP 0
#endif
// MD_H16_TILE: tile of the half computation precision's fast kernels: 0 the
// 4-wave 128 x 128 tile, 1 the 8-wave one (measured 0.82-0.99x tile 0 at
// 8192), 2 (default) the 8-wave 256 x 256 tile (1.23-1.39x tile 0 at 8192:
// with FP32 or FP64 operands the 128 x 128 tile is bound by operand traffic).
#ifndef MD_H16_TILE
#define MD_H16_TILE 2
#endif
constexpr int tile_kind(int prec, int cs, bool fast) {
    return !fast ? 0
         : prec == PREC_BF16X3 ? (MD_BF16X3_DEEP ? 3 : 0)
         : prec == PREC_H ? (MD_H16_TILE == 2 ? 4 : MD_H16_TILE == 1 ? 3 : 0)
         : (MD_WIDE & (prec == PREC_D ? 1 : 2)) ? 1
         : (MD_WIDE & (prec == PREC_D ? 4 : 8)) ? 2
         : (MD_WIDE & (prec == PREC_D ? 16 : 32)) ? 3 : 0 * cs;
}

// Products with few output tiles run on md_small_kernel (md_small.h): at
// most SMALL_MAX_TILES tiles of the tiled kernel and an inner dimension of the
// real product of at most SMALL_MAX_K.  MDGEMM_SMALL=0 in the environment
// turns it off (read on every call).
constexpr int SMALL_TILE = 32;
constexpr int SMALL_MAX_TILES = 16;
constexpr int64_t SMALL_MAX_K = 2048;

// Everything mdgemm decides before touching the device (mdgemm_api.cpp).
struct Decision {
    int status = MD_OK;
    int cs = MD_CASE_0;
    int prec = PREC_S;
    int quick = 0;  // 0 full product, 1 no-op, 2 C := beta*C
    GemmArgs g{};
};

// rsa/rsb/rsc: element stride along each stored column (1 for BLAS storage).
Decision decide(char transa, char transb, int64_t m, int64_t n, int64_t k, md_scalar alpha,
                const void *A, int dta, int64_t lda, const void *B, int dtb, int64_t ldb,
                md_scalar beta, void *C, int dtc, int64_t ldc, int comp,
                int64_t rsa = 1, int64_t rsb = 1, int64_t rsc = 1);

// Host-side launchers (mdgemm_launch.hip, mdgemm_packed.hip).
// may_split false: never split k or pack, so nothing is allocated (the split-k
// and packing workspaces are the plain path's only allocations).
int launch_gemm(int prec, int cs, const GemmArgs &a, void *stream, int64_t *wg_out, bool may_split = true);
int launch_small(int prec, int cs, const GemmArgs &a, void *stream);
// BF16x3 products with at least PACK_MIN_TILES 256 x 256 tiles (half the
// MI355X's CUs; a constant, so that planning needs no device) and k' >= 256
// run on packed operands (md_pack.h): the operands are cast, split and packed
// once into a per-stream workspace of at most PACK_MAX_BYTES, then multiplied
// with direct-to-LDS copies.  MDGEMM_PACK in the environment: 0 never, 2
// whenever the product qualifies otherwise (any size), else the size rule
// (read on every call).  launch_packed returns MD_ERR_BUDGET, having enqueued
// nothing, when the workspace cannot be had.
constexpr int PACK_TILE = 256;
constexpr int64_t PACK_MIN_TILES = 128;
constexpr size_t PACK_MAX_BYTES = (size_t)8 << 30;
int launch_packed(int cs, const GemmArgs &a, void *stream);
int launch_scale(const GemmArgs &a, void *stream);
void tile_shape(int prec, int cs, bool fast, int *bm, int *bn, int *bk);
void kernel_name(int prec, int cs, const GemmArgs &a, char *out, int len);

// Out-of-place forms used by the serving loop of the same library:
// C := beta*Cin + alpha*op(A)op(B), where Cin (m x n, C's storage type,
// leading dimension ldc) is read and C is written; a null c_in means in place.
// Validation and status codes are mdgemm's / mdgemm_grouped's.
int gemm_enqueue(const md_gemm_desc &d, const void *c_in, void *stream, bool may_split = true);

// Reusable descriptor-table workspace of one stream that issues grouped
// launches: page-locked host staging and its device copy, grown on demand.
// The caller guarantees that the launch which last used it has completed.
struct GroupedWs {
    char *host = nullptr;
    char *dev = nullptr;
    size_t cap = 0;
};
// noalloc: upload the work table into the library's fixed device array
// (MD_ERR_SCRATCH, nothing enqueued, if it does not fit) and run the
// products that take the plain kernels unsplit: nothing is allocated.
int grouped_enqueue(int64_t count, const md_gemm_desc *descs, const void *const *c_in, void *stream,
                    GroupedWs *ws, bool noalloc = false);
void grouped_ws_release(GroupedWs *ws);

}  // namespace md
