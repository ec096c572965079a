// md_tile.h -- device side of libmdgemm for gfx950 (CDNA4): the product kernel
// template, instantiated by mdgemm_kernels.hip.
//
// Each workgroup owns a tile of the real product C' += A' B' that its domain
// case lowers to (md_internal.h, Figure "mixeddom"):
//
//   1. cast-on-pack: A and B tiles are read from HBM in their storage type
//      with 16-byte loads, converted to the computation type in registers
//      (float -> double exact, double -> float round-to-nearest-even: the
//      typecasting pack of Section 5) and written to LDS already in the layout
//      of the real product: complex elements are split into their parts, parts
//      that cannot reach C are dropped, conjugation flips a sign, and case 3
//      writes A in the 1e arrangement of Eq. 1mc (each complex element becomes
//      the real 2x2 block [re -im; im re]) while B keeps the 1r arrangement
//      (re, im interleaved along k);
//   2. a double-buffered k loop of real MFMA (v_mfma_f64_16x16x4f64 or
//      v_mfma_f32_16x16x4f32) over the LDS tiles: the global loads of tile t+2
//      are in flight while tile t multiplies, the fragments of the next k group
//      are read while the current one multiplies, and the LDS writes of tile
//      t+1 are interleaved with the last MFMAs of tile t;
//   3. an epilogue that applies alpha (cast to the computation precision) and
//      beta (cast to C's storage precision), forms beta*C + alpha*AB in the
//      wider of the computation and C precisions, and rounds once to C's
//      storage type (Sections 5.1.3 and 7.1).
//
// LDS layout follows each operand's orientation in HBM so that the staging
// writes are 16-byte vectors without bank conflicts: an operand contiguous
// along m (or n) is kept as [k][mn], one contiguous along k as [mn][k].
// The MFMA is issued with B' as its first operand so that the accumulator
// lanes run along m: stores to column-major C are then contiguous.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "md_half.h"
#include "md_internal.h"

namespace md {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

constexpr int NT = 256;  // threads per workgroup: 4 waves of 64
constexpr int G = 16;    // MFMA block edge (16x16 output blocks)

// Build-time tuning knob: MD_OCC waves per SIMD the default-tile kernels are
// compiled for (2: two workgroups per CU share each SIMD, 256 registers per
// lane; 1: one workgroup per CU, 512 registers per lane).
#ifndef MD_OCC
#define MD_OCC 2
#endif

// LDS row padding of each layout per element type (chosen so that fragment
// reads and staging writes hit distinct banks).
template <class T> struct Pad;
template <> struct Pad<double> { static constexpr int PADW = 8, PADK = 2; };
template <> struct Pad<float> { static constexpr int PADW = 4, PADK = 4; };

// Tile configuration: workgroup tile BM x BN of the real product, computed by
// WGM x WGN waves of (BM/WGM) x (BN/WGN) = WMB x WNB MFMA blocks; k depth BK
// of one LDS tile; OCC waves per SIMD the kernel is compiled for (the
// register budget: 512 / OCC per lane); PIPE the order of the k loop
// (md_gemm_kernel).
template <class T, int BM_, int BN_, int BK_, int OCC_, int WGM_ = 2, int WGN_ = 2, bool PIPE_ = true>
struct TCfg {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, OCC = OCC_, WGM = WGM_, WGN = WGN_;
    static constexpr bool PIPE = PIPE_;
    static constexpr int NT = 64 * WGM * WGN;  // threads per workgroup
    static constexpr int PADW = Pad<T>::PADW, PADK = Pad<T>::PADK;
    static constexpr int WMB = BM / (WGM * 16), WNB = BN / (WGN * 16);
};
// The default configuration (also the BF16x3 kernel's): 128 x 128 tiles of
// 4 waves, two workgroups per CU.
template <class T> struct TileCfg;
template <> struct TileCfg<double> : TCfg<double, 128, 128, 16, MD_OCC, 2, 2, false> {};
template <> struct TileCfg<float> : TCfg<float, 128, 128, 32, MD_OCC> {};
// Wide configurations: 8 waves of 64 x 64 (the default's wave tile and
// register budget, two waves per SIMD) on one 128 x 256 (WideN) or 256 x 128
// (WideM) tile per CU, so a CU stages a quarter fewer operand bytes per k.
template <class T> struct WideN;
template <> struct WideN<double> : TCfg<double, 128, 256, 16, 2, 2, 4> {};
template <> struct WideN<float> : TCfg<float, 128, 256, 32, 2, 2, 4> {};
template <class T> struct WideM;
template <> struct WideM<double> : TCfg<double, 256, 128, 16, 2, 4, 2> {};
template <> struct WideM<float> : TCfg<float, 256, 128, 32, 2, 4, 2> {};
// Deep configuration: the default 128 x 128 tile split over 8 waves of
// 64 x 32, four waves per SIMD (128 registers per lane).
#ifndef MD_DEEP_OCC
#define MD_DEEP_OCC 4
#endif
// Build knobs of the FP32 form (measured against the defaults on the sweep):
// MD_F32_BK its k depth, MD_F32_OCC its waves per SIMD, MD_F32_WGM x
// MD_F32_WGN its wave grid.
#ifndef MD_F32_BK
#define MD_F32_BK 32
#endif
#ifndef MD_F32_OCC
#define MD_F32_OCC MD_DEEP_OCC
#endif
#ifndef MD_F32_WGM
#define MD_F32_WGM 2
#endif
#ifndef MD_F32_WGN
#define MD_F32_WGN 4
#endif
template <class T> struct Deep;
template <> struct Deep<double> : TCfg<double, 128, 128, 16, MD_DEEP_OCC, 2, 4> {};
template <> struct Deep<float> : TCfg<float, 128, 128, MD_F32_BK, MD_F32_OCC, MD_F32_WGM, MD_F32_WGN> {};
// 256 x 256 tiles of 8 waves (64 x 128 each): half the operand bytes per
// flop of a 128 x 128 tile, for the half computation precision, whose
// one-plane LDS tiles fit (80 KB double-buffered).
template <class T> struct Big;
template <> struct Big<float> : TCfg<float, 256, 256, 32, 2, 2, 4> {};

template <class T> struct AccT;
template <> struct AccT<double> { typedef v4d type; };
template <> struct AccT<float> { typedef v4f type; };

__device__ __forceinline__ v4d mfma16(double x, double y, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float x, float y, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
}

// Row (inside a 16x16 block) of accumulator item v held by `lane`; the column
// is lane & 15.  The two 16x16x4 instructions lay their results out
// differently (measured on gfx950).
template <class T> __device__ __forceinline__ int acc_row(int lane, int v);
template <> __device__ __forceinline__ int acc_row<double>(int lane, int v) { return 4 * v + (lane >> 4); }
template <> __device__ __forceinline__ int acc_row<float>(int lane, int v) { return 4 * (lane >> 4) + v; }

// LDS layout of one operand tile: BMN (m or n) x BK (k) elements of T.
template <class T, bool MNC, int BMN, class C = TileCfg<T>>
struct Lay {
    static constexpr int LD = MNC ? BMN + C::PADW : C::BK + C::PADK;
    static constexpr int SIZE = (MNC ? C::BK : BMN) * LD;
    __device__ __forceinline__ static int at(int kk, int mm) { return MNC ? kk * LD + mm : mm * LD + kk; }
};

// ---------------------------------------------------------------------------
// Operand staging (cast-on-pack)
// ---------------------------------------------------------------------------
// A staged chunk, released component by component where it is used.  An LDS
// write of the chunk as it is (double into an FP64 tile, float into an FP32
// tile) or a conversion from a double takes two or four registers of the
// loaded tuple together; across the k loop's back edge the compiler then
// splits that tuple and copies it right after the global load, which waits
// for the load at once.  And where parts of a chunk are never used (the
// imaginary parts in cases 1a and 1b), their registers are taken as
// temporaries while the load is still in flight, which waits for it too.
// An empty statement that reads and rewrites all four components in place
// (no instruction, no extra register) keeps every loaded register live until
// here and gives the tuple only single-register uses, so the load stays in
// flight through the MFMAs of a whole k-tile (checked on the generated code).
__device__ __forceinline__ uint4 detach(uint4 h) {
    asm("" : "+v"(h.x), "+v"(h.y), "+v"(h.z), "+v"(h.w));
    return h;
}

enum Mode {
    M_PLAIN = 0,   // real operand
    M_REONLY = 1,  // complex operand of which only Re reaches C (1a: A, 1b: B)
    M_KINT = 2,    // complex; Re/Im interleaved along k (2ab: A and B; 3: B = 1r)
    M_MNINT = 3,   // complex; Re/Im as separate rows/columns (2ac: A; 2bc: B)
    M_ONEE = 4     // complex A of case 3 in the 1e arrangement
};

template <int CS, bool IS_A> __host__ __device__ constexpr int mode_of() {
    if (IS_A) {
        return CS == MD_CASE_1A ? M_REONLY
             : CS == MD_CASE_2AB ? M_KINT
             : CS == MD_CASE_2AC ? M_MNINT
             : CS == MD_CASE_3 ? M_ONEE : M_PLAIN;
    }
    return CS == MD_CASE_1B ? M_REONLY
         : (CS == MD_CASE_2AB || CS == MD_CASE_3) ? M_KINT
         : CS == MD_CASE_2BC ? M_MNINT : M_PLAIN;
}

// Real row (or column) of the tile that holds part q of complex index mm when
// Re/Im are split: blocks of G alternate Re, Im so that both parts of one
// complex element land in the same lane of the same MFMA block pair.
__device__ __forceinline__ int split_pos(int mm, int q) { return (((mm >> 4) << 1) + q) * G + (mm & 15); }

// FAST: aligned operand, 16-byte buffer loads, LDS layout = orientation MNC
//       (true: contiguous along m/n in HBM).
// !FAST: any alignment / leading dimension; the orientation comes from the
//       trans argument at run time, components are loaded one by one and the
//       LDS layout is [k][mn] (MNC must be true).
// RAG (fast path only): the operand's columns may end inside a chunk; an
// operand stored contiguous along k then masks what a chunk reads past them.
// SCL: the operand is staged as (scale_re + i scale_im) times itself.
// RTO: double components become float by round-to-odd (float_rto), for the
// half kernels, which round the staged float once more to binary16.
// SH (fast path): binary16 storage, 8 components per 16-byte chunk.
template <class T, int CS, bool IS_A, bool FAST, bool SDBL, bool MNC, class C = TileCfg<T>, bool RAG = false,
          bool SCL = false, bool RTO = false, bool SH = false>
struct Stage {
    static constexpr int MODE = mode_of<CS, IS_A>();
    static constexpr int W = (MODE == M_PLAIN) ? 1 : 2;  // stored components per element
    static constexpr bool MN2 = (MODE == M_MNINT || MODE == M_ONEE);
    static constexpr bool K2 = (MODE == M_KINT || MODE == M_ONEE);
    static constexpr int BMN = IS_A ? C::BM : C::BN;
    typedef Lay<T, MNC, BMN, C> L;
    static constexpr int TMN = BMN / (MN2 ? 2 : 1);  // stored m (or n) extent of a tile
    static constexpr int TK = C::BK / (K2 ? 2 : 1);   // stored k extent of a tile
    static constexpr int ESZ = SDBL ? 8 : (SH ? 2 : 4);  // bytes per stored component
    static constexpr int CW = 16 / ESZ;               // components per chunk (one 16-byte load)
    static constexpr int CHUNKS = TMN * TK * W / CW;
    // A tile with fewer chunks than threads (possible with 8 waves) leaves
    // the last threads idle; chunk counts are multiples of 64, so whole waves.
    static constexpr bool PARTIAL = CHUNKS < C::NT;
    static constexpr int PER = PARTIAL ? 1 : CHUNKS / C::NT;
    static constexpr int CPC_MN = TMN * W / CW, CPC_K = TK * W / CW;
    // Sign applied to Im when it is placed at an odd k' row: -Im(A) in case 2ab
    // realises Re(AB) = ArBr - AiBi; B's Im enters positively.
    static constexpr bool KNEG = IS_A;
    static_assert(FAST || MNC, "the generic path stages into the [k][mn] layout");
    static_assert(!(SH && (SDBL || !FAST)), "binary16 chunks: fast path, single-width staging");
    static_assert(PARTIAL ? CHUNKS % 64 == 0 : CHUNKS % C::NT == 0, "tile does not split evenly over the workgroup");
    static_assert((TMN * W) % CW == 0 && (TK * W) % CW == 0, "chunks straddle columns");
    static_assert((CPC_MN & (CPC_MN - 1)) == 0 && (CPC_K & (CPC_K - 1)) == 0 && CPC_MN <= C::NT && CPC_K <= C::NT,
                  "chunk grid must be a power of two no wider than the workgroup");

    uint4 raw[PER];  // one tile's loads, held until converted

    const char *base;
    int64_t ld, rs, MN, K, mn0;  // rs: element stride along a stored column (generic path)
    bool half;                   // binary16 storage (generic path, single-width components)
    int64_t total_bytes;  // extent of the stored matrix
    bool mn_contig, conj;
    uint32_t cmask;  // sign bit of the imaginary components when conjugating, else 0
    // Scaling by a complex alpha while staging (literal interpretation, real C):
    // only the complex operand of cases 1a, 1b and 2ab is ever scaled.  A
    // compile-time choice: a run-time branch here slows the unscaled kernels.
    static_assert(!SCL || ((MODE == M_REONLY || MODE == M_KINT) && W == 2), "only a complex operand is scaled");
    T sre, sim;
    int cpc_log;          // log2 of chunks per stored column inside a tile
    int pos, col0;        // this thread's chunk 0: position in its column, column in the tile
    int col_step;         // columns between a thread's consecutive chunks
    bool active;          // this thread stages a chunk (always, unless PARTIAL)

    __device__ __forceinline__ Stage(const GemmArgs &g, int tid, int64_t mn0_) {
        const int tr = IS_A ? g.ta : g.tb;
        // A is stored along m for 'N'/'R', B along n for 'T'/'C'
        mn_contig = FAST ? MNC : (IS_A ? (tr == 0 || tr == 3) : (tr == 1 || tr == 2));
        conj = tr >= 2;
        cmask = (conj && W == 2) ? 0x80000000u : 0u;
        sre = (T)g.scale_re;
        sim = (T)g.scale_im;
        ld = IS_A ? g.lda : g.ldb;
        rs = IS_A ? g.rsa : g.rsb;
        half = !SDBL && (IS_A ? g.a_half : g.b_half);
        MN = IS_A ? g.m : g.n;
        K = g.k;
        mn0 = mn0_;
        base = (const char *)(IS_A ? g.A : g.B);
        const int cpc = mn_contig ? CPC_MN : CPC_K;
        cpc_log = __builtin_ctz(cpc);
        pos = tid & (cpc - 1);
        col0 = tid >> cpc_log;
        col_step = C::NT >> cpc_log;
        active = !PARTIAL || tid < CHUNKS;
        const int64_t rows_st = mn_contig ? MN : K, cols_st = mn_contig ? K : MN;
        // whole dwords: the buffer range check drops a dword that crosses the
        // limit, which binary16 data can end inside (the extra bytes share
        // the last valid element's word; k-contiguous chunks mask them)
        total_bytes = (((cols_st - 1) * ld + rows_st) * W * ESZ + 3) & ~(int64_t)3;
    }

    // FAST path: buffer loads.  A chunk outside the matrix gets an offset
    // beyond the resource's range and reads as zero, with no branch.  When the
    // stored columns end inside a chunk (RAG), a chunk can reach past its
    // column's end into the next column, padding, or nothing.  Along m or n
    // those components land in rows (columns) of the real product beyond the
    // matrix, which feed only outputs the epilogue never writes; along k they
    // would meet the other operand's k beyond the matrix, so there they are
    // zeroed after the load.
    __device__ __forceinline__ void load_fast(int t) {
        const int64_t k0 = (int64_t)t * TK;
        const int64_t base_off = (MNC ? (k0 * ld + mn0) : (mn0 * ld + k0)) * W * ESZ;
        const int64_t rem = total_bytes - base_off;
        const int nrec = rem > 0x7fffffffLL ? 0x7fffffff : (rem < 0 ? 0 : (int)rem);
        __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void *)(base + base_off), (short)0, nrec, 0x00020000);
        const int64_t lim64 = K - k0;
        const int klim = lim64 > (1 << 30) ? (1 << 30) : (int)lim64;
        const int64_t mlim64 = MN - mn0;
        const int mlim = mlim64 > (1 << 30) ? (1 << 30) : (int)mlim64;
        const uint32_t col_bytes = (uint32_t)(ld * W * ESZ);
        const int epos = (pos * CW) / W;  // first element of the chunk along the contiguous dim
#pragma unroll
        for (int c = 0; c < PER; ++c) {
            const int col = col0 + c * col_step;
            const int e_mn = MNC ? epos : col;
            const int e_k = MNC ? col : epos;
            const bool ok = (!PARTIAL || active) && (e_mn < mlim) && (e_k < klim);
            const uint32_t off = ok ? (uint32_t)col * col_bytes + (uint32_t)(pos * 16) : 0x80000000u;
            const auto x = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
            uint4 v = make_uint4(x[0], x[1], x[2], x[3]);
            if constexpr (RAG && !MNC) {
                // components of this chunk inside its column
                const int64_t lim = (int64_t)klim * W - pos * CW;
                if constexpr (SDBL) {
                    if (lim < 2) { v.z = 0u; v.w = 0u; }
                } else if constexpr (SH) {
                    // two binary16 components per word, the lower one first
                    auto keep = [&](uint32_t w, int i) {
                        return lim <= 2 * i ? 0u : (lim == 2 * i + 1 ? (w & 0xFFFFu) : w);
                    };
                    v.x = keep(v.x, 0);
                    v.y = keep(v.y, 1);
                    v.z = keep(v.z, 2);
                    v.w = keep(v.w, 3);
                } else {
                    if (lim < 2) v.y = 0u;
                    if (lim < 3) v.z = 0u;
                    if (lim < 4) v.w = 0u;
                }
            }
            raw[c] = v;
        }
    }

    // Generic path: components loaded one by one; outside the matrix reads zero.
    // Component x of a stored column sits at (x / W) * rs * W + x % W (x
    // itself when the elements of a column are adjacent).
    __device__ __forceinline__ void load_generic(int t) {
        const int64_t k0 = (int64_t)t * TK;
        const int64_t rows_st = mn_contig ? MN : K, cols_st = mn_contig ? K : MN;
        const int64_t r0 = mn_contig ? mn0 : k0, c0 = mn_contig ? k0 : mn0;
        const int64_t contig_len = rows_st * W, col_stride = ld * W, rsw = rs * W;
        auto at = [&](int64_t x) { return (x / W) * rsw + x % W; };
#pragma unroll
        for (int c = 0; c < PER; ++c) {
            const int64_t col = c0 + col0 + c * col_step, comp0 = r0 * W + pos * CW;
            const bool colok = (!PARTIAL || active) && col < cols_st;
            const int64_t cbase = col * col_stride;
            if constexpr (SDBL) {
                const uint2 *p = (const uint2 *)base + cbase;
                uint2 e0 = make_uint2(0u, 0u), e1 = e0;
                if (colok && comp0 + 0 < contig_len) e0 = p[at(comp0 + 0)];
                if (colok && comp0 + 1 < contig_len) e1 = p[at(comp0 + 1)];
                raw[c] = make_uint4(e0.x, e0.y, e1.x, e1.y);
            } else if (half) {
                // binary16 components widened exactly to float in the chunk registers
                const _Float16 *p = (const _Float16 *)base + cbase;
                uint32_t e0 = 0u, e1 = 0u, e2 = 0u, e3 = 0u;
                if (colok && comp0 + 0 < contig_len) e0 = __float_as_uint((float)p[at(comp0 + 0)]);
                if (colok && comp0 + 1 < contig_len) e1 = __float_as_uint((float)p[at(comp0 + 1)]);
                if (colok && comp0 + 2 < contig_len) e2 = __float_as_uint((float)p[at(comp0 + 2)]);
                if (colok && comp0 + 3 < contig_len) e3 = __float_as_uint((float)p[at(comp0 + 3)]);
                raw[c] = make_uint4(e0, e1, e2, e3);
            } else {
                const uint32_t *p = (const uint32_t *)base + cbase;
                uint32_t e0 = 0u, e1 = 0u, e2 = 0u, e3 = 0u;
                if (colok && comp0 + 0 < contig_len) e0 = p[at(comp0 + 0)];
                if (colok && comp0 + 1 < contig_len) e1 = p[at(comp0 + 1)];
                if (colok && comp0 + 2 < contig_len) e2 = p[at(comp0 + 2)];
                if (colok && comp0 + 3 < contig_len) e3 = p[at(comp0 + 3)];
                raw[c] = make_uint4(e0, e1, e2, e3);
            }
        }
    }

    // Issue the global loads of k-tile t.
    __device__ __forceinline__ void load(int t) {
        if constexpr (FAST) load_fast(t);
        else load_generic(t);
    }

    // Component q of a chunk converted to the computation type.
    __device__ __forceinline__ static T component(const uint4 &h, int q) {
        if constexpr (SDBL) {
            const uint32_t w0 = q ? h.z : h.x;
            const uint32_t w1 = q ? h.w : h.y;
            const double d = __builtin_bit_cast(double, ((uint64_t)w1 << 32) | w0);
            if constexpr (RTO) return (T)float_rto(d);
            else return (T)d;
        } else if constexpr (SH) {
            const int wi = q >> 1;
            const uint32_t w = wi == 0 ? h.x : (wi == 1 ? h.y : (wi == 2 ? h.z : h.w));
            const uint16_t b = (q & 1) ? (uint16_t)(w >> 16) : (uint16_t)(w & 0xFFFFu);
            return (T)(float)__builtin_bit_cast(_Float16, b);
        } else {
            const uint32_t w = q == 0 ? h.x : (q == 1 ? h.y : (q == 2 ? h.z : h.w));
            return (T)__builtin_bit_cast(float, w);
        }
    }

    // Place part `part` (0 Re, 1 Im) of stored element (mm, kk) of the tile at
    // its position (k', m') in the real product through `out.put(k', m', v)`.
    template <class Out>
    __device__ __forceinline__ static void emit(Out &out, int mm, int kk, int part, T v, bool conj) {
        if constexpr (MODE == M_PLAIN) {
            out.put(kk, mm, v);
        } else if constexpr (MODE == M_REONLY) {
            if (part == 0) out.put(kk, mm, v);
        } else {
            const T vi = conj ? -v : v;
            if constexpr (MODE == M_KINT) {
                if (part == 0) out.put(2 * kk, mm, v);
                else out.put(2 * kk + 1, mm, KNEG ? -vi : vi);
            } else if constexpr (MODE == M_MNINT) {
                if (part == 0) out.put(kk, split_pos(mm, 0), v);
                else out.put(kk, split_pos(mm, 1), vi);
            } else {  // M_ONEE: [re -im; im re] per complex element (Eq. 1mc)
                if (part == 0) {
                    out.put(2 * kk, split_pos(mm, 0), v);
                    out.put(2 * kk + 1, split_pos(mm, 1), v);
                } else {
                    out.put(2 * kk, split_pos(mm, 1), vi);
                    out.put(2 * kk + 1, split_pos(mm, 0), -vi);
                }
            }
        }
    }

    // Writes one element of the real product's tile into an LDS buffer of T.
    struct PlainOut {
        static constexpr bool NARROW = false;  // values go to LDS in T
        T *lds;
        __device__ __forceinline__ void put(int kk, int mm, T v) const { lds[L::at(kk, mm)] = v; }
    };

    // Position (mm, kk) of element e of chunk column col.
    __device__ __forceinline__ void where(int e, int col, int *mm, int *kk) const {
        if constexpr (FAST) {
            *mm = MNC ? e : col;
            *kk = MNC ? col : e;
        } else {
            *mm = mn_contig ? e : col;
            *kk = mn_contig ? col : e;
        }
    }

    // The scaled form of store_to: each complex element x (conjugated first
    // for 'C'/'R') is placed as alpha*x, rounded in the computation type.
    template <class Out>
    __device__ __forceinline__ void store_scaled(Out out) const {
#pragma unroll
        for (int c = 0; c < PER; ++c) {
            const int col = col0 + c * col_step;
            const uint4 h = detach(raw[c]);
#pragma unroll
            for (int q = 0; q < CW; q += 2) {
                const T re = component(h, q);
                const T im0 = component(h, q + 1);
                const T im = conj ? -im0 : im0;
                const T pr = fma(sre, re, -(sim * im));
                const T pi = fma(sre, im, sim * re);
                int mm, kk;
                where(pos * (CW / W) + q / W, col, &mm, &kk);
                emit(out, mm, kk, 0, pr, false);
                emit(out, mm, kk, 1, pi, false);
            }
        }
    }

    // Convert the staged registers and hand every element to `out`.
    template <class Out>
    __device__ __forceinline__ void store_to(Out out) const {
        if (PARTIAL && !active) return;
        if constexpr (SCL) {
            store_scaled(out);
            return;
        }
#pragma unroll
        for (int c = 0; c < PER; ++c) {
            const int col = col0 + c * col_step;
            // conjugation flips the sign bit of every imaginary component in
            // place (no select, no extra registers): the high word of the
            // second double, the odd float words, or the upper binary16 half
            // of every word
            // (an operand of which only Re reaches C, stored as double,
            // measured better without: its unused halves hold four registers
            // per chunk and spill)
            // (not needed where every value is converted to 16 bits on its
            // way to LDS: the BF16x3 and half outputs; there it costs a copy)
            uint4 h = ((MODE == M_REONLY && SDBL) || Out::NARROW) ? raw[c] : detach(raw[c]);
            if constexpr (W == 2) {
                if constexpr (SDBL) {
                    h.w ^= cmask;
                } else if constexpr (SH) {
                    h.x ^= cmask;
                    h.y ^= cmask;
                    h.z ^= cmask;
                    h.w ^= cmask;
                } else {
                    h.y ^= cmask;
                    h.w ^= cmask;
                }
            }
#pragma unroll
            for (int q = 0; q < CW; ++q) {
                const T v = component(h, q);
                const int e = pos * (CW / W) + q / W;
                const int part = q % W;
                if constexpr (FAST) {
                    if constexpr (MNC) emit(out, e, col, part, v, false);
                    else emit(out, col, e, part, v, false);
                } else {
                    const int mm = mn_contig ? e : col;
                    const int kk = mn_contig ? col : e;
                    emit(out, mm, kk, part, v, false);
                }
            }
        }
    }

    __device__ __forceinline__ void store(T *lds) const { store_to(PlainOut{lds}); }
};

// ---------------------------------------------------------------------------
// Workgroup -> tile mapping.  Workgroups are dealt round-robin to the 8 XCDs
// (each with its own L2); renumber so that each XCD gets a contiguous range of
// tiles, then walk that range in column groups of GROUP_M row-tiles so
// neighbouring workgroups share A row-panels and B column-panels in L2.
// ---------------------------------------------------------------------------
constexpr int NXCD = 8;
constexpr int GROUP_M = 8;

__device__ __forceinline__ void map_tile(int wg, int nwg, int tiles_m, int tiles_n, int *tm, int *tn) {
    const int q = nwg / NXCD, r = nwg % NXCD;
    const int xcd = wg % NXCD, local = wg / NXCD;
    const int lin = (xcd < r) ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
    const int group = GROUP_M * tiles_n;
    const int gid = lin / group;
    const int first_m = gid * GROUP_M;
    const int gm = min(tiles_m - first_m, GROUP_M);
    const int in = lin - gid * group;
    *tm = first_m + in % gm;
    *tn = in / gm;
}

// ---------------------------------------------------------------------------
// Epilogue: C := beta*C + alpha*AB, rounded once to C's storage type
// ---------------------------------------------------------------------------
// Partial product of split workgroup `split` for C(i, j): alpha-free (re, im)
// in the computation type, at part[split][j][i].
template <class T>
__device__ __forceinline__ void store_partial(const GemmArgs &g, int split, int64_t i, int64_t j, T re, T im) {
    if (i >= g.m || j >= g.n) return;
    T *p = (T *)g.part + 2 * (((int64_t)split * g.n + j) * g.m + i);
    p[0] = re;
    p[1] = im;
}

// GS: C may have an element stride along its columns (general storage; only
// the component-wise kernels are launched for it).
template <bool GS>
__device__ __forceinline__ int64_t c_offset(const GemmArgs &g, int64_t i, int64_t j) {
    return (GS ? i * g.rsc : i) + j * g.ldc;
}

// HC: C may be binary16 (the plain kernels and the split reduction; the
// grouped kernel, which never sees one, leaves that code out).
template <class T, bool GS = false, bool HC = false>
__device__ __forceinline__ void update_real(const GemmArgs &g, int64_t i, int64_t j, T acc) {
    if (i >= g.m || j >= g.n) return;
    const int64_t off = c_offset<GS>(g, i, j);
    const T ax = (T)g.alpha_re;
    if (HC && g.c_half) {
        // beta is already binary16, so beta*C is exact in the computation
        // type; the update is formed exactly and rounded once to binary16
        // (in double for the double precision, else a round-to-odd float)
        _Float16 *c = (_Float16 *)g.C;
        const T t = ax * acc;
        if (g.beta_zero) {
            c[off] = half_rn(t);
        } else {
            const T bc = (T)g.beta_re * (T)((const _Float16 *)g.Cin)[off];
            if constexpr (sizeof(T) == 8) c[off] = half_rn(bc + t);
            else c[off] = (_Float16)add_rto(bc, t);
        }
        return;
    }
    if (g.c_dbl) {
        double *c = (double *)g.C;
        const double *cin = (const double *)g.Cin;
        const double t = (double)ax * (double)acc;
        c[off] = g.beta_zero ? t : fma(g.beta_re, cin[off], t);
    } else {
        float *c = (float *)g.C;
        const float *cin = (const float *)g.Cin;
        const float bc = (float)g.beta_re;
        if constexpr (sizeof(T) == 8) {
            const double t = ax * acc;
            c[off] = (float)(g.beta_zero ? t : fma((double)bc, (double)cin[off], t));
        } else {
            const float t = ax * acc;
            c[off] = g.beta_zero ? t : fmaf(bc, cin[off], t);
        }
    }
}

// Complex C: (re, im) is alpha-free AB for this element (im == 0 in case 1c).
template <class T, class W>
__device__ __forceinline__ void cupdate(const GemmArgs &g, W *c2, const W *cin2, W re, W im, W ar, W ai) {
    const W tr = fma(ar, re, -(ai * im));
    const W ti = fma(ar, im, ai * re);
    if (g.beta_zero) {
        c2[0] = tr;
        c2[1] = ti;
    } else {
        const W br = (W)g.beta_re, bi = (W)g.beta_im;
        const W cr = cin2[0], ci = cin2[1];
        c2[0] = fma(br, cr, fma(-bi, ci, tr));
        c2[1] = fma(br, ci, fma(bi, cr, ti));
    }
}

template <class T, bool GS = false, bool HC = false>
__device__ __forceinline__ void update_cplx(const GemmArgs &g, int64_t i, int64_t j, T re, T im) {
    if (i >= g.m || j >= g.n) return;
    const int64_t off = 2 * c_offset<GS>(g, i, j);
    const T ar = (T)g.alpha_re, ai = (T)g.alpha_im;
    if (HC && g.c_half) {
        // alpha*AB in the computation precision; beta and C are binary16, so
        // each product beta_x * c_y is exact in the computation type and the
        // update of each part (up to three terms) is formed exactly and
        // rounded once to binary16 (in double for the double precision, else
        // through a round-to-odd float)
        _Float16 *c = (_Float16 *)g.C + off;
        const _Float16 *cin = (const _Float16 *)g.Cin + off;
        const T tr = fma(ar, re, -(ai * im));
        const T ti = fma(ar, im, ai * re);
        if (g.beta_zero) {
            c[0] = half_rn(tr);
            c[1] = half_rn(ti);
            return;
        }
        const T br = (T)g.beta_re, bi = (T)g.beta_im, cr = (T)cin[0], ci = (T)cin[1];
        if constexpr (sizeof(T) == 8) {
            c[0] = half_rn(fma(br, cr, fma(-bi, ci, tr)));
            c[1] = half_rn(fma(br, ci, fma(bi, cr, ti)));
        } else if (bi == 0.0f) {
            c[0] = (_Float16)add_rto(br * cr, tr);
            c[1] = (_Float16)add_rto(br * ci, ti);
        } else {
            c[0] = (_Float16)add3_rto(br * cr, -(bi * ci), tr);
            c[1] = (_Float16)add3_rto(br * ci, bi * cr, ti);
        }
        return;
    }
    if (g.c_dbl) {
        double *c = (double *)g.C + off;
        // beta is already double (C's precision); product in double.
        cupdate<T, double>(g, c, (const double *)g.Cin + off, (double)re, (double)im, (double)ar, (double)ai);
    } else if constexpr (sizeof(T) == 8) {
        // computation in double, C single: beta cast to single, update in double
        float *c = (float *)g.C + off;
        const float *cin = (const float *)g.Cin + off;
        const double br = (double)(float)g.beta_re, bi = (double)(float)g.beta_im;
        const double tr = fma(ar, re, -(ai * im));
        const double ti = fma(ar, im, ai * re);
        double rr = tr, ri = ti;
        if (!g.beta_zero) {
            const double cr = cin[0], ci = cin[1];
            rr = fma(br, cr, fma(-bi, ci, tr));
            ri = fma(br, ci, fma(bi, cr, ti));
        }
        c[0] = (float)rr;
        c[1] = (float)ri;
    } else {
        float *c = (float *)g.C + off;
        cupdate<T, float>(g, c, (const float *)g.Cin + off, re, im, ar, ai);
    }
}

// ---------------------------------------------------------------------------
// The product kernel
// ---------------------------------------------------------------------------
// MFMA fragments.  Within a "k group" of KV = 16/sizeof(T) consecutive
// k-steps, lane group g = lane >> 4 of step j multiplies k' = 4*KV*grp +
// KV*g + j -- the same mapping for A' and B' -- so an operand kept as [mn][k]
// delivers a whole group with one 16-byte LDS read per block, while an operand
// kept as [k][mn] is read one element per block and step.  Two buffers: the
// fragments of step s+1 are read while step s multiplies.
template <class T, bool MNC, int BMN, int NB, class C>
struct Frag {
    typedef Lay<T, MNC, BMN, C> L;
    static constexpr int KV = 16 / (int)sizeof(T);
    static constexpr int NE = MNC ? 1 : KV;
    T f[2][NB][NE];
    // Read what step s needs (for [mn][k]: its whole group, at the group's first step).
    __device__ __forceinline__ void read(const T *lds, int s, int lane, int w0) {
        const int g = lane >> 4, r = lane & 15;
        if constexpr (MNC) {
            const int row = (s / KV) * 4 * KV + KV * g + (s % KV);
#pragma unroll
            for (int i = 0; i < NB; ++i) f[s & 1][i][0] = lds[L::at(row, w0 + 16 * i + r)];
        } else {
            if (s % KV != 0) return;
            typedef T vec_t __attribute__((ext_vector_type(KV)));
            const int grp = s / KV;
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const vec_t x = *(const vec_t *)&lds[L::at(4 * KV * grp + KV * g, w0 + 16 * i + r)];
#pragma unroll
                for (int j = 0; j < KV; ++j) f[grp & 1][i][j] = x[j];
            }
        }
    }
    __device__ __forceinline__ T get(int s, int i) const {
        if constexpr (MNC) return f[s & 1][i][0];
        else return f[(s / KV) & 1][i][s % KV];
    }
};

// Order of the k loop (C::PIPE).  Early store: each iteration first writes
// the staged registers (tile t+1) to the free LDS buffer and at once issues
// the global loads of tile t+2, so a load has a whole iteration of MFMAs to
// arrive.  Late store: the staged tile is written during the last k-step and
// the next loads follow the barrier.  Measured at m=n=k=4096: early store is
// faster for every configuration except FP64 on 4 waves (late store up to 5 %
// faster there).

// SCL: the complex operand of case 1a, 2ab (A) or 1b (B) is staged scaled by
// the complex alpha (GemmArgs::scale_re/scale_im).  SH: A and B are both
// binary16 (fast path).
template <class T, int CS, bool FAST, bool AD, bool BD, bool AMNC, bool BMNC, class C = TileCfg<T>,
          bool RAG = false, bool SCL = false, bool SH = false>
__global__ __launch_bounds__(C::NT, C::OCC) void md_gemm_kernel(GemmArgs g) {
    typedef Stage<T, CS, true, FAST, AD, AMNC, C, RAG, SCL && CS != MD_CASE_1B, false, SH> SA;
    typedef Stage<T, CS, false, FAST, BD, BMNC, C, RAG, SCL && CS == MD_CASE_1B, false, SH> SB;
    constexpr bool PIPE = C::PIPE;
    constexpr int WMB = C::WMB, WNB = C::WNB;
    typedef typename AccT<T>::type acc_t;
    static_assert(SA::TK == SB::TK, "A and B disagree on the k lowering");
    constexpr bool MDBL = SA::MN2, NDBL = SB::MN2;
    constexpr bool CCPLX = (CS == MD_CASE_1C || CS == MD_CASE_2AC || CS == MD_CASE_2BC || CS == MD_CASE_3);

    __shared__ __attribute__((aligned(16))) T sA[2][SA::L::SIZE];
    __shared__ __attribute__((aligned(16))) T sB[2][SB::L::SIZE];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % C::WGM) * (C::BM / C::WGM), wn0 = (wave / C::WGM) * (C::BN / C::WGN);
    // With g.splits > 1 the workgroups of one tile take consecutive ranges of
    // its k-tiles and store their partial products (md_split_reduce finishes).
    const int nsplit = g.splits > 1 ? g.splits : 1;
    const int split = (int)(blockIdx.x % nsplit);
    int tm, tn;
    map_tile(blockIdx.x / nsplit, gridDim.x / nsplit, g.tiles_m, g.tiles_n, &tm, &tn);
    const int64_t mn0a = (int64_t)tm * SA::TMN, mn0b = (int64_t)tn * SB::TMN;
    const int nk_all = (int)((g.k + SA::TK - 1) / SA::TK);
    const int t0 = (int)((int64_t)nk_all * split / nsplit);
    const int nk = (int)((int64_t)nk_all * (split + 1) / nsplit) - t0;

    acc_t acc[WMB][WNB];
#pragma unroll
    for (int a = 0; a < WMB; ++a)
#pragma unroll
        for (int b = 0; b < WNB; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    SA la(g, tid, mn0a);
    SB lb(g, tid, mn0b);
    Frag<T, AMNC, C::BM, WMB, C> fa;
    Frag<T, BMNC, C::BN, WNB, C> fb;
    constexpr int S = C::BK / 4;  // MFMA k-steps per LDS tile

    // One LDS tile of S k-steps of 16 MFMAs.  The fragments of step s+1 are
    // read while step s multiplies; with STORE the next tile's staged
    // registers are converted and written to the other LDS buffer during the
    // last step.
    auto tile = [&](int cur, auto store_tag, int next_load) {
        constexpr bool STORE = decltype(store_tag)::value;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (PIPE && STORE && s == 0) {
                la.store(sA[cur ^ 1]);
                lb.store(sB[cur ^ 1]);
                if (next_load < nk) {
                    la.load(t0 + next_load);
                    lb.load(t0 + next_load);
                }
            }
            if (s + 1 < S) {
                fa.read(sA[cur], s + 1, lane, wm0);
                fb.read(sB[cur], s + 1, lane, wn0);
            }
            if (!PIPE && STORE && s == S - 1) {
                la.store(sA[cur ^ 1]);
                lb.store(sB[cur ^ 1]);
            }
#pragma unroll
            for (int a = 0; a < WMB; ++a)
#pragma unroll
                for (int b = 0; b < WNB; ++b) acc[a][b] = mfma16(fb.get(s, b), fa.get(s, a), acc[a][b]);
        }
    };

    la.load(t0);
    lb.load(t0);
    la.store(sA[0]);
    lb.store(sB[0]);
    __syncthreads();
    if (nk > 1) {
        la.load(t0 + 1);
        lb.load(t0 + 1);
    }
    fa.read(sA[0], 0, lane, wm0);
    fb.read(sB[0], 0, lane, wn0);
    int t = 0;
    for (; t + 1 < nk; ++t) {
        const int cur = t & 1;
        tile(cur, std::true_type{}, t + 2);
        __syncthreads();
        if (!PIPE && t + 2 < nk) {
            la.load(t0 + t + 2);
            lb.load(t0 + t + 2);
        }
        fa.read(sA[cur ^ 1], 0, lane, wm0);
        fb.read(sB[cur ^ 1], 0, lane, wn0);
    }
    tile(t & 1, std::false_type{}, nk);

    // Epilogue.  acc[a][b] item v is C'(row m = wm0 + 16a + (lane & 15),
    //                                   col n = wn0 + 16b + acc_row(lane, v)).
    // A split workgroup stores its partial (re, im) instead.  Split and
    // binary16-C stores are decided once per workgroup, so the common case
    // keeps the plain epilogue's code.  Where a thread holds many
    // accumulators the general update is too large to inline at each: its
    // loop over row blocks stays rolled and picks the accumulator with
    // selects (an indexed access would put the accumulators in scratch).
    auto epilogue = [&](auto general_tag) {
        constexpr bool GEN = decltype(general_tag)::value;
        auto put_cplx = [&](int64_t i, int64_t j, T re, T im) {
            if constexpr (GEN) {
                if (nsplit > 1) store_partial(g, split, i, j, re, im);
                else update_cplx<T, !FAST, true>(g, i, j, re, im);
            } else {
                update_cplx<T, !FAST, false>(g, i, j, re, im);
            }
        };
        auto put_real = [&](int64_t i, int64_t j, T re) {
            if constexpr (GEN) {
                if (nsplit > 1) store_partial(g, split, i, j, re, (T)0);
                else update_real<T, !FAST, true>(g, i, j, re);
            } else {
                update_real<T, !FAST, false>(g, i, j, re);
            }
        };
        auto pick = [&](int a, int b, int v) {
            T r = acc[0][b][v];
#pragma unroll
            for (int x = 1; x < WMB; ++x) r = (a == x) ? acc[x][b][v] : r;
            return r;
        };
        // general updates per thread: rolled from 64 on
        constexpr int NCALL = WNB * 4 * (MDBL ? WMB / 2 : WMB) / (NDBL ? 2 : 1);
        constexpr bool ROLL = GEN && NCALL >= 64;
        auto rows = [&](int count, auto fn) {
            if constexpr (ROLL) {
#pragma unroll 1
                for (int a = 0; a < count; ++a) fn(a);
            } else {
#pragma unroll
                for (int a = 0; a < count; ++a) fn(a);
            }
        };
        const int ml = lane & 15;
#pragma unroll
        for (int b = 0; b < WNB; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int nl = acc_row<T>(lane, v);
                if constexpr (MDBL) {
                    rows(WMB / 2, [&](int q) {
                        const int64_t i = (int64_t)tm * SA::TMN + wm0 / 2 + q * 16 + ml;
                        const int64_t j = (int64_t)tn * SB::TMN + wn0 + b * 16 + nl;
                        put_cplx(i, j, pick(2 * q, b, v), pick(2 * q + 1, b, v));
                    });
                } else if constexpr (NDBL) {
                    if ((b & 1) == 0) {
                        rows(WMB, [&](int a) {
                            const int64_t i = (int64_t)tm * SA::TMN + wm0 + a * 16 + ml;
                            const int64_t j = (int64_t)tn * SB::TMN + wn0 / 2 + (b / 2) * 16 + nl;
                            put_cplx(i, j, pick(a, b, v), pick(a, b + 1, v));
                        });
                    }
                } else {
                    rows(WMB, [&](int a) {
                        const int64_t i = (int64_t)tm * SA::TMN + wm0 + a * 16 + ml;
                        const int64_t j = (int64_t)tn * SB::TMN + wn0 + b * 16 + nl;
                        if constexpr (CCPLX) put_cplx(i, j, pick(a, b, v), (T)0);
                        else put_real(i, j, pick(a, b, v));
                    });
                }
            }
        }
    };
    if (nsplit > 1 || g.c_half) epilogue(std::true_type{});
    else epilogue(std::false_type{});
}

}  // namespace md
