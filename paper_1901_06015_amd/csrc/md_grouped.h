// md_grouped.h -- the persistent kernel behind mdgemm_grouped: many products
// of uneven shapes and mixed storage types / computation precisions in ONE
// launch.
//
// The host builds a work table (one GDesc per product, one GTile per output
// tile, largest work first) and the kernel's workgroups pop tile indices from
// an atomic counter until the table is exhausted.  Because one launch mixes
// every variant, the tile routine decodes the domain case, the storage
// precisions and the operand orientation at run time, element by element
// (`GStager`), instead of using the specialised staging of md_tile.h; the
// lowering it realises is the same (Figure "mixeddom" cases onto one real
// product, Re/Im split in blocks of 16, 1e/1r arrangement for case 3), and the
// epilogue is md_tile.h's.
#pragma once
#include "md_tile.h"
#include "md_tile_bf16.h"

namespace md {

// Tile configurations of the grouped kernel (the md_gtile values of
// mdgemm.h): real-product workgroup tile and k-tile depth.
enum { GCFG_64 = MD_GTILE_64x64, GCFG_128 = MD_GTILE_128x128, GCFG_128x64 = MD_GTILE_128x64,
       GCFG_64x128 = MD_GTILE_64x128, GCFG_64K = MD_GTILE_64x64_DEEPK, GCFG_COUNT = MD_GTILE_COUNT };
// workgroup tile edges along m' and n' of each configuration
constexpr int gcfg_bm(int c) { return (c == GCFG_128 || c == GCFG_128x64) ? 128 : 64; }
constexpr int gcfg_bn(int c) { return (c == GCFG_128 || c == GCFG_64x128) ? 128 : 64; }

struct GDesc {
    GemmArgs g;
    int prec;   // PREC_S / PREC_D / PREC_BF16X3
    int cs;     // md_case
    int cfg;    // GCFG_*
    int kind;   // 0: product; 1: C := beta*C only (alpha == 0 or k == 0)
    int tiles_m, tiles_n;
};

struct GTile {
    int desc, tm, tn, pad;
};

// Threads of a grouped workgroup: 8 waves (two workgroups per CU, four
// waves per SIMD; every tile routine fits 128 registers per lane).
constexpr int GNT = 512;

// Shape of a grouped tile routine: BM x BN real-product tile, k-tile depth
// BK (sized so that the staged words fit the register budget), the 8 waves
// as WGM x WGN wave tiles of
// WMB x WNB 16x16 blocks and KG = 8 / (WGM * WGN) groups that split each
// k-tile's steps (summed through LDS before the epilogue).  Every wave holds
// at least 2 x 2 blocks so that the Re and Im blocks of an m- or n-doubled
// operand meet in one wave's accumulators.  LDS: two stages of A' and B' as
// [k][mn] with padded rows.
template <class T, int BM_, int BN_, int WGM_, int WGN_, int BK_>
struct GShape {
    static constexpr int BM = BM_, BN = BN_, WGM = WGM_, WGN = WGN_;
    static constexpr int KG = 8 / (WGM * WGN);
    static constexpr int WMB = BM / (16 * WGM), WNB = BN / (16 * WGN);
    static constexpr int BK = BK_;
    static constexpr int PAD = sizeof(T) == 8 ? 8 : 4;
    static constexpr int LDA = BM + PAD, LDB = BN + PAD;
    static constexpr int STAGE = BK * (LDA + LDB);  // elements of T per stage (A' then B')
    static constexpr int SMEM = 2 * STAGE * (int)sizeof(T);
    static constexpr int EA = BM * BK / GNT, EB = BN * BK / GNT;  // staged elements per thread
    static_assert(KG * WGM * WGN == 8 && WMB >= 2 && WNB >= 2 && WMB % 2 == 0 && WNB % 2 == 0, "wave tiling");
    static_assert(EA * GNT == BM * BK && EB * GNT == BN * BK, "staging");
    static_assert((BK / 4) % KG == 0, "k-steps split evenly between the groups");
    // the k-groups' partial sums go through the (then free) staging LDS
    static_assert(KG == 1 || (KG - 1) * (8 / KG) * 64 * WMB * WNB * 4 * (int)sizeof(T) <= SMEM, "reduction");
};
// the shapes of each configuration (GCFG_*), single and double
typedef GShape<float, 64, 64, 2, 2, 32> GS_S64;
typedef GShape<float, 128, 128, 2, 4, 16> GS_S128;
typedef GShape<float, 128, 64, 4, 2, 32> GS_S128x64;
typedef GShape<float, 64, 128, 2, 4, 32> GS_S64x128;
typedef GShape<float, 64, 64, 2, 2, 64> GS_S64K;
typedef GShape<double, 64, 64, 2, 2, 16> GS_D64;
typedef GShape<double, 128, 128, 2, 4, 8> GS_D128;
typedef GShape<double, 128, 64, 4, 2, 16> GS_D128x64;
typedef GShape<double, 64, 128, 2, 4, 16> GS_D64x128;
typedef GShape<double, 64, 64, 2, 2, 32> GS_D64K;
// BF16x3: 64 x 64 tiles, four bf16 planes (A hi/lo, B hi/lo) of BK3 = 64 k
// each per stage, one 16x16x32 step per k-group.
constexpr int BK3 = 64, LDW3 = 64 + 4;
constexpr int BF16X3_GROUPED_SMEM = 2 * 4 * BK3 * LDW3 * 2;
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int GROUPED_SMEM =
    cmax(cmax(cmax(cmax(GS_S64::SMEM, GS_S128::SMEM), cmax(GS_S128x64::SMEM, GS_S64x128::SMEM)),
              cmax(cmax(GS_D64::SMEM, GS_D128::SMEM), cmax(GS_D128x64::SMEM, GS_D64x128::SMEM))),
         cmax(cmax(GS_S64K::SMEM, GS_D64K::SMEM), BF16X3_GROUPED_SMEM));
static_assert(2 * GROUPED_SMEM <= 160 * 1024, "two grouped workgroups per CU");

// Runtime description of one staged operand (A' or B').
struct GOp {
    const char *base;
    int64_t ld, MN, K;
    int mode;
    bool dbl, cplx, mnc, conj, kneg;
};

__device__ __forceinline__ int mode_rt(int cs, bool is_a) {
    if (is_a) {
        return cs == MD_CASE_1A ? M_REONLY
             : cs == MD_CASE_2AB ? M_KINT
             : cs == MD_CASE_2AC ? M_MNINT
             : cs == MD_CASE_3 ? M_ONEE : M_PLAIN;
    }
    return cs == MD_CASE_1B ? M_REONLY
         : (cs == MD_CASE_2AB || cs == MD_CASE_3) ? M_KINT
         : cs == MD_CASE_2BC ? M_MNINT : M_PLAIN;
}

__device__ __forceinline__ GOp make_gop(const GemmArgs &g, int cs, bool is_a) {
    GOp o;
    const int tr = is_a ? g.ta : g.tb;
    o.base = (const char *)(is_a ? g.A : g.B);
    o.ld = is_a ? g.lda : g.ldb;
    o.MN = is_a ? g.m : g.n;
    o.K = g.k;
    o.mode = mode_rt(cs, is_a);
    o.dbl = is_a ? g.a_dbl : g.b_dbl;
    o.cplx = o.mode != M_PLAIN;
    o.mnc = is_a ? (tr == 0 || tr == 3) : (tr == 1 || tr == 2);
    o.conj = tr >= 2;
    o.kneg = is_a;
    return o;
}

__device__ __forceinline__ bool gop_mn2(const GOp &o) { return o.mode == M_MNINT || o.mode == M_ONEE; }
__device__ __forceinline__ bool gop_k2(const GOp &o) { return o.mode == M_KINT || o.mode == M_ONEE; }

// The thread index, read afresh by each tile routine for everything
// lane-dependent: the persistent loop runs many routines, and without this the
// compiler hoists every routine's lane-dependent constants (staging slots,
// fragment addresses) out of the loop, keeping them all live at once (far
// beyond the register budget).
__device__ __forceinline__ int tile_tid() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Raw stored words of one staged element: one word for single storage, a
// register pair for double storage (loaded with one 64-bit load).
template <bool DBL> struct RawT { typedef uint32_t type; };
template <> struct RawT<true> { typedef uint64_t type; };

// Per-thread staging plan for the E elements a thread moves per k-tile of a
// BMN x BK tile, everything that depends on the operand's lowering
// (orientation, Re/Im split, k interleave, signs) decided once per tile in
// init():
//   off[e]  byte offset of element e's stored component from the tile's
//           origin at k-tile 0 (32-bit: the host keeps products whose leading
//           dimensions could overflow it out of the grouped launch), or an
//           offset beyond every resource when it lies outside the matrix;
//   ks[e]   bits 0-23: its LDS byte offset inside the operand's stage
//           ([k][mn], row stride LDW elements of LSZ bytes); bits 24-30: its
//           stored k index inside the k-tile;
//   negm    bit e: it enters negated.
// Consecutive lanes take consecutive elements along the operand's contiguous
// dimension in HBM (m/n for an m/n-contiguous operand, k otherwise), so every
// load instruction reads whole cache lines.  Loads go through a buffer
// resource that starts at the k-tile's origin and ends at the matrix's last
// byte: an element past the matrix's end reads zero.  That also bounds k for
// an m/n-contiguous operand; a k-contiguous one compares k indices (only the
// last k-tile can fail the compare).
template <int E, int BMN, int BK, int LDW, int LSZ>
struct GStager {
    const char *base;
    int off[E];
    int ks[E];
    uint32_t negm;
    int64_t tile0;   // bytes from the matrix origin to the tile's origin at k-tile 0
    int64_t kbytes;  // bytes between consecutive k-tiles
    int64_t total;   // bytes from the matrix origin to its end
    int64_t K;
    int tk;
    bool kchk;       // k-contiguous: the last k-tile checks k
    static_assert(BK < 128 && 2 * BK * LDW * LSZ < (1 << 24), "ks fields");
    __device__ __forceinline__ void init(const GOp &o, int64_t mn0, int tk_, int tid) {
        base = o.base;
        K = o.K;
        tk = tk_;
        kchk = !o.mnc;
        const int W = o.cplx ? 2 : 1, esz = o.dbl ? 8 : 4;
        const int64_t rows_st = o.mnc ? o.MN : o.K, cols_st = o.mnc ? o.K : o.MN;
        total = ((cols_st - 1) * o.ld + rows_st) * W * esz;
        tile0 = (o.mnc ? mn0 : mn0 * o.ld) * W * esz;
        kbytes = (int64_t)tk * (o.mnc ? o.ld : 1) * W * esz;
        negm = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = tid + e * GNT;
            const int kr = o.mnc ? idx / BMN : idx % BK, mr = o.mnc ? idx % BMN : idx / BK;
            int i = mr, qm = 0;
            if (gop_mn2(o)) {
                const int blk = mr >> 4;
                qm = blk & 1;
                i = ((blk >> 1) << 4) | (mr & 15);
            }
            int p = kr, qk = 0;
            if (gop_k2(o)) {
                p = kr >> 1;
                qk = kr & 1;
            }
            int comp = 0;
            bool ng = false;
            if (o.mode == M_KINT) {
                comp = qk;
                ng = qk && o.kneg;
            } else if (o.mode == M_MNINT) {
                comp = qm;
            } else if (o.mode == M_ONEE) {
                comp = qm ^ qk;
                ng = (qm == 0 && qk == 1);
            }
            if (comp == 1 && o.conj) ng = !ng;
            if (ng) negm |= 1u << e;
            const int64_t rel = o.mnc ? ((int64_t)i + (int64_t)p * o.ld) : ((int64_t)p + (int64_t)i * o.ld);
            off[e] = (mn0 + i < o.MN) ? (int)((rel * W + comp) * esz) : (int)0x80000000;
            ks[e] = (p << 24) | ((kr * LDW + mr) * LSZ);
        }
    }
    // Issue the loads of the E elements of k-tile t (converted only where
    // they are stored, a k-tile later).
    template <bool DBL>
    __device__ __forceinline__ void issue(int t, typename RawT<DBL>::type (&r)[E]) const {
        const int64_t b = tile0 + (int64_t)t * kbytes;
        const int64_t rem = total - b;
        const int nrec = rem > 0x7fffffffLL ? 0x7fffffff : (rem < 0 ? 0 : (int)rem);
        __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)(base + b), (short)0, nrec, 0x00020000);
        auto load = [&](int e, int o) {
            if constexpr (DBL) r[e] = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(rs, o, 0, 0));
            else r[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, o, 0, 0);
        };
        // branch-free k check: ks[e] holds the element's k index in its top
        // bits, so one unsigned compare with the (uniform) cap decides; the
        // cap passes everything for full k-tiles and m/n-contiguous operands
        const int64_t kl = K - (int64_t)t * tk;
        const uint32_t kcap = (kchk && kl < tk) ? (uint32_t)kl << 24 : 0xffffffffu;
#pragma unroll
        for (int e = 0; e < E; ++e) load(e, (uint32_t)ks[e] < kcap ? off[e] : (int)0x80000000);
    }
    // Element e of an issued k-tile, signed (a sign-bit flip, exact either
    // side of the rounding) and converted to T (float -> double is exact,
    // double -> float rounds to nearest even).
    template <class T, bool DBL>
    __device__ __forceinline__ T value(int e, typename RawT<DBL>::type r) const {
        const uint32_t sg = ((negm >> e) & 1u) << 31;
        if constexpr (DBL) return (T)__builtin_bit_cast(double, r ^ ((uint64_t)sg << 32));
        else return (T)__builtin_bit_cast(float, r ^ sg);
    }
    // LDS byte offset of element e inside its operand's stage.
    __device__ __forceinline__ int lds_byte(int e) const { return ks[e] & 0xffffff; }
};

// Raw words of a staged k-tile, pinned where they are converted: the loads
// were issued a k-tile earlier, and this keeps the compiler from converting
// (and so waiting for) them right after issuing them.
template <int E, class R>
__device__ __forceinline__ void pin_raw(R (&r)[E]) {
#pragma unroll
    for (int e = 0; e < E; ++e) asm("" : "+v"(r[e]));
}

// Epilogue shared by the grouped tile routines: acc[a][b] item v is
// C'(m = wm0 + 16a + (lane & 15), n = wn0 + 16b + acc_row(lane, v)).
template <class T, class ACC, int WMB, int WNB>
__device__ __forceinline__ void grouped_epilogue(const GemmArgs &g, bool mdbl, bool ndbl, bool ccplx,
                                                 int64_t i0, int64_t j0, int wm0, int wn0, int lane,
                                                 ACC (&acc)[WMB][WNB]) {
    const int ml = lane & 15;
#pragma unroll
    for (int b = 0; b < WNB; ++b) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int nl = acc_row<T>(lane, v);
            if (mdbl) {
#pragma unroll
                for (int q = 0; q < WMB / 2; ++q) {
                    const int64_t i = i0 + wm0 / 2 + q * 16 + ml;
                    const int64_t j = j0 + wn0 + b * 16 + nl;
                    update_cplx<T>(g, i, j, acc[2 * q][b][v], acc[2 * q + 1][b][v]);
                }
            } else if (ndbl) {
                if ((b & 1) == 0) {
#pragma unroll
                    for (int a = 0; a < WMB; ++a) {
                        const int64_t i = i0 + wm0 + a * 16 + ml;
                        const int64_t j = j0 + wn0 / 2 + (b / 2) * 16 + nl;
                        update_cplx<T>(g, i, j, acc[a][b][v], acc[a][b + 1][v]);
                    }
                }
            } else {
#pragma unroll
                for (int a = 0; a < WMB; ++a) {
                    const int64_t i = i0 + wm0 + a * 16 + ml;
                    const int64_t j = j0 + wn0 + b * 16 + nl;
                    if (ccplx) update_cplx<T>(g, i, j, acc[a][b][v], (T)0);
                    else update_real<T>(g, i, j, acc[a][b][v]);
                }
            }
        }
    }
}

// With KG = 2 the waves of k-group 1 add their partial accumulators into
// k-group 0's through LDS (the staging buffers, free after the k loop's last
// barrier); group 0 then runs the epilogue.  Returns whether this wave holds
// the sums.
template <class T, class ACC, int KG, int WMB, int WNB>
__device__ __forceinline__ bool grouped_reduce(ACC (&acc)[WMB][WNB], T *red, int wave, int lane) {
    if constexpr (KG == 1) {
        return true;
    } else {
        constexpr int NV = WMB * WNB * 4, WPG = 8 / KG;
        const int kg = wave / WPG, w = wave % WPG;
        if (kg == 1) {
#pragma unroll
            for (int a = 0; a < WMB; ++a)
#pragma unroll
                for (int b = 0; b < WNB; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v) red[(w * NV + (a * WNB + b) * 4 + v) * 64 + lane] = acc[a][b][v];
        }
        __syncthreads();
        if (kg == 0) {
#pragma unroll
            for (int a = 0; a < WMB; ++a)
#pragma unroll
                for (int b = 0; b < WNB; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[a][b][v] += red[(w * NV + (a * WNB + b) * 4 + v) * 64 + lane];
        }
        return kg == 0;
    }
}

// One output tile of a product computed in T (float or double) with FP32 /
// FP64 MFMA, in the shape SH (GShape).  LDS holds one k-tile of A' and B' as
// [k][mn]; the next k-tile's elements are loaded into registers during the
// MFMAs.
template <class T, class SH, bool AD, bool BD>
__device__ __forceinline__ void grouped_tile(const GDesc &d, int tm, int tn, char *smem) {
    typedef typename AccT<T>::type acc_t;
    constexpr int BM = SH::BM, BN = SH::BN, BK = SH::BK, LDA = SH::LDA, LDB = SH::LDB;
    constexpr int WMB = SH::WMB, WNB = SH::WNB, KG = SH::KG, EA = SH::EA, EB = SH::EB;
    constexpr int S = BK / 4, SG = S / KG;  // k-steps per k-tile, per k-group
    static_assert(SH::SMEM <= GROUPED_SMEM, "grouped LDS too small");
    T *const buf = (T *)smem;  // stage s: A' at buf + s*STAGE, B' BK*LDA further
    const GemmArgs &g = d.g;
    const GOp oa = make_gop(g, d.cs, true), ob = make_gop(g, d.cs, false);
    const bool mdbl = gop_mn2(oa), ndbl = gop_mn2(ob), kdbl = gop_k2(oa);
    const bool ccplx = g.c_cplx;
    const int tmn_a = mdbl ? BM / 2 : BM, tmn_b = ndbl ? BN / 2 : BN, tk = kdbl ? BK / 2 : BK;
    const int64_t mn0a = (int64_t)tm * tmn_a, mn0b = (int64_t)tn * tmn_b;
    const int nk = (int)((g.k + tk - 1) / tk);
    // lane-derived values from the per-tile thread index (see tile_tid)
    const int stid = tile_tid(), lane = stid & 63, wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int wg = wave % (SH::WGM * SH::WGN), kg = wave / (SH::WGM * SH::WGN);
    const int wm0 = (wg % SH::WGM) * 16 * WMB, wn0 = (wg / SH::WGM) * 16 * WNB;

    acc_t acc[WMB][WNB];
#pragma unroll
    for (int a = 0; a < WMB; ++a)
#pragma unroll
        for (int b = 0; b < WNB; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    GStager<EA, BM, BK, LDA, sizeof(T)> sa;
    GStager<EB, BN, BK, LDB, sizeof(T)> sb;
    sa.init(oa, mn0a, tk, stid);
    sb.init(ob, mn0b, tk, stid);
    typename RawT<AD>::type ra[EA];
    typename RawT<BD>::type rb[EB];
    auto issue = [&](int t) {
        sa.template issue<AD>(t, ra);
        sb.template issue<BD>(t, rb);
    };
    auto store = [&](int stage) {
        pin_raw(ra);
        pin_raw(rb);
        char *la = (char *)(buf + stage * SH::STAGE), *lb = la + BK * LDA * (int)sizeof(T);
#pragma unroll
        for (int e = 0; e < EA; ++e) *(T *)(la + sa.lds_byte(e)) = sa.template value<T, AD>(e, ra[e]);
#pragma unroll
        for (int e = 0; e < EB; ++e) *(T *)(lb + sb.lds_byte(e)) = sb.template value<T, BD>(e, rb[e]);
    };

    // Two LDS stages and one k-tile of loads in flight: iteration t first
    // writes the raw words of tile t+1 (issued during iteration t-1) to the
    // free stage (last read before the previous barrier), then issues the
    // loads of tile t+2, then multiplies its k-group's steps of tile t, so
    // every load has a whole k-tile of MFMAs to arrive; one barrier per
    // k-tile.
    issue(0);
    store(0);
    if (nk > 1) issue(1);
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        const T *la = buf + (t & 1) * SH::STAGE, *lb = la + BK * LDA;
        if (t + 1 < nk) store((t + 1) & 1);
        if (t + 2 < nk) issue(t + 2);
#pragma unroll
        for (int s = 0; s < SG; ++s) {
            const int kr = (kg * SG + s) * 4 + (lane >> 4);
            T fa[WMB], fb[WNB];
#pragma unroll
            for (int i = 0; i < WMB; ++i) fa[i] = la[kr * LDA + wm0 + 16 * i + (lane & 15)];
#pragma unroll
            for (int i = 0; i < WNB; ++i) fb[i] = lb[kr * LDB + wn0 + 16 * i + (lane & 15)];
#pragma unroll
            for (int a = 0; a < WMB; ++a)
#pragma unroll
                for (int b = 0; b < WNB; ++b) acc[a][b] = mfma16(fb[b], fa[a], acc[a][b]);
        }
        __syncthreads();
    }
    if (grouped_reduce<T, acc_t, KG, WMB, WNB>(acc, buf, wave, lane))
        grouped_epilogue<T, acc_t, WMB, WNB>(g, mdbl, ndbl, ccplx, (int64_t)tm * tmn_a, (int64_t)tn * tmn_b, wm0,
                                             wn0, lane, acc);
}

// BF16x3 form of grouped_tile: single-precision semantics from three bf16
// products per 16x16x32 block (see md_tile_bf16.h).  64 x 64 tiles, 2 x 2
// waves of 32 x 32 in two k-groups, one 16x16x32 step each per 64-deep
// k-tile.
template <bool AD, bool BD>
__device__ __forceinline__ void grouped_tile_bf16x3(const GDesc &d, int tm, int tn, char *smem) {
    constexpr int BM = 64, BN = 64, BK = BK3, LDW = LDW3, PLANE = BK * LDW, STAGE = 4 * PLANE;
    constexpr int WMB = 2, WNB = 2, KG = 2;
    static_assert(2 * STAGE * 2 <= GROUPED_SMEM, "grouped LDS too small");
    static_assert(KG * 4 * 64 * WMB * WNB * 4 * 4 <= 2 * STAGE * 2, "reduction");
    constexpr int EA = BM * BK / GNT, EB = BN * BK / GNT;
    __bf16 *const buf = (__bf16 *)smem;  // stage s: planes Ah, Al, Bh, Bl
    const GemmArgs &g = d.g;
    const GOp oa = make_gop(g, d.cs, true), ob = make_gop(g, d.cs, false);
    const bool mdbl = gop_mn2(oa), ndbl = gop_mn2(ob), kdbl = gop_k2(oa);
    const bool ccplx = g.c_cplx;
    const int tmn_a = mdbl ? BM / 2 : BM, tmn_b = ndbl ? BN / 2 : BN, tk = kdbl ? BK / 2 : BK;
    const int64_t mn0a = (int64_t)tm * tmn_a, mn0b = (int64_t)tn * tmn_b;
    const int nk = (int)((g.k + tk - 1) / tk);
    // lane-derived values from the per-tile thread index (see tile_tid)
    const int stid = tile_tid(), lane = stid & 63, wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int wg = wave & 3, kg = wave >> 2;
    const int wm0 = (wg & 1) * 16 * WMB, wn0 = (wg >> 1) * 16 * WNB;

    v4f acc[WMB][WNB];
#pragma unroll
    for (int a = 0; a < WMB; ++a)
#pragma unroll
        for (int b = 0; b < WNB; ++b) acc[a][b] = v4f{0, 0, 0, 0};

    GStager<EA, BM, BK, LDW, 2> sa;
    GStager<EB, BN, BK, LDW, 2> sb;
    sa.init(oa, mn0a, tk, stid);
    sb.init(ob, mn0b, tk, stid);
    typename RawT<AD>::type ra[EA];
    typename RawT<BD>::type rb[EB];
    auto issue = [&](int t) {
        sa.template issue<AD>(t, ra);
        sb.template issue<BD>(t, rb);
    };
    auto split = [](float v, __bf16 &h, __bf16 &l) {
        h = (__bf16)v;
        l = (__bf16)(v - (float)h);
    };
    auto store = [&](int stage) {
        pin_raw(ra);
        pin_raw(rb);
        char *ah = (char *)(buf + stage * STAGE), *al = ah + 2 * PLANE, *bh = al + 2 * PLANE, *bl = bh + 2 * PLANE;
#pragma unroll
        for (int e = 0; e < EA; ++e)
            split(sa.template value<float, AD>(e, ra[e]), *(__bf16 *)(ah + sa.lds_byte(e)),
                  *(__bf16 *)(al + sa.lds_byte(e)));
#pragma unroll
        for (int e = 0; e < EB; ++e)
            split(sb.template value<float, BD>(e, rb[e]), *(__bf16 *)(bh + sb.lds_byte(e)),
                  *(__bf16 *)(bl + sb.lds_byte(e)));
    };
    static_assert(LDW % 4 == 0, "transposing reads need 8-byte aligned rows");
    // k = k0 + 8g .. k0 + 8g+7 of column w0 + 16 i + (lane & 15) in two
    // transposing reads (see read_bf16_frag); k0 = 32 x this k-group
    auto frag = [&](const __bf16 *plane, int w0, int i) {
        const int gq = lane >> 4, a4 = lane & 3, j4 = (lane >> 2) & 3;
        const __bf16 *p = plane + (32 * kg + 8 * gq + j4) * LDW + w0 + 16 * i + 4 * a4;
        const bf16x4 x0 = lds_read_tr16(p), x1 = lds_read_tr16(p + 4 * LDW);
        return bf16x8{x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3]};
    };

    // the k loop of grouped_tile: raw words of tile t+1 stored first, loads
    // of tile t+2 issued, then this k-group's step of tile t
    issue(0);
    store(0);
    if (nk > 1) issue(1);
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        const __bf16 *ah = buf + (t & 1) * STAGE, *al = ah + PLANE, *bh = al + PLANE, *bl = bh + PLANE;
        if (t + 1 < nk) store((t + 1) & 1);
        if (t + 2 < nk) issue(t + 2);
        bf16x8 fah[WMB], fal[WMB], fbh[WNB], fbl[WNB];
#pragma unroll
        for (int i = 0; i < WMB; ++i) {
            fah[i] = frag(ah, wm0, i);
            fal[i] = frag(al, wm0, i);
        }
#pragma unroll
        for (int i = 0; i < WNB; ++i) {
            fbh[i] = frag(bh, wn0, i);
            fbl[i] = frag(bl, wn0, i);
        }
#pragma unroll
        for (int a = 0; a < WMB; ++a)
#pragma unroll
            for (int b = 0; b < WNB; ++b) {
                acc[a][b] = mfma_bf16(fbl[b], fah[a], acc[a][b]);
                acc[a][b] = mfma_bf16(fbh[b], fal[a], acc[a][b]);
                acc[a][b] = mfma_bf16(fbh[b], fah[a], acc[a][b]);
            }
        __syncthreads();
    }
    if (grouped_reduce<float, v4f, KG, WMB, WNB>(acc, (float *)smem, wave, lane))
        grouped_epilogue<float, v4f, WMB, WNB>(g, mdbl, ndbl, ccplx, (int64_t)tm * tmn_a, (int64_t)tn * tmn_b, wm0,
                                               wn0, lane, acc);
}

// C := beta*C on a 64x64 region (products with alpha == 0 or k == 0).
__device__ __forceinline__ void grouped_scale_tile(const GemmArgs &g, int tm, int tn) {
    for (int e = threadIdx.x; e < 64 * 64; e += GNT) {
        const int64_t i = (int64_t)tm * 64 + (e & 63), j = (int64_t)tn * 64 + (e >> 6);
        if (i >= g.m || j >= g.n) continue;
        const int64_t off = i + j * g.ldc;
        if (g.c_cplx) {
            if (g.c_dbl) {
                double *c = (double *)g.C + 2 * off;
                const double *cin = (const double *)g.Cin + 2 * off;
                if (g.beta_zero) { c[0] = 0.0; c[1] = 0.0; }
                else {
                    const double cr = cin[0], ci = cin[1];
                    c[0] = fma(g.beta_re, cr, -(g.beta_im * ci));
                    c[1] = fma(g.beta_re, ci, g.beta_im * cr);
                }
            } else {
                float *c = (float *)g.C + 2 * off;
                const float *cin = (const float *)g.Cin + 2 * off;
                if (g.beta_zero) { c[0] = 0.0f; c[1] = 0.0f; }
                else {
                    const float br = (float)g.beta_re, bi = (float)g.beta_im, cr = cin[0], ci = cin[1];
                    c[0] = fmaf(br, cr, -(bi * ci));
                    c[1] = fmaf(br, ci, bi * cr);
                }
            }
        } else if (g.c_dbl) {
            double *c = (double *)g.C;
            c[off] = g.beta_zero ? 0.0 : g.beta_re * ((const double *)g.Cin)[off];
        } else {
            float *c = (float *)g.C;
            c[off] = g.beta_zero ? 0.0f : (float)g.beta_re * ((const float *)g.Cin)[off];
        }
    }
}

// Workgroups of the persistent kernel per CU (the grid is GROUPED_OCC x the
// CU count) and the waves per SIMD that makes (its register budget is 512 /
// GROUPED_WAVES per lane).
constexpr int GROUPED_OCC = 2;
constexpr int GROUPED_WAVES = GROUPED_OCC * (GNT / 64) / 4;

// The persistent kernel (defined in mdgemm_grouped_kernel.hip) and its
// launcher: `grid` workgroups of GNT threads on `s`.
void launch_grouped_kernel(int grid, hipStream_t s, const GDesc *descs, const GTile *tiles, int ntiles,
                           int *hdr);

}  // namespace md
