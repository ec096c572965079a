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

// Tile shapes of the grouped kernel (real-product workgroup tile).
enum { GCFG_64 = 0, GCFG_128 = 1, GCFG_COUNT = 2 };

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

// LDS bytes of each tile routine: two stages of the A' and B' k-tiles
// ([k][mn], padded) of T, or two stages of four bf16 planes for BF16x3; the
// kernel reserves the largest.
template <class T, int WB>
struct GShape {
    static constexpr int BM = 32 * WB;
    static constexpr int BK = (sizeof(T) == 8 ? 16 : 32) * 2 / WB;
    static constexpr int LDW = BM + (sizeof(T) == 8 ? 8 : 4);
    static constexpr int STAGE = 2 * BK * LDW;  // elements of T per stage (A' then B')
    static constexpr int SMEM = 2 * STAGE * (int)sizeof(T);
};
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int BF16X3_GROUPED_SMEM = 2 * 4 * 32 * (64 + 4) * 2;
constexpr int GROUPED_SMEM = cmax(cmax(cmax(GShape<float, 2>::SMEM, GShape<float, 4>::SMEM),
                                       cmax(GShape<double, 2>::SMEM, GShape<double, 4>::SMEM)),
                                  BF16X3_GROUPED_SMEM);

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

// Per-thread staging plan for the E elements a thread moves per k-tile of a
// BMN x BK tile.  For each element: the byte offset of its stored component
// from the tile's origin at k-tile 0 (32-bit: the host keeps products whose
// leading dimensions could overflow it out of the grouped launch) and its
// sign; its k index inside the tile and its LDS slot ([k][mn], row stride
// LDW) follow from the thread index and are recomputed where needed.
// Consecutive lanes take consecutive elements along the operand's contiguous
// dimension in HBM (m/n for an m/n-contiguous operand, k otherwise), so every
// load instruction reads whole cache lines.  Loads go through a buffer
// resource that starts at the k-tile's origin and ends at the matrix's last
// byte: an element outside the matrix gets an offset beyond the resource and
// reads zero, with no branch and no 64-bit arithmetic in the loop.
template <int E, int BMN, int BK, int LDW>
struct GStager {
    const char *base;
    int off[E];
    uint32_t negm;   // bit e: element e enters negated
    int64_t tile0;   // bytes from the matrix origin to the tile's origin at k-tile 0
    int64_t kbytes;  // bytes between consecutive k-tiles
    int64_t total;   // bytes from the matrix origin to its end
    int64_t K;
    int tk;
    bool mnc, k2;
    // tile coordinates (k row, m/n column) of element e of this thread
    __device__ __forceinline__ int kr_of(int e) const {
        const int idx = (int)threadIdx.x + e * NT;
        return mnc ? idx / BMN : idx % BK;
    }
    __device__ __forceinline__ int mr_of(int e) const {
        const int idx = (int)threadIdx.x + e * NT;
        return mnc ? idx % BMN : idx / BK;
    }
    __device__ __forceinline__ int slot(int e) const { return kr_of(e) * LDW + mr_of(e); }
    __device__ __forceinline__ int kp(int e) const { return k2 ? kr_of(e) >> 1 : kr_of(e); }
    __device__ __forceinline__ void init(const GOp &o, int64_t mn0, int tk_, int tid) {
        base = o.base;
        K = o.K;
        tk = tk_;
        mnc = o.mnc;
        k2 = gop_k2(o);
        const int W = o.cplx ? 2 : 1, esz = o.dbl ? 8 : 4;
        const int64_t rows_st = o.mnc ? o.MN : o.K, cols_st = o.mnc ? o.K : o.MN;
        total = ((cols_st - 1) * o.ld + rows_st) * W * esz;
        tile0 = (o.mnc ? mn0 : mn0 * o.ld) * W * esz;
        kbytes = (int64_t)tk * (o.mnc ? o.ld : 1) * W * esz;
        negm = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = tid + e * NT;
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
        }
    }
    // Issue the loads of the E elements of k-tile t: the raw words (the low
    // word, and for double storage the high word, of each element).  They
    // are converted only where they are stored (value), a k-tile later.
    template <bool DBL>
    __device__ __forceinline__ void issue(int t, uint32_t (&lo)[E], uint32_t (&hi)[E]) const {
        const int64_t b = tile0 + (int64_t)t * kbytes;
        const int64_t rem = total - b;
        const int nrec = rem > 0x7fffffffLL ? 0x7fffffff : (rem < 0 ? 0 : (int)rem);
        __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)(base + b), (short)0, nrec, 0x00020000);
        const int64_t kl = K - (int64_t)t * tk;
        const int klim = kl > (1 << 30) ? (1 << 30) : (int)kl;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            // along k the resource's end only bounds an m/n-contiguous operand
            const int o = (mnc || kp(e) < klim) ? off[e] : (int)0x80000000;
            if constexpr (DBL) {
                // two word loads rather than one pair, so that no register
                // pair has to survive the k loop's back edge
                lo[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, o, 0, 0);
                hi[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, o + 4, 0, 0);
            } else {
                lo[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, o, 0, 0);
            }
        }
    }
    // Element e of an issued k-tile, converted to T (float -> double is exact,
    // double -> float rounds to nearest even) and signed.
    template <class T, bool DBL>
    __device__ __forceinline__ T value(int e, uint32_t lo, uint32_t hi) const {
        T v;
        if constexpr (DBL) v = (T)__builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
        else v = (T)__builtin_bit_cast(float, lo);
        return ((negm >> e) & 1) ? -v : v;
    }
};

// Raw words of a staged k-tile, pinned where they are converted: the loads
// were issued a k-tile earlier, and this keeps the compiler from converting
// (and so waiting for) them right after issuing them.
template <int E, bool DBL>
__device__ __forceinline__ void pin_raw(uint32_t (&lo)[E], uint32_t (&hi)[E]) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if constexpr (DBL) asm("" : "+v"(lo[e]), "+v"(hi[e]));
        else asm("" : "+v"(lo[e]));
    }
}

// Epilogue shared by the grouped tile routines: acc[a][b] item v is
// C'(m = wm0 + 16a + (lane & 15), n = wn0 + 16b + acc_row(lane, v)).
template <class T, class ACC, int WB>
__device__ __forceinline__ void grouped_epilogue(const GemmArgs &g, bool mdbl, bool ndbl, bool ccplx,
                                                 int64_t i0, int64_t j0, int wm0, int wn0, int lane,
                                                 ACC (&acc)[WB][WB]) {
    const int ml = lane & 15;
#pragma unroll
    for (int b = 0; b < WB; ++b) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int nl = acc_row<T>(lane, v);
            if (mdbl) {
#pragma unroll
                for (int q = 0; q < WB / 2; ++q) {
                    const int64_t i = i0 + wm0 / 2 + q * 16 + ml;
                    const int64_t j = j0 + wn0 + b * 16 + nl;
                    update_cplx<T>(g, i, j, acc[2 * q][b][v], acc[2 * q + 1][b][v]);
                }
            } else if (ndbl) {
                if ((b & 1) == 0) {
#pragma unroll
                    for (int a = 0; a < WB; ++a) {
                        const int64_t i = i0 + wm0 + a * 16 + ml;
                        const int64_t j = j0 + wn0 / 2 + (b / 2) * 16 + nl;
                        update_cplx<T>(g, i, j, acc[a][b][v], acc[a][b + 1][v]);
                    }
                }
            } else {
#pragma unroll
                for (int a = 0; a < WB; ++a) {
                    const int64_t i = i0 + wm0 + a * 16 + ml;
                    const int64_t j = j0 + wn0 + b * 16 + nl;
                    if (ccplx) update_cplx<T>(g, i, j, acc[a][b][v], (T)0);
                    else update_real<T>(g, i, j, acc[a][b][v]);
                }
            }
        }
    }
}

// One output tile of a product computed in T (float or double) with FP32 /
// FP64 MFMA.  WB: 16x16 blocks per wave and dimension (2: 64x64 workgroup
// tile; 4: 128x128).  LDS holds one k-tile of A' and B' as [k][mn]; the next
// k-tile's elements are prefetched into registers during the MFMAs.
template <class T, int WB, bool AD, bool BD>
__device__ __forceinline__ void grouped_tile(const GDesc &d, int tm, int tn, char *smem) {
    typedef typename AccT<T>::type acc_t;
    // k depth per LDS tile: the 128x128 shape halves it so that every shape
    // stages the same number of elements per thread (8 per operand for f32,
    // 4 for f64)
    typedef GShape<T, WB> SH;
    constexpr int BM = SH::BM, BN = SH::BM, BK = SH::BK, LDW = SH::LDW;
    static_assert(SH::SMEM <= GROUPED_SMEM, "grouped LDS too small");
    constexpr int EA = BM * BK / NT, EB = BN * BK / NT;
    T *const buf = (T *)smem;  // stage s: A' at buf + s*STAGE, B' BK*LDW further
    const GemmArgs &g = d.g;
    const GOp oa = make_gop(g, d.cs, true), ob = make_gop(g, d.cs, false);
    const bool mdbl = gop_mn2(oa), ndbl = gop_mn2(ob), kdbl = gop_k2(oa);
    const bool ccplx = g.c_cplx;
    const int tmn_a = mdbl ? BM / 2 : BM, tmn_b = ndbl ? BN / 2 : BN, tk = kdbl ? BK / 2 : BK;
    const int64_t mn0a = (int64_t)tm * tmn_a, mn0b = (int64_t)tn * tmn_b;
    const int nk = (int)((g.k + tk - 1) / tk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave & 1) * 16 * WB, wn0 = (wave >> 1) * 16 * WB;

    acc_t acc[WB][WB];
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    GStager<EA, BM, BK, LDW> sa;
    GStager<EB, BN, BK, LDW> sb;
    sa.init(oa, mn0a, tk, tid);
    sb.init(ob, mn0b, tk, tid);
    uint32_t alo[EA], ahi[EA], blo[EB], bhi[EB];
    auto issue = [&](int t) {
        sa.template issue<AD>(t, alo, ahi);
        sb.template issue<BD>(t, blo, bhi);
    };
    auto store = [&](int stage) {
        pin_raw<EA, AD>(alo, ahi);
        pin_raw<EB, BD>(blo, bhi);
        T *la = buf + stage * SH::STAGE, *lb = la + BK * LDW;
#pragma unroll
        for (int e = 0; e < EA; ++e) la[sa.slot(e)] = sa.template value<T, AD>(e, alo[e], ahi[e]);
#pragma unroll
        for (int e = 0; e < EB; ++e) lb[sb.slot(e)] = sb.template value<T, BD>(e, blo[e], bhi[e]);
    };

    // Two LDS stages and one k-tile of loads in flight: iteration t first
    // writes the raw words of tile t+1 (issued during iteration t-1) to the
    // free stage (last read before the previous barrier), then issues the
    // loads of tile t+2, then multiplies tile t, so every load has a whole
    // k-tile of MFMAs to arrive; one barrier per k-tile.
    issue(0);
    store(0);
    if (nk > 1) issue(1);
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        const T *la = buf + (t & 1) * SH::STAGE, *lb = la + BK * LDW;
        if (t + 1 < nk) store((t + 1) & 1);
        if (t + 2 < nk) issue(t + 2);
#pragma unroll
        for (int s = 0; s < BK / 4; ++s) {
            const int kr = s * 4 + (lane >> 4);
            T fa[WB], fb[WB];
#pragma unroll
            for (int i = 0; i < WB; ++i) fa[i] = la[kr * LDW + wm0 + 16 * i + (lane & 15)];
#pragma unroll
            for (int i = 0; i < WB; ++i) fb[i] = lb[kr * LDW + wn0 + 16 * i + (lane & 15)];
#pragma unroll
            for (int a = 0; a < WB; ++a)
#pragma unroll
                for (int b = 0; b < WB; ++b) acc[a][b] = mfma16(fb[b], fa[a], acc[a][b]);
        }
        __syncthreads();
    }
    grouped_epilogue<T, acc_t, WB>(g, mdbl, ndbl, ccplx, (int64_t)tm * tmn_a, (int64_t)tn * tmn_b, wm0, wn0,
                                   lane, acc);
}

// BF16x3 form of grouped_tile: single-precision semantics from three bf16
// products per 16x16x32 block (see md_tile_bf16.h).
template <int WB, bool AD, bool BD>
__device__ __forceinline__ void grouped_tile_bf16x3(const GDesc &d, int tm, int tn, char *smem) {
    constexpr int BM = 32 * WB, BN = 32 * WB, BK = 32;
    constexpr int LDW = BM + 4, PLANE = BK * LDW, STAGE = 4 * PLANE;
    static_assert(2 * STAGE * 2 <= GROUPED_SMEM, "grouped LDS too small");
    constexpr int EA = BM * BK / NT, EB = BN * BK / NT;
    __bf16 *const buf = (__bf16 *)smem;  // stage s: planes Ah, Al, Bh, Bl
    const GemmArgs &g = d.g;
    const GOp oa = make_gop(g, d.cs, true), ob = make_gop(g, d.cs, false);
    const bool mdbl = gop_mn2(oa), ndbl = gop_mn2(ob), kdbl = gop_k2(oa);
    const bool ccplx = g.c_cplx;
    const int tmn_a = mdbl ? BM / 2 : BM, tmn_b = ndbl ? BN / 2 : BN, tk = kdbl ? BK / 2 : BK;
    const int64_t mn0a = (int64_t)tm * tmn_a, mn0b = (int64_t)tn * tmn_b;
    const int nk = (int)((g.k + tk - 1) / tk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave & 1) * 16 * WB, wn0 = (wave >> 1) * 16 * WB;

    v4f acc[WB][WB];
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b) acc[a][b] = v4f{0, 0, 0, 0};

    GStager<EA, BM, BK, LDW> sa;
    GStager<EB, BN, BK, LDW> sb;
    sa.init(oa, mn0a, tk, tid);
    sb.init(ob, mn0b, tk, tid);
    uint32_t alo[EA], ahi[EA], blo[EB], bhi[EB];
    auto issue = [&](int t) {
        sa.template issue<AD>(t, alo, ahi);
        sb.template issue<BD>(t, blo, bhi);
    };
    auto split = [](float v, __bf16 &h, __bf16 &l) {
        h = (__bf16)v;
        l = (__bf16)(v - (float)h);
    };
    auto store = [&](int stage) {
        pin_raw<EA, AD>(alo, ahi);
        pin_raw<EB, BD>(blo, bhi);
        __bf16 *ah = buf + stage * STAGE, *al = ah + PLANE, *bh = al + PLANE, *bl = bh + PLANE;
#pragma unroll
        for (int e = 0; e < EA; ++e)
            split(sa.template value<float, AD>(e, alo[e], ahi[e]), ah[sa.slot(e)], al[sa.slot(e)]);
#pragma unroll
        for (int e = 0; e < EB; ++e)
            split(sb.template value<float, BD>(e, blo[e], bhi[e]), bh[sb.slot(e)], bl[sb.slot(e)]);
    };
    static_assert(LDW % 4 == 0, "transposing reads need 8-byte aligned rows");
    // k = 8g .. 8g+7 of column w0 + 16 i + (lane & 15) in two transposing
    // reads (see read_bf16_frag)
    auto frag = [&](const __bf16 *plane, int w0, int i) {
        const int gq = lane >> 4, a4 = lane & 3, j4 = (lane >> 2) & 3;
        const __bf16 *p = plane + (8 * gq + j4) * LDW + w0 + 16 * i + 4 * a4;
        const bf16x4 x0 = lds_read_tr16(p), x1 = lds_read_tr16(p + 4 * LDW);
        return bf16x8{x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3]};
    };

    // the k loop of grouped_tile: raw words of tile t+1 stored first, loads
    // of tile t+2 issued, then the MFMAs of tile t
    issue(0);
    store(0);
    if (nk > 1) issue(1);
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        const __bf16 *ah = buf + (t & 1) * STAGE, *al = ah + PLANE, *bh = al + PLANE, *bl = bh + PLANE;
        if (t + 1 < nk) store((t + 1) & 1);
        if (t + 2 < nk) issue(t + 2);
        bf16x8 fah[WB], fal[WB], fbh[WB], fbl[WB];
#pragma unroll
        for (int i = 0; i < WB; ++i) {
            fah[i] = frag(ah, wm0, i);
            fal[i] = frag(al, wm0, i);
            fbh[i] = frag(bh, wn0, i);
            fbl[i] = frag(bl, wn0, i);
        }
#pragma unroll
        for (int a = 0; a < WB; ++a)
#pragma unroll
            for (int b = 0; b < WB; ++b) {
                acc[a][b] = mfma_bf16(fbl[b], fah[a], acc[a][b]);
                acc[a][b] = mfma_bf16(fbh[b], fal[a], acc[a][b]);
                acc[a][b] = mfma_bf16(fbh[b], fah[a], acc[a][b]);
            }
        __syncthreads();
    }
    grouped_epilogue<float, v4f, WB>(g, mdbl, ndbl, ccplx, (int64_t)tm * tmn_a, (int64_t)tn * tmn_b, wm0, wn0,
                                     lane, acc);
}

// C := beta*C on a 64x64 region (products with alpha == 0 or k == 0).
__device__ __forceinline__ void grouped_scale_tile(const GemmArgs &g, int tm, int tn) {
    for (int e = threadIdx.x; e < 64 * 64; e += NT) {
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



// Workgroups of the persistent kernel per CU (its register budget is
// 512 / GROUPED_OCC per lane; the grid is GROUPED_OCC x the CU count).
#ifndef MD_GOCC
#define MD_GOCC 2
#endif
constexpr int GROUPED_OCC = MD_GOCC;

// The persistent kernel (defined in mdgemm_grouped_kernel.hip) and its
// launcher: `grid` workgroups of NT threads on `s`.
void launch_grouped_kernel(int grid, hipStream_t s, const GDesc *descs, const GTile *tiles, int ntiles,
                           int *hdr);

}  // namespace md
