// md_tile_bf16.h -- the BF16x3 form of the product kernel (computation
// precision MD_COMP_S_BF16X3).
//
// Single-precision semantics on the bfloat16 matrix cores: staging converts
// each element to FP32 exactly as the single-precision path does, then splits
// it into hi = bf16(a) and lo = bf16(a - hi) (both round-to-nearest-even;
// a - hi is exact in FP32) and writes hi and lo to two LDS planes.  Each
// product of the real product is formed from three bf16 products,
//     a*b ~ hi_a*hi_b + hi_a*lo_b + lo_a*hi_b,
// accumulated in FP32 by v_mfma_f32_16x16x32_bf16.  bf16 keeps 8 significant
// bits, so |lo| <= 2^-8 |a| and a - hi - lo <= 2^-16 |a|: the dropped
// lo_a*lo_b and the two residuals leave up to about 3 * 2^-16 |a||b| per
// product, inside the single-precision bound 4 k u_s |a||b| from k ~ 192 on
// (below that the split's term is the larger one).  The lowering of the
// domain cases, the staging loads and the epilogue are those of md_tile.h with
// T = float.  This precision form is an addition of this library, not of the
// paper.
//
// With H16 the same kernel is the half computation precision (MD_COMP_H):
// staging rounds each FP32 value to binary16 into one LDS plane and every
// 16x16x32 step is one v_mfma_f32_16x16x32_f16 with FP32 accumulation.
#pragma once
#include "md_tile.h"

namespace md {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// One LDS plane of bf16: [k][mn] (row stride BMN+4) for an operand contiguous
// along m/n, [mn][k] (row stride 40) for one contiguous along k.  The paddings
// put the 4 lane groups of a fragment read on distinct banks.
template <bool MNC, int BMN>
struct LayBF {
    static constexpr int BK = 32;
    static constexpr int LD = MNC ? BMN + 4 : BK + 8;
    static constexpr int SIZE = (MNC ? BK : BMN) * LD;
    __device__ __forceinline__ static int at(int kk, int mm) { return MNC ? kk * LD + mm : mm * LD + kk; }
};

// Staging output that writes the hi and lo halves of each FP32 value.
template <bool MNC, int BMN>
struct SplitOut {
    static constexpr bool NARROW = true;  // every value converted to bf16
    typedef LayBF<MNC, BMN> L;
    __bf16 *hi, *lo;
    __device__ __forceinline__ void put(int kk, int mm, float v) const {
        const __bf16 h = (__bf16)v;
        const __bf16 l = (__bf16)(v - (float)h);
        hi[L::at(kk, mm)] = h;
        lo[L::at(kk, mm)] = l;
    }
};

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;
typedef __attribute__((address_space(3))) __bf16 lds_bf16;

// Transposing LDS read (ds_read_b64_tr_b16): inside each group of 16 lanes,
// lane 4a+b receives element b of the 8-byte reads addressed by lanes a,
// a+4, a+8 and a+12 (measured on gfx950).
__device__ __forceinline__ bf16x4 lds_read_tr16(const __bf16 *p) {
    return __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4 *)(lds_bf16 *)p);
}

// Fragment of one 16x16x32 MFMA operand for block i: lane group g = lane >> 4
// holds k = 8g .. 8g+7 of row (or column) w0 + 16 i + (lane & 15).  From a
// [k][mn] plane it takes two transposing reads: lane 16g + a + 4j addresses
// k = 8g + j (then 8g + j + 4) at columns 4a .. 4a+3 of the block, so lane
// 16g + r receives the 4 consecutive k of column r; from a [mn][k] plane the
// 8 k are one 16-byte read.
// Staging output that rounds each FP32 value to binary16 (nearest even).
template <bool MNC, int BMN>
struct HalfOut {
    static constexpr bool NARROW = true;  // every value converted to binary16
    typedef LayBF<MNC, BMN> L;
    __bf16 *plane;  // 16-bit LDS storage, written as binary16
    __device__ __forceinline__ void put(int kk, int mm, float v) const {
        ((_Float16 *)plane)[L::at(kk, mm)] = (_Float16)v;
    }
};

template <bool MNC, int BMN>
__device__ __forceinline__ bf16x8 read_bf16_frag(const __bf16 *plane, int lane, int w0, int i) {
    typedef LayBF<MNC, BMN> L;
    static_assert(!MNC || L::LD % 4 == 0, "transposing reads need 8-byte aligned rows");
    const int g = lane >> 4;
    if constexpr (MNC) {
        const int a4 = lane & 3, j4 = (lane >> 2) & 3;
        const int row = 8 * g + j4, col = w0 + 16 * i + 4 * a4;
        const bf16x4 x0 = lds_read_tr16(&plane[L::at(row, col)]);
        const bf16x4 x1 = lds_read_tr16(&plane[L::at(row + 4, col)]);
        return bf16x8{x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3]};
    } else {
        const int mm = w0 + 16 * i + (lane & 15);
        return *(const bf16x8 *)&plane[L::at(8 * g, mm)];
    }
}

__device__ __forceinline__ v4f mfma_bf16(bf16x8 x, bf16x8 y, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
}

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// The same fragments (16-bit lanes) taken as binary16.
__device__ __forceinline__ v4f mfma_f16(bf16x8 x, bf16x8 y, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, x), __builtin_bit_cast(f16x8, y), c, 0,
                                                  0, 0);
}

// Epilogue of the 16-bit-product kernels: acc[a][b] item v is
// C'(row m = wm0 + 16a + (lane & 15), col n = wn0 + 16b + acc_row(lane, v)) of
// the workgroup tile whose first stored rows / columns are i0 / j0.  GS: C has
// general strides.  Binary16 C takes the general update (decided once per
// workgroup), so the common case keeps the plain update's code.  The general
// update is too large to inline at every accumulator of the wide tiles: there
// the loop over row blocks stays rolled and picks its accumulator with
// selects (an indexed access would put the accumulators in scratch).
template <int CS, bool GS, int WMB, int WNB>
__device__ __forceinline__ void x16_epilogue(const GemmArgs &g, v4f (&acc)[WMB][WNB], int64_t i0, int64_t j0,
                                             int wm0, int wn0, int lane) {
    constexpr int MODE_A = mode_of<CS, true>(), MODE_B = mode_of<CS, false>();
    constexpr bool MDBL = MODE_A == M_MNINT || MODE_A == M_ONEE;
    constexpr bool NDBL = MODE_B == M_MNINT || MODE_B == M_ONEE;
    constexpr bool CCPLX = (CS == MD_CASE_1C || CS == MD_CASE_2AC || CS == MD_CASE_2BC || CS == MD_CASE_3);
    auto epilogue = [&](auto general_tag) {
        constexpr bool GEN = decltype(general_tag)::value;
        auto pick = [&](int a, int b, int v) {
            float r = acc[0][b][v];
#pragma unroll
            for (int x = 1; x < WMB; ++x) r = (a == x) ? acc[x][b][v] : r;
            return r;
        };
        // updates per thread: the general one rolled from 64 on, the plain
        // one from 256 on
        constexpr int NCALL = WNB * 4 * (MDBL ? WMB / 2 : WMB) / (NDBL ? 2 : 1);
        constexpr bool ROLL = (GEN && NCALL >= 64) || NCALL >= 256;
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
                const int nl = acc_row<float>(lane, v);
                if constexpr (MDBL) {
                    rows(WMB / 2, [&](int q) {
                        const int64_t i = i0 + wm0 / 2 + q * 16 + ml;
                        const int64_t j = j0 + wn0 + b * 16 + nl;
                        update_cplx<float, GS, GEN>(g, i, j, pick(2 * q, b, v), pick(2 * q + 1, b, v));
                    });
                } else if constexpr (NDBL) {
                    if ((b & 1) == 0) {
                        rows(WMB, [&](int a) {
                            const int64_t i = i0 + wm0 + a * 16 + ml;
                            const int64_t j = j0 + wn0 / 2 + (b / 2) * 16 + nl;
                            update_cplx<float, GS, GEN>(g, i, j, pick(a, b, v), pick(a, b + 1, v));
                        });
                    }
                } else {
                    rows(WMB, [&](int a) {
                        const int64_t i = i0 + wm0 + a * 16 + ml;
                        const int64_t j = j0 + wn0 + b * 16 + nl;
                        if constexpr (CCPLX) update_cplx<float, GS, GEN>(g, i, j, pick(a, b, v), 0.0f);
                        else update_real<float, GS, GEN>(g, i, j, pick(a, b, v));
                    });
                }
            }
        }
    };
    if (g.c_half) epilogue(std::true_type{});
    else epilogue(std::false_type{});
}

template <int CS, bool FAST, bool AD, bool BD, bool AMNC, bool BMNC, class C = TileCfg<float>, bool RAG = false,
          bool SCL = false, bool H16 = false, bool SH = false>
__global__ __launch_bounds__(C::NT, C::OCC) void md_bf16x3_kernel(GemmArgs g) {
    static_assert(C::BK == 32, "one 16x16x32 step per LDS tile");
    typedef Stage<float, CS, true, FAST, AD, AMNC, C, RAG, SCL && CS != MD_CASE_1B, H16 && AD, SH> SA;
    typedef Stage<float, CS, false, FAST, BD, BMNC, C, RAG, SCL && CS == MD_CASE_1B, H16 && BD, SH> SB;
    constexpr int WMB = C::WMB, WNB = C::WNB;
    typedef LayBF<AMNC, C::BM> LA;
    typedef LayBF<BMNC, C::BN> LB;
    static_assert(SA::TK == SB::TK, "A and B disagree on the k lowering");
    static_assert(SA::MN2 == (mode_of<CS, true>() == M_MNINT || mode_of<CS, true>() == M_ONEE), "m' doubling");

    // [buffer][plane hi/lo (one binary16 plane with H16)][...]
    constexpr int NPL = H16 ? 1 : 2;
    __shared__ __attribute__((aligned(16))) __bf16 sA[2][NPL][LA::SIZE];
    __shared__ __attribute__((aligned(16))) __bf16 sB[2][NPL][LB::SIZE];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % C::WGM) * (C::BM / C::WGM), wn0 = (wave / C::WGM) * (C::BN / C::WGN);
    int tm, tn;
    map_tile(blockIdx.x, gridDim.x, g.tiles_m, g.tiles_n, &tm, &tn);
    const int64_t mn0a = (int64_t)tm * SA::TMN, mn0b = (int64_t)tn * SB::TMN;
    const int nk = (int)((g.k + SA::TK - 1) / SA::TK);

    v4f acc[WMB][WNB];
#pragma unroll
    for (int a = 0; a < WMB; ++a)
#pragma unroll
        for (int b = 0; b < WNB; ++b) acc[a][b] = v4f{0, 0, 0, 0};

    SA la(g, tid, mn0a);
    SB lb(g, tid, mn0b);
    auto stage_out = [&](int buf) {
        if constexpr (H16) {
            la.store_to(HalfOut<AMNC, C::BM>{sA[buf][0]});
            lb.store_to(HalfOut<BMNC, C::BN>{sB[buf][0]});
        } else {
            la.store_to(SplitOut<AMNC, C::BM>{sA[buf][0], sA[buf][NPL - 1]});
            lb.store_to(SplitOut<BMNC, C::BN>{sB[buf][0], sB[buf][NPL - 1]});
        }
    };
    // One LDS tile = one 32-deep step: 3 bf16 MFMAs per 16x16 block.  With
    // store_next the staged registers of tile t+1 go to the other buffer
    // (last read before the previous barrier) and the loads of tile
    // `next_load` are issued before the MFMAs, which they then overlap.
    auto tile = [&](int cur, bool store_next, int next_load) {
        bf16x8 ah[WMB], al[WMB], bh[WNB], bl[WNB];
#pragma unroll
        for (int i = 0; i < WMB; ++i) {
            ah[i] = read_bf16_frag<AMNC, C::BM>(sA[cur][0], lane, wm0, i);
            if constexpr (!H16) al[i] = read_bf16_frag<AMNC, C::BM>(sA[cur][NPL - 1], lane, wm0, i);
        }
#pragma unroll
        for (int i = 0; i < WNB; ++i) {
            bh[i] = read_bf16_frag<BMNC, C::BN>(sB[cur][0], lane, wn0, i);
            if constexpr (!H16) bl[i] = read_bf16_frag<BMNC, C::BN>(sB[cur][NPL - 1], lane, wn0, i);
        }
        if (store_next) stage_out(cur ^ 1);
        if (next_load < nk) {
            la.load(next_load);
            lb.load(next_load);
        }
#pragma unroll
        for (int a = 0; a < WMB; ++a)
#pragma unroll
            for (int b = 0; b < WNB; ++b) {
                if constexpr (H16) {
                    acc[a][b] = mfma_f16(bh[b], ah[a], acc[a][b]);
                } else {
                    acc[a][b] = mfma_bf16(bl[b], ah[a], acc[a][b]);
                    acc[a][b] = mfma_bf16(bh[b], al[a], acc[a][b]);
                    acc[a][b] = mfma_bf16(bh[b], ah[a], acc[a][b]);
                }
            }
    };

    la.load(0);
    lb.load(0);
    stage_out(0);
    __syncthreads();
    if (nk > 1) {
        la.load(1);
        lb.load(1);
    }
    int t = 0;
    for (; t + 1 < nk; ++t) {
        tile(t & 1, true, t + 2);
        __syncthreads();
    }
    tile(t & 1, false, nk);

    x16_epilogue<CS, !FAST, WMB, WNB>(g, acc, (int64_t)tm * SA::TMN, (int64_t)tn * SB::TMN, wm0, wn0, lane);
}

}  // namespace md
