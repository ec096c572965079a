// md_small.h -- the product kernel for products with few output tiles.
//
// A product whose real product (md_internal.h, Figure "mixeddom") has few
// 128 x 128 tiles cannot fill the GPU with the tiled kernel of md_tile.h; this
// kernel cuts the real product into 32 x 32 tiles instead and gives each tile
// one workgroup of SM_W waves that share its inner dimension: wave w
// multiplies a contiguous range of the MFMA k-steps.  Each wave reads its
// MFMA fragments straight from HBM (every fragment element through the case's
// lowering: which stored element, which part, which sign), converting as it
// reads (the typecasting pack of Section 5, element by element), so the k
// loop has no LDS and no barrier; the waves' partial 32 x 32 products are then
// summed through LDS and one pass applies the epilogue of md_tile.h.  One
// launch, no workspace.
#pragma once
#include "md_tile.h"

namespace md {

constexpr int SM_TILE = 32;        // real-product tile edge
constexpr int SM_W = 8;            // waves per workgroup, sharing the inner dimension
constexpr int SM_NT = 64 * SM_W;   // threads per workgroup
constexpr int SM_U = 4;            // MFMA k-steps whose fragments a wave loads together

// One operand of the real product as the small kernel reads it: element
// (r, kk) of A' (r along m') or B' (r along n'), kk along k'.
template <class T, int CS, bool IS_A, bool SDBL>
struct SmallOp {
    static constexpr int MODE = mode_of<CS, IS_A>();
    static constexpr int W = (MODE == M_PLAIN) ? 1 : 2;
    static constexpr bool MN2 = (MODE == M_MNINT || MODE == M_ONEE);
    static constexpr bool K2 = (MODE == M_KINT || MODE == M_ONEE);
    const char *base;
    int64_t ld, MN, K;
    bool mnc, conj;

    __device__ __forceinline__ SmallOp(const GemmArgs &g) {
        const int tr = IS_A ? g.ta : g.tb;
        base = (const char *)(IS_A ? g.A : g.B);
        ld = IS_A ? g.lda : g.ldb;
        MN = IS_A ? g.m : g.n;
        K = g.k;
        mnc = IS_A ? (tr == 0 || tr == 3) : (tr == 1 || tr == 2);
        conj = tr >= 2;
    }

    // Where element (r, kk) of the real product's operand lives: the byte
    // offset of its stored component (0, the first element, when it lies
    // outside the matrix or `use` is false: such an element reads as zero),
    // whether it counts, and whether it enters negated.
    __device__ __forceinline__ int64_t where(int64_t r, int64_t kk, bool use, bool *valid, bool *neg) const {
        int64_t i = r, p = kk;
        int qm = 0, qk = 0;
        if constexpr (MN2) {  // Re/Im in alternating blocks of 16 rows (or columns)
            qm = (int)((r >> 4) & 1);
            i = ((r >> 5) << 4) | (r & 15);
        }
        if constexpr (K2) {  // Re/Im interleaved along k
            qk = (int)(kk & 1);
            p = kk >> 1;
        }
        int comp = 0;
        bool ng = false;
        if constexpr (MODE == M_KINT) {
            comp = qk;
            ng = qk && IS_A;  // -Im(A) at odd k' (Re(AB) = ArBr - AiBi)
        } else if constexpr (MODE == M_MNINT) {
            comp = qm;
        } else if constexpr (MODE == M_ONEE) {  // [re -im; im re] per complex element (Eq. 1mc)
            comp = qm ^ qk;
            ng = (qm == 0 && qk == 1);
        }
        if (comp == 1 && conj) ng = !ng;
        *neg = ng;
        // no branch: the offset is always formed and then selected
        const bool ok = use & (i < MN) & (p < K);
        *valid = ok;
        const int64_t off = ((mnc ? (i + p * ld) : (p + i * ld)) * W + comp) * (SDBL ? 8 : 4);
        return ok ? off : (int64_t)0;
    }
    // Issue the load of the raw words at byte offset off.
    __device__ __forceinline__ void issue(int64_t off, uint32_t *lo, uint32_t *hi) const {
        const uint32_t *q = (const uint32_t *)(base + off);
        *lo = q[0];
        if constexpr (SDBL) *hi = q[1];
    }
    // The loaded words as a value of T: zero when not valid, signed.
    __device__ __forceinline__ static T value(uint32_t lo, uint32_t hi, bool valid, bool neg) {
        T v;
        if constexpr (SDBL) v = (T)__builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
        else v = (T)__builtin_bit_cast(float, lo);
        v = valid ? v : (T)0;
        return neg ? -v : v;
    }
};

template <class T, int CS, bool AD, bool BD>
__global__ __launch_bounds__(SM_NT, 1) void md_small_kernel(GemmArgs g) {
    typedef SmallOp<T, CS, true, AD> OA;
    typedef SmallOp<T, CS, false, BD> OB;
    typedef typename AccT<T>::type acc_t;
    constexpr bool MDBL = OA::MN2, NDBL = OB::MN2;
    constexpr bool CCPLX = (CS == MD_CASE_1C || CS == MD_CASE_2AC || CS == MD_CASE_2BC || CS == MD_CASE_3);
    constexpr int TMN_A = SM_TILE / (MDBL ? 2 : 1), TMN_B = SM_TILE / (NDBL ? 2 : 1);
    constexpr int LDR = SM_TILE + 1;  // row stride of the reduction buffer
    __shared__ T red[SM_W][SM_TILE * LDR];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tm = (int)(blockIdx.x % (unsigned)g.tiles_m), tn = (int)(blockIdx.x / (unsigned)g.tiles_m);
    const OA oa(g);
    const OB ob(g);
    // real-product rows and columns of this tile
    const int64_t r0a = (int64_t)tm * SM_TILE, r0b = (int64_t)tn * SM_TILE;
    const int64_t kr = g.k * (OA::K2 ? 2 : 1);
    const int64_t nsteps = (kr + 3) / 4;
    const int64_t s0 = nsteps * wave / SM_W, s1 = nsteps * (wave + 1) / SM_W;
    const int r = lane & 15, gq = lane >> 4;

    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    // fragments of SM_U consecutive k-steps, two register sets: the raw words
    // of the next group are loaded while the current group is converted and
    // multiplied (converting is where a load is waited for)
    uint32_t alo[2][SM_U][2], ahi[2][SM_U][2], blo[2][SM_U][2], bhi[2][SM_U][2];
    uint32_t amask[2], bmask[2];  // per element: bit 2e valid, bit 2e+1 negated
    auto load_group = [&](auto bufc, int64_t sg) {
        constexpr int buf = decltype(bufc)::value;
        amask[buf] = 0;
        bmask[buf] = 0;
#pragma unroll
        for (int u = 0; u < SM_U; ++u) {
            const int64_t s = sg + u;
            const bool use = s < s1;
            const int64_t kk = 4 * s + gq;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                bool v, n;
                const int64_t off = oa.where(r0a + 16 * i + r, kk, use, &v, &n);
                oa.issue(off, &alo[buf][u][i], &ahi[buf][u][i]);
                amask[buf] |= ((uint32_t)v | ((uint32_t)n << 1)) << (2 * (2 * u + i));
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                bool v, n;
                const int64_t off = ob.where(r0b + 16 * j + r, kk, use, &v, &n);
                ob.issue(off, &blo[buf][u][j], &bhi[buf][u][j]);
                bmask[buf] |= ((uint32_t)v | ((uint32_t)n << 1)) << (2 * (2 * u + j));
            }
        }
    };
    auto multiply = [&](auto bufc) {
        constexpr int buf = decltype(bufc)::value;
        // nothing moves across: the conversions below stay after the MFMAs
        // of the previous group, which cover the loads of this one
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < SM_U; ++u) {
            T fa[2], fb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                if constexpr (AD) asm("" : "+v"(alo[buf][u][i]), "+v"(ahi[buf][u][i]));
                else asm("" : "+v"(alo[buf][u][i]));
                const uint32_t mk = amask[buf] >> (2 * (2 * u + i));
                fa[i] = OA::value(alo[buf][u][i], ahi[buf][u][i], mk & 1, (mk >> 1) & 1);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if constexpr (BD) asm("" : "+v"(blo[buf][u][j]), "+v"(bhi[buf][u][j]));
                else asm("" : "+v"(blo[buf][u][j]));
                const uint32_t mk = bmask[buf] >> (2 * (2 * u + j));
                fb[j] = OB::value(blo[buf][u][j], bhi[buf][u][j], mk & 1, (mk >> 1) & 1);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(fb[b], fa[a], acc[a][b]);
        }
    };
    std::integral_constant<int, 0> b0;
    std::integral_constant<int, 1> b1;
    load_group(b0, s0);
    for (int64_t sg = s0; sg < s1; sg += 2 * SM_U) {
        load_group(b1, sg + SM_U);
        multiply(b0);
        if (sg + 2 * SM_U < s1) load_group(b0, sg + 2 * SM_U);
        if (sg + SM_U < s1) multiply(b1);
    }

    // acc[a][b] item v is the wave's partial C'(16a + (lane & 15), 16b + acc_row(lane, v))
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                red[wave][(16 * a + r) * LDR + 16 * b + acc_row<T>(lane, v)] = acc[a][b][v];
    __syncthreads();

    auto sum = [&](int row, int col) {
        T s = 0;
#pragma unroll
        for (int w = 0; w < SM_W; ++w) s += red[w][row * LDR + col];
        return s;
    };
    // one thread per element of C in the tile
    constexpr int NC = TMN_A * TMN_B;
    for (int e = tid; e < NC; e += SM_NT) {
        const int ci = e % TMN_A, cj = e / TMN_A;
        const int64_t i = (int64_t)tm * TMN_A + ci, j = (int64_t)tn * TMN_B + cj;
        if constexpr (MDBL) {
            // complex row ci: Re in real row split_pos(ci, 0), Im in split_pos(ci, 1)
            update_cplx<T, false, true>(g, i, j, sum(split_pos(ci, 0), cj), sum(split_pos(ci, 1), cj));
        } else if constexpr (NDBL) {
            update_cplx<T, false, true>(g, i, j, sum(ci, split_pos(cj, 0)), sum(ci, split_pos(cj, 1)));
        } else if constexpr (CCPLX) {
            update_cplx<T, false, true>(g, i, j, sum(ci, cj), (T)0);
        } else {
            update_real<T, false, true>(g, i, j, sum(ci, cj));
        }
    }
}

}  // namespace md
