// mdgemm_kernels.hip -- device side of libmdgemm for gfx950 (CDNA4).
//
// One templated kernel per (computation precision, domain case).  Each
// workgroup owns a tile of the real product C' += A' B' that its case lowers
// to (md_internal.h, Figure "mixeddom"):
//
//   1. cast-on-pack: A and B tiles are read from HBM in their storage type
//      with 16-byte vector loads, converted to the computation type in
//      registers (float -> double exact, double -> float round-to-nearest-even,
//      the typecasting pack of Section 4) and written to LDS already in the
//      layout of the real product: complex elements are split into their
//      parts, the parts that cannot reach C are dropped, conjugation flips a
//      sign, and case 3 writes A in the 1e arrangement of Eq. 1mc (each complex
//      element becomes the real 2x2 block [re -im; im re]) while B keeps the
//      1r arrangement (re, im interleaved along k);
//   2. a double-buffered k loop of real MFMA (v_mfma_f64_16x16x4f64 or
//      v_mfma_f32_16x16x4f32) over the LDS tiles: the global loads of tile t+1
//      are in flight while tile t is multiplied;
//   3. an epilogue that applies alpha (cast to the computation precision) and
//      beta (cast to C's storage precision), forms beta*C + alpha*AB in the
//      wider of the computation and C precisions, and rounds once to C's
//      storage type (Sections 4.1.3 and 6.1).
//
// The MFMA is issued with B' as its first operand so that the accumulator
// lanes run along m: stores to column-major C are then contiguous.
#include <hip/hip_runtime.h>

#include "md_internal.h"

namespace md {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int NT = 256;  // threads per workgroup: 4 waves of 64
constexpr int G = 16;    // MFMA block edge (16x16 output blocks)

template <class T> struct TileCfg;
template <> struct TileCfg<double> {
    static constexpr int BM = 128, BN = 128, BK = 16, PAD = 16;
};
template <> struct TileCfg<float> {
    static constexpr int BM = 128, BN = 128, BK = 32, PAD = 16;
};

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

// ---------------------------------------------------------------------------
// Operand staging (cast-on-pack)
// ---------------------------------------------------------------------------
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

template <class T, int CS, bool IS_A>
struct Stage {
    typedef TileCfg<T> C;
    static constexpr int MODE = mode_of<CS, IS_A>();
    static constexpr int W = (MODE == M_PLAIN) ? 1 : 2;  // stored components per element
    static constexpr bool MN2 = (MODE == M_MNINT || MODE == M_ONEE);
    static constexpr bool K2 = (MODE == M_KINT || MODE == M_ONEE);
    static constexpr int BMN = IS_A ? C::BM : C::BN;
    static constexpr int TMN = BMN / (MN2 ? 2 : 1);  // stored m (or n) extent of a tile
    static constexpr int TK = C::BK / (K2 ? 2 : 1);   // stored k extent of a tile
    static constexpr int CHUNKS = TMN * TK * W / 4;   // 4 components per chunk
    static constexpr int PER = CHUNKS / NT;
    static constexpr int LDW = BMN + C::PAD;          // LDS row stride (elements)
    // Sign applied to Im when it is placed at an odd k' row: -Im(A) in case 2ab
    // realises Re(AB) = ArBr - AiBi; B's Im enters positively.
    static constexpr bool KNEG = IS_A;
    static_assert(CHUNKS % NT == 0, "tile does not split evenly over the workgroup");
    static_assert((TMN * W) % 4 == 0 && (TK * W) % 4 == 0, "chunks straddle columns");

    // Registers holding one tile's loads until they are converted: 4 stored
    // components per chunk (lo only for single storage, lo+hi for double).
    struct Chunk { uint4 lo, hi; };
    Chunk raw[PER];

    // Issue the global loads of one tile: stored-index origin mn0 (m or n) and
    // k0.  With VEC (aligned operand whose columns hold a multiple of four
    // components) each chunk is one predicated 16-byte load (two for double);
    // otherwise components are loaded one by one.  Anything outside the
    // matrix reads as zero, which adds nothing to the product.
    template <bool VEC, bool DBL>
    __device__ __forceinline__ void load_impl(const GemmArgs &g, int64_t mn0, int64_t k0, int tid) {
        const int tr = IS_A ? g.ta : g.tb;
        const bool mn_contig = IS_A ? (tr == 0) : (tr != 0);
        const int64_t ld = IS_A ? g.lda : g.ldb;
        const int64_t MN = IS_A ? g.m : g.n;
        const char *base = (const char *)(IS_A ? g.A : g.B);
        const int64_t rows_st = mn_contig ? MN : g.k;
        const int64_t cols_st = mn_contig ? g.k : MN;
        const int64_t r0 = mn_contig ? mn0 : k0;
        const int64_t c0 = mn_contig ? k0 : mn0;
        const int cpc = (mn_contig ? TMN : TK) * W / 4;
        const int64_t contig_len = rows_st * W;
        const int64_t col_stride = ld * W;
        const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int c = 0; c < PER; ++c) {
            const int ch = tid + c * NT;
            const int col_in = ch / cpc, pos = ch - col_in * cpc;
            const int64_t col = c0 + col_in, comp0 = r0 * W + pos * 4;
            const bool colok = col < cols_st;
            const int64_t idx = col * col_stride + comp0;
            Chunk x;
            x.lo = zero;
            x.hi = zero;
            if constexpr (VEC) {
                if (colok && comp0 < contig_len) {
                    if constexpr (DBL) {
                        const uint4 *p = (const uint4 *)((const double *)base + idx);
                        x.lo = p[0];
                        x.hi = p[1];
                    } else {
                        x.lo = *(const uint4 *)((const float *)base + idx);
                    }
                }
            } else if constexpr (DBL) {
                const uint2 *p = (const uint2 *)base + idx;
                uint2 e0 = make_uint2(0u, 0u), e1 = e0, e2 = e0, e3 = e0;
                if (colok && comp0 + 0 < contig_len) e0 = p[0];
                if (colok && comp0 + 1 < contig_len) e1 = p[1];
                if (colok && comp0 + 2 < contig_len) e2 = p[2];
                if (colok && comp0 + 3 < contig_len) e3 = p[3];
                x.lo = make_uint4(e0.x, e0.y, e1.x, e1.y);
                x.hi = make_uint4(e2.x, e2.y, e3.x, e3.y);
            } else {
                const uint32_t *p = (const uint32_t *)base + idx;
                uint32_t e0 = 0u, e1 = 0u, e2 = 0u, e3 = 0u;
                if (colok && comp0 + 0 < contig_len) e0 = p[0];
                if (colok && comp0 + 1 < contig_len) e1 = p[1];
                if (colok && comp0 + 2 < contig_len) e2 = p[2];
                if (colok && comp0 + 3 < contig_len) e3 = p[3];
                x.lo = make_uint4(e0, e1, e2, e3);
            }
            raw[c] = x;
        }
    }

    __device__ __forceinline__ void load(const GemmArgs &g, int64_t mn0, int64_t k0, int tid) {
        const bool dbl = IS_A ? g.a_dbl : g.b_dbl;
        const bool vec = IS_A ? g.a_vec : g.b_vec;
        if (vec) {
            if (dbl) load_impl<true, true>(g, mn0, k0, tid);
            else load_impl<true, false>(g, mn0, k0, tid);
        } else {
            if (dbl) load_impl<false, true>(g, mn0, k0, tid);
            else load_impl<false, false>(g, mn0, k0, tid);
        }
    }

    __device__ __forceinline__ static T component(const Chunk &x, int q, bool dbl) {
        if (dbl) {
            const uint4 h = q < 2 ? x.lo : x.hi;
            const uint32_t w0 = (q & 1) ? h.z : h.x;
            const uint32_t w1 = (q & 1) ? h.w : h.y;
            return (T)__builtin_bit_cast(double, ((uint64_t)w1 << 32) | w0);
        }
        const uint32_t w = q == 0 ? x.lo.x : (q == 1 ? x.lo.y : (q == 2 ? x.lo.z : x.lo.w));
        return (T)__builtin_bit_cast(float, w);
    }

    __device__ __forceinline__ static void emit(T *lds, int mm, int kk, int part, T v, bool conj) {
        if constexpr (MODE == M_PLAIN) {
            lds[kk * LDW + mm] = v;
        } else if constexpr (MODE == M_REONLY) {
            if (part == 0) lds[kk * LDW + mm] = v;
        } else {
            const T vi = conj ? -v : v;
            if constexpr (MODE == M_KINT) {
                if (part == 0) lds[(2 * kk) * LDW + mm] = v;
                else lds[(2 * kk + 1) * LDW + mm] = KNEG ? -vi : vi;
            } else if constexpr (MODE == M_MNINT) {
                if (part == 0) lds[kk * LDW + split_pos(mm, 0)] = v;
                else lds[kk * LDW + split_pos(mm, 1)] = vi;
            } else {  // M_ONEE: [re -im; im re] per complex element (Eq. 1mc)
                if (part == 0) {
                    lds[(2 * kk) * LDW + split_pos(mm, 0)] = v;
                    lds[(2 * kk + 1) * LDW + split_pos(mm, 1)] = v;
                } else {
                    lds[(2 * kk) * LDW + split_pos(mm, 1)] = vi;
                    lds[(2 * kk + 1) * LDW + split_pos(mm, 0)] = -vi;
                }
            }
        }
    }

    // Convert the staged registers to T and write them to one LDS buffer.
    __device__ __forceinline__ void store(const GemmArgs &g, T *lds, int tid) const {
        const bool dbl = IS_A ? g.a_dbl : g.b_dbl;
        const int tr = IS_A ? g.ta : g.tb;
        const bool mn_contig = IS_A ? (tr == 0) : (tr != 0);
        const bool conj = (tr == 2);
        const int cpc = (mn_contig ? TMN : TK) * W / 4;
#pragma unroll
        for (int c = 0; c < PER; ++c) {
            const int ch = tid + c * NT;
            const int col_in = ch / cpc, pos = ch - (ch / cpc) * cpc;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const T v = component(raw[c], q, dbl);
                const int e = pos * (4 / W) + q / W;
                const int part = q % W;
                if (mn_contig) emit(lds, e, col_in, part, v, conj);
                else emit(lds, col_in, e, part, v, conj);
            }
        }
    }
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
template <class T>
__device__ __forceinline__ void update_real(const GemmArgs &g, int64_t i, int64_t j, T acc) {
    if (i >= g.m || j >= g.n) return;
    const int64_t off = i + j * g.ldc;
    const T ax = (T)g.alpha_re;
    if (g.c_dbl) {
        double *c = (double *)g.C;
        const double t = (double)ax * (double)acc;
        c[off] = g.beta_zero ? t : fma(g.beta_re, c[off], t);
    } else {
        float *c = (float *)g.C;
        const float bc = (float)g.beta_re;
        if constexpr (sizeof(T) == 8) {
            const double t = ax * acc;
            c[off] = (float)(g.beta_zero ? t : fma((double)bc, (double)c[off], t));
        } else {
            const float t = ax * acc;
            c[off] = g.beta_zero ? t : fmaf(bc, c[off], t);
        }
    }
}

// Complex C: (re, im) is alpha-free AB for this element (im == 0 in case 1c).
template <class T, class W>
__device__ __forceinline__ void cupdate(const GemmArgs &g, W *c2, W re, W im, W ar, W ai) {
    const W tr = fma(ar, re, -(ai * im));
    const W ti = fma(ar, im, ai * re);
    if (g.beta_zero) {
        c2[0] = tr;
        c2[1] = ti;
    } else {
        const W br = (W)g.beta_re, bi = (W)g.beta_im;
        const W cr = c2[0], ci = c2[1];
        c2[0] = fma(br, cr, fma(-bi, ci, tr));
        c2[1] = fma(br, ci, fma(bi, cr, ti));
    }
}

template <class T>
__device__ __forceinline__ void update_cplx(const GemmArgs &g, int64_t i, int64_t j, T re, T im) {
    if (i >= g.m || j >= g.n) return;
    const int64_t off = 2 * (i + j * g.ldc);
    const T ar = (T)g.alpha_re, ai = (T)g.alpha_im;
    if (g.c_dbl) {
        double *c = (double *)g.C + off;
        // beta is already double (C's precision); product in double.
        cupdate<T, double>(g, c, (double)re, (double)im, (double)ar, (double)ai);
    } else if constexpr (sizeof(T) == 8) {
        // computation in double, C single: beta cast to single, update in double
        float *c = (float *)g.C + off;
        const double br = (double)(float)g.beta_re, bi = (double)(float)g.beta_im;
        const double tr = fma(ar, re, -(ai * im));
        const double ti = fma(ar, im, ai * re);
        double rr = tr, ri = ti;
        if (!g.beta_zero) {
            const double cr = c[0], ci = c[1];
            rr = fma(br, cr, fma(-bi, ci, tr));
            ri = fma(br, ci, fma(bi, cr, ti));
        }
        c[0] = (float)rr;
        c[1] = (float)ri;
    } else {
        float *c = (float *)g.C + off;
        cupdate<T, float>(g, c, re, im, ar, ai);
    }
}

// ---------------------------------------------------------------------------
// The product kernel
// ---------------------------------------------------------------------------
template <class T, int CS>
__global__ __launch_bounds__(NT, 2) void md_gemm_kernel(GemmArgs g) {
    typedef TileCfg<T> C;
    typedef Stage<T, CS, true> SA;
    typedef Stage<T, CS, false> SB;
    typedef typename AccT<T>::type acc_t;
    static_assert(SA::TK == SB::TK, "A and B disagree on the k lowering");
    constexpr bool MDBL = SA::MN2, NDBL = SB::MN2;
    constexpr bool CCPLX = (CS == MD_CASE_1C || CS == MD_CASE_2AC || CS == MD_CASE_2BC || CS == MD_CASE_3);

    __shared__ T sA[2][C::BK * SA::LDW];
    __shared__ T sB[2][C::BK * SB::LDW];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave & 1) * 64, wn0 = (wave >> 1) * 64;
    int tm, tn;
    map_tile(blockIdx.x, gridDim.x, g.tiles_m, g.tiles_n, &tm, &tn);
    const int64_t mn0a = (int64_t)tm * SA::TMN, mn0b = (int64_t)tn * SB::TMN;
    const int nk = (int)((g.k + SA::TK - 1) / SA::TK);

    acc_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    SA la;
    SB lb;
    la.load(g, mn0a, 0, tid);
    lb.load(g, mn0b, 0, tid);
    la.store(g, sA[0], tid);
    lb.store(g, sB[0], tid);
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) {
            la.load(g, mn0a, (int64_t)(kt + 1) * SA::TK, tid);
            lb.load(g, mn0b, (int64_t)(kt + 1) * SB::TK, tid);
        }
        const T *pa = sA[cur];
        const T *pb = sB[cur];
#pragma unroll
        for (int s = 0; s < C::BK / 4; ++s) {
            const int kr = s * 4 + (lane >> 4);
            T fa[4], fb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) fa[i] = pa[kr * SA::LDW + wm0 + i * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i) fb[i] = pb[kr * SB::LDW + wn0 + i * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = mfma16(fb[b], fa[a], acc[a][b]);
        }
        if (more) {
            la.store(g, sA[cur ^ 1], tid);
            lb.store(g, sB[cur ^ 1], tid);
        }
        __syncthreads();
    }

    // Epilogue.  acc[a][b] item v is C'(row m = wm0 + 16a + (lane & 15),
    //                                   col n = wn0 + 16b + acc_row(lane, v)).
    const int ml = lane & 15;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int nl = acc_row<T>(lane, v);
            if constexpr (MDBL) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int64_t i = (int64_t)tm * SA::TMN + wm0 / 2 + q * 16 + ml;
                    const int64_t j = (int64_t)tn * SB::TMN + wn0 + b * 16 + nl;
                    update_cplx<T>(g, i, j, acc[2 * q][b][v], acc[2 * q + 1][b][v]);
                }
            } else if constexpr (NDBL) {
                if ((b & 1) == 0) {
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const int64_t i = (int64_t)tm * SA::TMN + wm0 + a * 16 + ml;
                        const int64_t j = (int64_t)tn * SB::TMN + wn0 / 2 + (b / 2) * 16 + nl;
                        update_cplx<T>(g, i, j, acc[a][b][v], acc[a][b + 1][v]);
                    }
                }
            } else {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int64_t i = (int64_t)tm * SA::TMN + wm0 + a * 16 + ml;
                    const int64_t j = (int64_t)tn * SB::TMN + wn0 + b * 16 + nl;
                    if constexpr (CCPLX) update_cplx<T>(g, i, j, acc[a][b][v], (T)0);
                    else update_real<T>(g, i, j, acc[a][b][v]);
                }
            }
        }
    }
}

// C := beta*C (alpha == 0 or k == 0).  beta == 0 writes zeros without reading C.
__global__ __launch_bounds__(256) void md_scale_kernel(GemmArgs g) {
    const int64_t total = g.m * g.n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t % g.m, j = t / g.m;
        const int64_t off = i + j * g.ldc;
        if (g.c_cplx) {
            if (g.c_dbl) {
                double *c = (double *)g.C + 2 * off;
                if (g.beta_zero) { c[0] = 0.0; c[1] = 0.0; }
                else {
                    const double br = g.beta_re, bi = g.beta_im, cr = c[0], ci = c[1];
                    c[0] = fma(br, cr, -(bi * ci));
                    c[1] = fma(br, ci, bi * cr);
                }
            } else {
                float *c = (float *)g.C + 2 * off;
                if (g.beta_zero) { c[0] = 0.0f; c[1] = 0.0f; }
                else {
                    const float br = (float)g.beta_re, bi = (float)g.beta_im, cr = c[0], ci = c[1];
                    c[0] = fmaf(br, cr, -(bi * ci));
                    c[1] = fmaf(br, ci, bi * cr);
                }
            }
        } else if (g.c_dbl) {
            double *c = (double *)g.C;
            c[off] = g.beta_zero ? 0.0 : g.beta_re * c[off];
        } else {
            float *c = (float *)g.C;
            c[off] = g.beta_zero ? 0.0f : (float)g.beta_re * c[off];
        }
    }
}

// ---------------------------------------------------------------------------
// Host-side launch helpers
// ---------------------------------------------------------------------------
template <class T, int CS>
static int launch_t(const GemmArgs &a, hipStream_t s, int64_t *wg) {
    const int64_t n = (int64_t)a.tiles_m * a.tiles_n;
    if (wg) *wg = n;
    if (n <= 0) return 0;
    hipLaunchKernelGGL((md_gemm_kernel<T, CS>), dim3((unsigned)n), dim3(NT), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : MD_ERR_HIP;
}

template <class T>
static int launch_case(int cs, const GemmArgs &a, hipStream_t s, int64_t *wg) {
    switch (cs) {
    case MD_CASE_0: return launch_t<T, MD_CASE_0>(a, s, wg);
    case MD_CASE_1A: return launch_t<T, MD_CASE_1A>(a, s, wg);
    case MD_CASE_1B: return launch_t<T, MD_CASE_1B>(a, s, wg);
    case MD_CASE_1C: return launch_t<T, MD_CASE_1C>(a, s, wg);
    case MD_CASE_2AB: return launch_t<T, MD_CASE_2AB>(a, s, wg);
    case MD_CASE_2AC: return launch_t<T, MD_CASE_2AC>(a, s, wg);
    case MD_CASE_2BC: return launch_t<T, MD_CASE_2BC>(a, s, wg);
    case MD_CASE_3: return launch_t<T, MD_CASE_3>(a, s, wg);
    }
    return MD_ERR_UNSUPPORTED;
}

int launch_gemm(int prec, int cs, const GemmArgs &a, void *stream, int64_t *wg) {
    hipStream_t s = (hipStream_t)stream;
    if (prec == PREC_D) return launch_case<double>(cs, a, s, wg);
    if (prec == PREC_S) return launch_case<float>(cs, a, s, wg);
    return MD_ERR_UNSUPPORTED;
}

int launch_scale(const GemmArgs &a, void *stream) {
    const int64_t total = a.m * a.n;
    if (total <= 0) return 0;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(md_scale_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? 0 : MD_ERR_HIP;
}

void tile_shape(int prec, int cs, int *bm, int *bn, int *bk) {
    (void)cs;
    if (prec == PREC_D) {
        *bm = TileCfg<double>::BM; *bn = TileCfg<double>::BN; *bk = TileCfg<double>::BK;
    } else {
        *bm = TileCfg<float>::BM; *bn = TileCfg<float>::BN; *bk = TileCfg<float>::BK;
    }
}

const char *kernel_name(int prec, int cs) {
    static const char *names[2][8] = {
        {"md_gemm_f32_case0", "md_gemm_f32_case1a", "md_gemm_f32_case1b", "md_gemm_f32_case1c",
         "md_gemm_f32_case2ab", "md_gemm_f32_case2ac", "md_gemm_f32_case2bc", "md_gemm_f32_case3"},
        {"md_gemm_f64_case0", "md_gemm_f64_case1a", "md_gemm_f64_case1b", "md_gemm_f64_case1c",
         "md_gemm_f64_case2ab", "md_gemm_f64_case2ac", "md_gemm_f64_case2bc", "md_gemm_f64_case3"}};
    if (prec < 0 || prec > 1 || cs < 0 || cs > 7) return "none";
    return names[prec][cs];
}

}  // namespace md
