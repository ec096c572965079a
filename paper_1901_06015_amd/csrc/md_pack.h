// md_pack.h -- BF16x3 on packed operands, for products large enough to fill
// the GPU with 256 x 256 tiles.
//
// The typecasting pack of Section 5 done once per call instead of once per
// tile: md_pack_x3_kernel reads each operand of the real product (Figure
// "mixeddom" lowering, element by element as md_small.h does), casts it to
// FP32, splits it into bf16 hi = RNE(a) and lo = RNE(a - hi) and writes both
// planes in the layout the multiply kernel's LDS tiles use.  The multiply
// kernel then copies packed tiles from HBM straight into LDS (gfx950 direct
// 16-byte loads, no registers and no conversion in the k loop) and runs the
// three bf16 MFMAs per block of md_bf16x3_kernel in the same order (on exact
// inputs its results equal the plain definition bit for bit).
#pragma once
#include "md_small.h"
#include "md_tile_bf16.h"

namespace md {

// MD_PACK_FAST=0: every block through the general (range-checked,
// element-wise) path; build option, measured against the default.
#ifndef MD_PACK_FAST
#define MD_PACK_FAST 1
#endif
constexpr int PK_ROWS = 256;                   // rows (m' or n') of a packed block
constexpr int PK_K = 32;                       // k' of a packed block
constexpr int PK_BLOCK = PK_ROWS * PK_K * 2;   // bytes of one plane of one block (16 KB)

// Packed layout of an operand X' of the real product (rows along m' for A',
// along n' for B'; k' the depth), both padded with zeros to whole blocks:
// block (rb, kb) of plane p (0 = hi, 1 = lo) at byte ((rb * nkb + kb) * 2 +
// p) * PK_BLOCK.  Inside a block, row r holds its 32 k as four 16-byte chunks;
// chunk q (k = 8q .. 8q+7) of row r is the 16-byte unit number pk_chunk(r, q):
// the 16 lanes of an MFMA fragment (rows r0 .. r0+15, one q) then read 16
// distinct groups of 4 LDS banks.
__host__ __device__ constexpr int pk_chunk(int r, int q) { return 4 * r + (q ^ ((r >> 2) & 3)); }

// Split the FP32 values of a thread's four chunks into bf16 hi and lo and
// store both planes.
__device__ __forceinline__ void pack_store(const float (&v)[4][8], const int (&cr)[4], const int (&cq)[4], char *hi,
                                           char *lo) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        bf16x8 h, l;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const __bf16 vh = (__bf16)v[c][j];
            h[j] = vh;
            l[j] = (__bf16)(v[c][j] - (float)vh);
        }
        *(bf16x8 *)(hi + pk_chunk(cr[c], cq[c]) * 16) = h;
        *(bf16x8 *)(lo + pk_chunk(cr[c], cq[c]) * 16) = l;
    }
}

// A block wholly inside the matrix (the common case): no range checks, and
// offsets within 2 GiB of the block's first stored element, so buffer loads
// with 32-bit offsets.  Stored along k, a chunk's 8 elements are one run of
// stored components (8 for the plain and k-interleaved lowerings, 16 taking
// every other for the Re-only and m/n-interleaved ones) read with 16-byte
// loads (4-byte alignment suffices); stored along m' or n', one load per
// element as in the general path, its k offset in a scalar register.
template <int CS, bool IS_A, bool SDBL, bool MNC>
__device__ __forceinline__ void pack_inside(const SmallOp<float, CS, IS_A, SDBL> &op, int64_t r0, int64_t k0,
                                            const int (&cr)[4], const int (&cq)[4], char *hi, char *lo) {
    typedef SmallOp<float, CS, IS_A, SDBL> Op;
    constexpr int ESZ = SDBL ? 8 : 4, W = Op::W, MODE = Op::MODE;
    constexpr bool MN2 = Op::MN2, K2 = Op::K2;
    // stored index (column or row) of real row r, and its part (Re 0, Im 1)
    auto row_of = [](int64_t r, int *qm) {
        *qm = MN2 ? (int)((r >> 4) & 1) : 0;
        return MN2 ? (((r >> 5) << 4) | (r & 15)) : r;
    };
    const int64_t i0 = MN2 ? ((r0 >> 5) << 4) : r0, p0 = K2 ? (k0 >> 1) : k0;
    const char *base = op.base + (MNC ? (i0 + p0 * op.ld) : (p0 + i0 * op.ld)) * W * ESZ;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, 0x7fffffff, 0x00020000);
    float v[4][8];
    if constexpr (!MNC) {
        constexpr bool STRIDE2 = (W == 2 && !K2);
        constexpr int NV = (STRIDE2 ? 16 : 8) * ESZ / 16;  // 16-byte loads per chunk
        uint32_t w[4][4 * NV];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            int qm;
            const int64_t i = row_of(r0 + cr[c], &qm);
            const int64_t kk0 = k0 + 8 * cq[c], pc = K2 ? (kk0 >> 1) : kk0;
            const uint32_t off = (uint32_t)(((i - i0) * op.ld + (pc - p0)) * W * ESZ);
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const auto x = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(off + 16 * q), 0, 0);
                w[c][4 * q] = x[0];
                w[c][4 * q + 1] = x[1];
                w[c][4 * q + 2] = x[2];
                w[c][4 * q + 3] = x[3];
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            int qm;
            const int64_t r = r0 + cr[c];
            (void)row_of(r, &qm);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                // component of element j within the run: its position, or
                // the pair partner for the 1e lowering's odd rows (Im first),
                // or every other component (offset by the part for m/n pairs)
                int e0, e1;
                if constexpr (K2) {
                    e0 = j;
                    e1 = (MODE == M_ONEE) ? (j ^ 1) : j;
                } else if constexpr (STRIDE2) {
                    e0 = 2 * j;
                    e1 = (MODE == M_MNINT) ? 2 * j + 1 : 2 * j;
                } else {
                    e0 = e1 = j;
                }
                // both candidates as registers before the select (a select
                // of two array elements would become an indexed access and
                // put the array in scratch)
                constexpr bool SEL = (K2 && MODE == M_ONEE) || (STRIDE2 && MODE == M_MNINT);
                uint32_t lo_w, hi_w = 0;
                if constexpr (!SEL) {
                    lo_w = w[c][SDBL ? 2 * e0 : e0];
                    if constexpr (SDBL) hi_w = w[c][2 * e0 + 1];
                } else if constexpr (SDBL) {
                    uint32_t a0 = w[c][2 * e0], a1 = w[c][2 * e0 + 1], b0 = w[c][2 * e1], b1 = w[c][2 * e1 + 1];
                    asm("" : "+v"(a0), "+v"(a1), "+v"(b0), "+v"(b1));
                    lo_w = qm ? b0 : a0;
                    hi_w = qm ? b1 : a1;
                } else {
                    uint32_t a0 = w[c][e0], b0 = w[c][e1];
                    asm("" : "+v"(a0), "+v"(b0));
                    lo_w = qm ? b0 : a0;
                }
                bool valid, neg;
                (void)op.where(r, k0 + 8 * cq[c] + j, true, &valid, &neg);
                v[c][j] = Op::value(lo_w, hi_w, true, neg);
            }
        }
    } else {
        uint32_t wl[4][8], wh[4][8];
        int qm;
        const int64_t i = row_of(r0 + cr[0], &qm);
        const uint32_t lane_off = (uint32_t)((i - i0) * W * ESZ);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int64_t kk = k0 + 8 * cq[c] + j, p = K2 ? (kk >> 1) : kk;
                const int qk = K2 ? (int)(kk & 1) : 0;
                const int comp = MODE == M_KINT ? qk : MODE == M_MNINT ? qm : MODE == M_ONEE ? (qm ^ qk) : 0;
                const int koff = (int)((p - p0) * op.ld * W * ESZ);
                const uint32_t off = lane_off + (uint32_t)(comp * ESZ);
                if constexpr (SDBL) {
                    const auto x = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, koff, 0);
                    wl[c][j] = x[0];
                    wh[c][j] = x[1];
                } else {
                    wl[c][j] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, koff, 0);
                    wh[c][j] = 0;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                bool valid, neg;
                (void)op.where(r0 + cr[c], k0 + 8 * cq[c] + j, true, &valid, &neg);
                v[c][j] = Op::value(wl[c][j], wh[c][j], true, neg);
            }
    }
    pack_store(v, cr, cq, hi, lo);
}

// One workgroup per packed block (blk = rb * nkb + kb): 32 elements of
// the real product's operand per row, cast to FP32 as the staging of
// md_tile.h does (double -> float rounds to nearest even), split and stored;
// elements outside the matrix are zero.  The threads follow the operand's
// storage (MNC: stored along m' or n', as the operation makes it; chosen by
// the host): for an operand stored along m' or n' one thread per row (lanes of
// a load read consecutive rows: consecutive addresses); for one stored along
// k four consecutive lanes take the four 8-element chunks of one row (16
// rows of 32 consecutive elements per wave).  Blocks wholly inside the
// matrix take pack_inside; on the edges each thread issues all 32 element
// loads before converting (the output is restrict, so no store holds a load
// back).
template <int CS, bool IS_A, bool SDBL, bool MNC>
__device__ __forceinline__ void pack_block(const GemmArgs &g, char *__restrict__ out, int nkb, unsigned blk) {
    typedef SmallOp<float, CS, IS_A, SDBL> Op;
    const Op op(g);
    const int rb = (int)(blk / (unsigned)nkb), kb = (int)(blk % (unsigned)nkb);
    const int tid = threadIdx.x;
    const int64_t k0 = (int64_t)kb * PK_K;
    char *hi = out + (int64_t)blk * 2 * PK_BLOCK, *lo = hi + PK_BLOCK;
    // this thread's four chunks: (block row, chunk index)
    int cr[4], cq[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        cr[c] = MNC ? tid : c * (PK_ROWS / 4) + (tid >> 2);
        cq[c] = MNC ? c : (tid & 3);
    }
    {
        // the block's last stored row (or column) and k, and the byte span
        // of its stored elements from the first: inside the matrix and
        // within 2 GiB, take the fast path (uniform across the workgroup)
        const int64_t r0 = (int64_t)rb * PK_ROWS, rl = r0 + PK_ROWS - 1;
        const int64_t il = Op::MN2 ? (((rl >> 5) << 4) | 15) : rl;
        const int64_t pl = Op::K2 ? ((k0 + PK_K - 1) >> 1) : (k0 + PK_K - 1);
        const int64_t irange = il - (Op::MN2 ? ((r0 >> 5) << 4) : r0), prange = pl - (Op::K2 ? (k0 >> 1) : k0);
        const int64_t span = ((MNC ? (irange + prange * op.ld) : (prange + irange * op.ld)) * Op::W + 2) *
                             (SDBL ? 8 : 4);
        if (MD_PACK_FAST && il < op.MN && pl < op.K && op.mnc == MNC && span < 0x7fff0000LL) {
            pack_inside<CS, IS_A, SDBL, MNC>(op, r0, k0, cr, cq, hi, lo);
            return;
        }
    }
    uint32_t wlo[4][8], whi[4][8];
    uint32_t vmask = 0, nmask = 0;
    // a block on the matrix's edge: every element's offset and validity
    // formed separately, elements outside reading the first (and counting
    // as zero)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            bool valid, neg;
            const int64_t off = op.where((int64_t)rb * PK_ROWS + cr[c], k0 + 8 * cq[c] + j, true, &valid, &neg);
            vmask |= (uint32_t)valid << (8 * c + j);
            nmask |= (uint32_t)neg << (8 * c + j);
            whi[c][j] = 0;
            op.issue(off, &wlo[c][j], &whi[c][j]);
        }
    }
    float v[4][8];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = 8 * c + j;
            v[c][j] = Op::value(wlo[c][j], whi[c][j], (vmask >> e) & 1, (nmask >> e) & 1);
        }
    pack_store(v, cr, cq, hi, lo);
}

// One launch packs both operands: blocks [0, na) are A' blocks, the rest B'
// blocks (the two packs overlap instead of running one after the other).
template <int CS, bool AD, bool AMNC, bool BD, bool BMNC>
__global__ __launch_bounds__(PK_ROWS) void md_pack_x3_kernel(GemmArgs g, char *__restrict__ pa,
                                                             char *__restrict__ pb, int nkb, unsigned na) {
    if (blockIdx.x < na) pack_block<CS, true, AD, AMNC>(g, pa, nkb, blockIdx.x);
    else pack_block<CS, false, BD, BMNC>(g, pb, nkb, blockIdx.x - na);
}

// MD_PX_TWO_BARRIERS: refill a stage two tiles ahead behind a second
// barrier per k-tile instead of one tile ahead behind the first (build
// option; measured against the default).
#ifndef MD_PX_TWO_BARRIERS
#define MD_PX_TWO_BARRIERS 0
#endif
// MD_PX_WAVES=4: 4 waves of 128 x 128 (a third fewer LDS reads per flop,
// accumulators in AGPRs, one wave per SIMD); build option, measured 0.93x
// the default 8 waves of 64 x 128 with MD_PX_PIPE=0 (with the default
// MD_PX_PIPE its two register sets of A fragments do not fit and spill).
#ifndef MD_PX_WAVES
#define MD_PX_WAVES 8
#endif
// MD_PX_PIPE=0: one barrier at the top of each k-tile, then its fragment
// reads in the compiler's schedule (all of A and two B blocks before the
// first MFMA, each later B block just before its MFMAs); build option,
// measured against the default.
#ifndef MD_PX_PIPE
#define MD_PX_PIPE 1
#endif
constexpr int PX_WGM = MD_PX_WAVES == 4 ? 2 : 4, PX_WGN = 2;
constexpr int PX_WMB = PK_ROWS / (16 * PX_WGM), PX_WNB = PK_ROWS / (16 * PX_WGN);  // blocks per wave
constexpr int PX_NT = 64 * PX_WGM * PX_WGN;
constexpr int PX_CPT = 2 * PK_BLOCK / 16 / PX_NT;  // 16-byte chunks per thread per operand and k-tile
constexpr int PX_WAVES_PER_SIMD = PX_NT / 64 / 4;
static_assert(!MD_PX_TWO_BARRIERS || PX_CPT == 4, "the two-barrier loop waits for 8 copies per thread");
static_assert(!(MD_PX_TWO_BARRIERS && MD_PX_PIPE), "MD_PX_TWO_BARRIERS is a variant of the MD_PX_PIPE=0 loop");
static_assert(!MD_PX_PIPE || PX_WNB % 2 == 0, "the last B block and the next tile's first share no register");
constexpr int PX_STAGE = 4 * PK_BLOCK;

template <int CS>
__global__ __launch_bounds__(PX_NT, PX_WAVES_PER_SIMD) void md_packed_x3_kernel(GemmArgs g, const char *pa, const char *pb,
                                                                int nkb) {
    typedef __attribute__((address_space(3))) void lds_void;
    __shared__ __attribute__((aligned(16))) char lds[2 * PX_STAGE];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % PX_WGM) * (PK_ROWS / PX_WGM), wn0 = (wave / PX_WGM) * (PK_ROWS / PX_WGN);
    int tm, tn;
    map_tile(blockIdx.x, gridDim.x, g.tiles_m, g.tiles_n, &tm, &tn);
    // this tile's row blocks: nkb (hi, lo) block pairs each, k-tile t at 2 t blocks
    const char *ga = pa + (int64_t)tm * nkb * 2 * PK_BLOCK;
    const char *gb = pb + (int64_t)tn * nkb * 2 * PK_BLOCK;

    // k-tile t into stage s: 2 x 2048 chunks, chunk c * PX_NT + tid of each
    // operand by this thread; a wave's 64 chunks of one load land contiguously
    auto issue = [&](int t, int s) {
        char *st = lds + s * PX_STAGE;
#pragma unroll
        for (int c = 0; c < PX_CPT; ++c) {
            const int ch = c * PX_NT + tid, wch = c * PX_NT + wave * 64;
            __builtin_amdgcn_global_load_lds((const void *)(ga + (int64_t)t * 2 * PK_BLOCK + ch * 16),
                                             (lds_void *)(st + wch * 16), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void *)(gb + (int64_t)t * 2 * PK_BLOCK + ch * 16),
                                             (lds_void *)(st + 2 * PK_BLOCK + wch * 16), 16, 0, 0);
        }
    };
    // fragment of rows r0 .. r0+15 (this lane's row r0 + (lane & 15)), k = 8 (lane >> 4) .. +7
    auto frag = [&](const char *plane, int r0) {
        const int r = r0 + (lane & 15);
        return *(const bf16x8 *)(plane + pk_chunk(r, lane >> 4) * 16);
    };

    v4f acc[PX_WMB][PX_WNB];
#pragma unroll
    for (int a = 0; a < PX_WMB; ++a)
#pragma unroll
        for (int b = 0; b < PX_WNB; ++b) acc[a][b] = v4f{0, 0, 0, 0};

#if MD_PX_PIPE
    // Fragments are read one step ahead of their MFMAs: B block b+1 right
    // after the first MFMA of block b, and the next k-tile's A and B block 0
    // (into the other register set) right after the first MFMA of the last
    // block.  The compiler's waits here are for every outstanding LDS read,
    // so each group of reads is issued just after a wait and has the rest of
    // a block (3 * PX_WMB - 1 MFMAs) to arrive.  The k loop is unrolled by 2
    // so that the register set is known at compile time.
    bf16x8 ah[2][PX_WMB], al[2][PX_WMB], bh[2], bl[2];
    auto read_a = [&](const char *st, auto set_tag) {
        constexpr int P = decltype(set_tag)::value;
#pragma unroll
        for (int a = 0; a < PX_WMB; ++a) {
            ah[P][a] = frag(st, wm0 + 16 * a);
            al[P][a] = frag(st + PK_BLOCK, wm0 + 16 * a);
        }
    };
    auto read_b = [&](const char *st, int b, int q) {
        bh[q] = frag(st + 2 * PK_BLOCK, wn0 + 16 * b);
        bl[q] = frag(st + 3 * PK_BLOCK, wn0 + 16 * b);
    };
    // the three products of block (a, b), from product `from` on
    auto mfma_b = [&](auto set_tag, int b, int a, int from = 0) {
        constexpr int P = decltype(set_tag)::value;
        if (from <= 0) acc[a][b] = mfma_bf16(bl[b & 1], ah[P][a], acc[a][b]);
        if (from <= 1) acc[a][b] = mfma_bf16(bh[b & 1], al[P][a], acc[a][b]);
        acc[a][b] = mfma_bf16(bh[b & 1], ah[P][a], acc[a][b]);
    };
    // k-tile t, held in stage P = t & 1 and register set P
    auto ktile = [&](auto set_tag, int t) {
        constexpr int P = decltype(set_tag)::value;
        const char *st = lds + P * PX_STAGE, *nx = lds + (P ^ 1) * PX_STAGE;
#pragma unroll
        for (int b = 0; b < PX_WNB; ++b) {
            // the first product of the block, then the reads
            acc[0][b] = mfma_bf16(bl[b & 1], ah[P][0], acc[0][b]);
            if (b + 1 < PX_WNB) {
                read_b(st, b + 1, (b + 1) & 1);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
            } else if (t + 1 < nkb) {
                // every read of stage P is done (block b's B was waited for
                // by the MFMA above) and tile t+1 has landed for every wave:
                // refill stage P with tile t+2, read tile t+1's first
                // fragments while this block multiplies
                asm volatile("s_waitcnt lgkmcnt(0)\n\ts_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
                if (t + 2 < nkb) issue(t + 2, P);
                read_b(nx, 0, 0);
                read_a(nx, std::integral_constant<int, P ^ 1>{});
                __builtin_amdgcn_sched_group_barrier(0x100, 2 + 2 * PX_WMB, 0);
            }
            mfma_b(set_tag, b, 0, 1);
#pragma unroll
            for (int a = 1; a < PX_WMB; ++a) mfma_b(set_tag, b, a);
            __builtin_amdgcn_sched_group_barrier(0x008, 3 * PX_WMB - 1, 0);
            // keep the next block's MFMAs (and their wait) behind this one's
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    issue(0, 0);
    asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
    if (nkb > 1) issue(1, 1);
    read_b(lds, 0, 0);
    read_a(lds, std::integral_constant<int, 0>{});
    for (int t = 0; t < nkb; t += 2) {
        ktile(std::integral_constant<int, 0>{}, t);
        if (t + 1 < nkb) ktile(std::integral_constant<int, 1>{}, t + 1);
    }
#else
#if MD_PX_TWO_BARRIERS
    issue(0, 0);
    if (nkb > 1) issue(1, 1);
#else
    issue(0, 0);
#endif
    for (int t = 0; t < nkb; ++t) {
#if MD_PX_TWO_BARRIERS
        if (t + 1 < nkb) asm volatile("s_waitcnt vmcnt(8)\n\ts_barrier" ::: "memory");
        else asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
#else
        // tile t has landed for every wave, and every wave has finished
        // reading the other stage (tile t-1): refill it with tile t+1 at once,
        // so the copies have this tile's MFMAs to arrive
        asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
        if (t + 1 < nkb) issue(t + 1, (t + 1) & 1);
#endif
        const char *st = lds + (t & 1) * PX_STAGE;
        const char *ah_p = st, *al_p = st + PK_BLOCK, *bh_p = st + 2 * PK_BLOCK, *bl_p = st + 3 * PK_BLOCK;
        bf16x8 ah[PX_WMB], al[PX_WMB];
#pragma unroll
        for (int a = 0; a < PX_WMB; ++a) {
            ah[a] = frag(ah_p, wm0 + 16 * a);
            al[a] = frag(al_p, wm0 + 16 * a);
        }
#pragma unroll
        for (int b = 0; b < PX_WNB; ++b) {
            const bf16x8 bh = frag(bh_p, wn0 + 16 * b), bl = frag(bl_p, wn0 + 16 * b);
#pragma unroll
            for (int a = 0; a < PX_WMB; ++a) {
                acc[a][b] = mfma_bf16(bl, ah[a], acc[a][b]);
                acc[a][b] = mfma_bf16(bh, al[a], acc[a][b]);
                acc[a][b] = mfma_bf16(bh, ah[a], acc[a][b]);
            }
        }
#if MD_PX_TWO_BARRIERS
        // every wave's reads of this stage are done before it is refilled
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        if (t + 2 < nkb) issue(t + 2, t & 1);
#endif
    }
#endif
    constexpr int MODE_A = mode_of<CS, true>(), MODE_B = mode_of<CS, false>();
    constexpr bool MDBL = MODE_A == M_MNINT || MODE_A == M_ONEE, NDBL = MODE_B == M_MNINT || MODE_B == M_ONEE;
    x16_epilogue<CS, false, PX_WMB, PX_WNB>(g, acc, (int64_t)tm * (PK_ROWS / (MDBL ? 2 : 1)),
                                            (int64_t)tn * (PK_ROWS / (NDBL ? 2 : 1)), wm0, wn0, lane);
}

}  // namespace md
