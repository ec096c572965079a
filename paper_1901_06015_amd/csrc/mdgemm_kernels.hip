// mdgemm_kernels.hip -- instantiations of the product kernel (md_tile.h).
//
// Compiled once per (computation precision, domain case) with
// -DMD_KT=<0 single | 1 double | 2 BF16x3 | 3 half> and -DMD_KCASE=<md_case> so
// that the variants (4 computation precisions x 8 cases x 4 storage precisions
// of A and B x 5 load paths: the fast path for each of the 4 operand
// orientations and the generic path) build in parallel.
#include "md_small.h"
#include "md_tile.h"
#include "md_tile_bf16.h"

#ifndef MD_KT
#error "MD_KT must be defined"
#endif
#ifndef MD_KCASE
#error "MD_KCASE must be defined"
#endif

namespace md {

// MD_KT: 0 = single (FP32 MFMA), 1 = double (FP64 MFMA), 2 = BF16x3, 3 = half (FP16 MFMA).
#if MD_KT == 1
typedef double KT;
#else
typedef float KT;
#endif

template <int CS, bool FAST, bool AD, bool BD, bool AMNC, bool BMNC, bool RAG, bool SCL, bool SH = false>
static void launch_k(const GemmArgs &a, hipStream_t s, unsigned nwg) {
#if MD_KT == 2 || MD_KT == 3
    constexpr bool H16 = MD_KT == 3;
    if constexpr (H16 && tile_kind(PREC_H, CS, FAST) == 4)
        hipLaunchKernelGGL((md_bf16x3_kernel<CS, FAST, AD, BD, AMNC, BMNC, Big<float>, RAG, SCL, H16, SH>), dim3(nwg),
                           dim3(Big<float>::NT), 0, s, a);
    else if constexpr (tile_kind(H16 ? PREC_H : PREC_BF16X3, CS, FAST) == 3)
        hipLaunchKernelGGL((md_bf16x3_kernel<CS, FAST, AD, BD, AMNC, BMNC, Deep<float>, RAG, SCL, H16, SH>), dim3(nwg),
                           dim3(Deep<float>::NT), 0, s, a);
    else
        hipLaunchKernelGGL((md_bf16x3_kernel<CS, FAST, AD, BD, AMNC, BMNC, TileCfg<float>, RAG, SCL, H16, SH>),
                           dim3(nwg), dim3(NT), 0, s, a);
#else
    constexpr int kind = tile_kind(MD_KT == 1 ? PREC_D : PREC_S, CS, FAST);
    if constexpr (kind == 1)
        hipLaunchKernelGGL((md_gemm_kernel<KT, CS, FAST, AD, BD, AMNC, BMNC, WideN<KT>, RAG, SCL, SH>), dim3(nwg),
                           dim3(WideN<KT>::NT), 0, s, a);
    else if constexpr (kind == 2)
        hipLaunchKernelGGL((md_gemm_kernel<KT, CS, FAST, AD, BD, AMNC, BMNC, WideM<KT>, RAG, SCL, SH>), dim3(nwg),
                           dim3(WideM<KT>::NT), 0, s, a);
    else if constexpr (kind == 3)
        hipLaunchKernelGGL((md_gemm_kernel<KT, CS, FAST, AD, BD, AMNC, BMNC, Deep<KT>, RAG, SCL, SH>), dim3(nwg),
                           dim3(Deep<KT>::NT), 0, s, a);
    else
        hipLaunchKernelGGL((md_gemm_kernel<KT, CS, FAST, AD, BD, AMNC, BMNC, TileCfg<KT>, RAG, SCL, SH>), dim3(nwg),
                           dim3(NT), 0, s, a);
#endif
}

template <int CS, bool FAST, bool AMNC, bool BMNC, bool RAG, bool SCL>
static void launch_v(const GemmArgs &a, hipStream_t s, unsigned nwg) {
#if MD_KT == 0 || MD_KT == 3
    // binary16 A and B on the fast path (single and half precision only)
    if constexpr (FAST) {
        if (a.a_half) {
            launch_k<CS, FAST, false, false, AMNC, BMNC, RAG, SCL, true>(a, s, nwg);
            return;
        }
    }
#endif
    if (a.a_dbl) {
        if (a.b_dbl) launch_k<CS, FAST, true, true, AMNC, BMNC, RAG, SCL>(a, s, nwg);
        else launch_k<CS, FAST, true, false, AMNC, BMNC, RAG, SCL>(a, s, nwg);
    } else {
        if (a.b_dbl) launch_k<CS, FAST, false, true, AMNC, BMNC, RAG, SCL>(a, s, nwg);
        else launch_k<CS, FAST, false, false, AMNC, BMNC, RAG, SCL>(a, s, nwg);
    }
}

// The fast kernels take the operands' orientation (A contiguous along m for
// 'N'/'R', B contiguous along n for 'T'/'C') as template parameters, and a ragged
// variant for operands stored along k whose columns end inside a chunk (never
// the case when both are stored along m/n); the generic kernels read the
// orientation from the arguments.
template <int CS, bool SCL>
static void launch_o(const GemmArgs &a, hipStream_t s, unsigned nwg) {
    if (a.a_vec && a.b_vec) {
        const bool am = a.ta == 0 || a.ta == 3, bm = a.tb == 1 || a.tb == 2, rag = a.a_ragged || a.b_ragged;
        if (am) {
            if (bm) launch_v<CS, true, true, true, false, SCL>(a, s, nwg);
            else if (rag) launch_v<CS, true, true, false, true, SCL>(a, s, nwg);
            else launch_v<CS, true, true, false, false, SCL>(a, s, nwg);
        } else {
            if (bm) {
                if (rag) launch_v<CS, true, false, true, true, SCL>(a, s, nwg);
                else launch_v<CS, true, false, true, false, SCL>(a, s, nwg);
            } else {
                if (rag) launch_v<CS, true, false, false, true, SCL>(a, s, nwg);
                else launch_v<CS, true, false, false, false, SCL>(a, s, nwg);
            }
        }
    } else {
        launch_v<CS, false, true, true, false, SCL>(a, s, nwg);
    }
}

// Cases 1a, 1b and 2ab also have the variants that stage their complex operand
// scaled by a complex alpha (the literal interpretation with C real).
template <int CS>
static void launch_c(const GemmArgs &a, hipStream_t s, unsigned nwg) {
    if constexpr (CS == MD_CASE_1A || CS == MD_CASE_1B || CS == MD_CASE_2AB) {
        if (a.a_scale || a.b_scale) {
            launch_o<CS, true>(a, s, nwg);
            return;
        }
    }
    launch_o<CS, false>(a, s, nwg);
}

#define MD_PART_NAME2(t, c) launch_part_##t##_##c
#define MD_PART_NAME(t, c) MD_PART_NAME2(t, c)
#define MD_SMALL_NAME2(t, c) launch_small_##t##_##c
#define MD_SMALL_NAME(t, c) MD_SMALL_NAME2(t, c)

void MD_PART_NAME(MD_KT, MD_KCASE)(const GemmArgs &a, hipStream_t s, unsigned nwg) {
    launch_c<MD_KCASE>(a, s, nwg);
}

#if MD_KT == 0 || MD_KT == 1
// The small kernel of this precision and case, for each storage precision of
// A and B.
void MD_SMALL_NAME(MD_KT, MD_KCASE)(const GemmArgs &a, hipStream_t s, unsigned nwg) {
    if (a.a_dbl) {
        if (a.b_dbl) hipLaunchKernelGGL((md_small_kernel<KT, MD_KCASE, true, true>), dim3(nwg), dim3(SM_NT), 0, s, a);
        else hipLaunchKernelGGL((md_small_kernel<KT, MD_KCASE, true, false>), dim3(nwg), dim3(SM_NT), 0, s, a);
    } else {
        if (a.b_dbl) hipLaunchKernelGGL((md_small_kernel<KT, MD_KCASE, false, true>), dim3(nwg), dim3(SM_NT), 0, s, a);
        else hipLaunchKernelGGL((md_small_kernel<KT, MD_KCASE, false, false>), dim3(nwg), dim3(SM_NT), 0, s, a);
    }
}
#endif

}  // namespace md
