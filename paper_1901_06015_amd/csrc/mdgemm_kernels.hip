// mdgemm_kernels.hip -- instantiations of the product kernel (md_tile.h).
//
// Compiled once per (computation precision, domain case) with
// -DMD_KT=<0 single | 1 double> and -DMD_KCASE=<md_case> so that the 128
// variants (2 computation precisions x 8 cases x 2 load paths x 4 storage
// precisions of A and B) build in parallel.
#include "md_tile.h"

#ifndef MD_KT
#error "MD_KT must be defined"
#endif
#ifndef MD_KCASE
#error "MD_KCASE must be defined"
#endif

namespace md {

#if MD_KT == 0
typedef float KT;
#else
typedef double KT;
#endif

template <int CS, bool FAST>
static void launch_v(const GemmArgs &a, hipStream_t s, unsigned nwg) {
    if (a.a_dbl) {
        if (a.b_dbl) hipLaunchKernelGGL((md_gemm_kernel<KT, CS, FAST, true, true>), dim3(nwg), dim3(NT), 0, s, a);
        else hipLaunchKernelGGL((md_gemm_kernel<KT, CS, FAST, true, false>), dim3(nwg), dim3(NT), 0, s, a);
    } else {
        if (a.b_dbl) hipLaunchKernelGGL((md_gemm_kernel<KT, CS, FAST, false, true>), dim3(nwg), dim3(NT), 0, s, a);
        else hipLaunchKernelGGL((md_gemm_kernel<KT, CS, FAST, false, false>), dim3(nwg), dim3(NT), 0, s, a);
    }
}

template <int CS>
static void launch_c(const GemmArgs &a, hipStream_t s, unsigned nwg) {
    if (a.a_vec && a.b_vec) launch_v<CS, true>(a, s, nwg);
    else launch_v<CS, false>(a, s, nwg);
}

#define MD_PART_NAME2(t, c) launch_part_##t##_##c
#define MD_PART_NAME(t, c) MD_PART_NAME2(t, c)

void MD_PART_NAME(MD_KT, MD_KCASE)(const GemmArgs &a, hipStream_t s, unsigned nwg) {
    launch_c<MD_KCASE>(a, s, nwg);
}

}  // namespace md
