// mdgemm_grouped_kernel.hip -- the persistent kernel of mdgemm_grouped (its
// host side, the work table and the tile order, is mdgemm_grouped.hip).
#include "md_grouped.h"

namespace md {

// The persistent kernel.  `hdr[0]` is the tile counter (zeroed by the host's
// upload of the table); every workgroup exits once the counter passes
// `ntiles`.
__global__ __launch_bounds__(GNT, GROUPED_WAVES) void md_grouped_kernel(const GDesc *__restrict__ descs,
                                                                     const GTile *__restrict__ tiles, int ntiles,
                                                            int *hdr) {
    __shared__ __attribute__((aligned(16))) char smem[GROUPED_SMEM];
    __shared__ int s_t;
    for (;;) {
        if (threadIdx.x == 0) s_t = atomicAdd(hdr, 1);
        __syncthreads();
        // the tile index is uniform across the workgroup: keep it (and the
        // descriptor loads that depend on it) in scalar registers
        const int t = __builtin_amdgcn_readfirstlane(s_t);
        __syncthreads();
        if (t >= ntiles) break;
        const GTile tl = tiles[t];
        const GDesc &d = descs[__builtin_amdgcn_readfirstlane(tl.desc)];
        const int tm = __builtin_amdgcn_readfirstlane(tl.tm), tn = __builtin_amdgcn_readfirstlane(tl.tn);
        if (d.kind == 1) {
            grouped_scale_tile(d.g, tm, tn);
            continue;
        }
        // one routine per (computation precision, tile shape, storage
        // precisions of A and B); everything else is decoded per tile
        const int sel = ((d.prec * GCFG_COUNT + d.cfg) * 2 + d.g.a_dbl) * 2 + d.g.b_dbl;
#define MD_GSEL(p, c, ad, bd) ((((p) * GCFG_COUNT + (c)) * 2 + (ad)) * 2 + (bd))
#define MD_GCASES(p, c, T, SH)                                                                              \
    case MD_GSEL(p, c, 0, 0): grouped_tile<T, SH, false, false>(d, tm, tn, smem); break;                   \
    case MD_GSEL(p, c, 0, 1): grouped_tile<T, SH, false, true>(d, tm, tn, smem); break;                    \
    case MD_GSEL(p, c, 1, 0): grouped_tile<T, SH, true, false>(d, tm, tn, smem); break;                    \
    case MD_GSEL(p, c, 1, 1): grouped_tile<T, SH, true, true>(d, tm, tn, smem); break;
#define MD_GCASES_BF(c)                                                                                     \
    case MD_GSEL(PREC_BF16X3, c, 0, 0): grouped_tile_bf16x3<false, false>(d, tm, tn, smem); break;         \
    case MD_GSEL(PREC_BF16X3, c, 0, 1): grouped_tile_bf16x3<false, true>(d, tm, tn, smem); break;          \
    case MD_GSEL(PREC_BF16X3, c, 1, 0): grouped_tile_bf16x3<true, false>(d, tm, tn, smem); break;          \
    case MD_GSEL(PREC_BF16X3, c, 1, 1): grouped_tile_bf16x3<true, true>(d, tm, tn, smem); break;
        switch (sel) {
            MD_GCASES(PREC_S, GCFG_64, float, GS_S64)
            MD_GCASES(PREC_S, GCFG_128, float, GS_S128)
            MD_GCASES(PREC_S, GCFG_128x64, float, GS_S128x64)
            MD_GCASES(PREC_S, GCFG_64x128, float, GS_S64x128)
            MD_GCASES(PREC_S, GCFG_64K, float, GS_S64K)
            MD_GCASES(PREC_D, GCFG_64, double, GS_D64)
            MD_GCASES(PREC_D, GCFG_128, double, GS_D128)
            MD_GCASES(PREC_D, GCFG_128x64, double, GS_D128x64)
            MD_GCASES(PREC_D, GCFG_64x128, double, GS_D64x128)
            MD_GCASES(PREC_D, GCFG_64K, double, GS_D64K)
            // BF16x3 has a single (64x64) shape in the grouped kernel
            MD_GCASES_BF(GCFG_64)
        default: break;
        }
#undef MD_GCASES_BF
#undef MD_GCASES
#undef MD_GSEL
    }
}

void launch_grouped_kernel(int grid, hipStream_t s, const GDesc *descs, const GTile *tiles, int ntiles,
                           int *hdr) {
    hipLaunchKernelGGL(md_grouped_kernel, dim3(grid), dim3(GNT), 0, s, descs, tiles, ntiles, hdr);
}

}  // namespace md
