// mdgemm_launch.hip -- host-side dispatch to the product kernels, the
// beta-scaling kernel used by the quick returns, and tile/kernel metadata.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <mutex>
#include <utility>

#include "md_half.h"
#include "md_internal.h"
#include "md_tile.h"

namespace md {

#define MD_DECL_PARTS(t)                                                       \
    void launch_part_##t##_0(const GemmArgs &, hipStream_t, unsigned);         \
    void launch_part_##t##_1(const GemmArgs &, hipStream_t, unsigned);         \
    void launch_part_##t##_2(const GemmArgs &, hipStream_t, unsigned);         \
    void launch_part_##t##_3(const GemmArgs &, hipStream_t, unsigned);         \
    void launch_part_##t##_4(const GemmArgs &, hipStream_t, unsigned);         \
    void launch_part_##t##_5(const GemmArgs &, hipStream_t, unsigned);         \
    void launch_part_##t##_6(const GemmArgs &, hipStream_t, unsigned);         \
    void launch_part_##t##_7(const GemmArgs &, hipStream_t, unsigned);
MD_DECL_PARTS(0)
MD_DECL_PARTS(1)
MD_DECL_PARTS(2)
MD_DECL_PARTS(3)

#define MD_DECL_SMALL(t)                                                       \
    void launch_small_##t##_0(const GemmArgs &, hipStream_t, unsigned);        \
    void launch_small_##t##_1(const GemmArgs &, hipStream_t, unsigned);        \
    void launch_small_##t##_2(const GemmArgs &, hipStream_t, unsigned);        \
    void launch_small_##t##_3(const GemmArgs &, hipStream_t, unsigned);        \
    void launch_small_##t##_4(const GemmArgs &, hipStream_t, unsigned);        \
    void launch_small_##t##_5(const GemmArgs &, hipStream_t, unsigned);        \
    void launch_small_##t##_6(const GemmArgs &, hipStream_t, unsigned);        \
    void launch_small_##t##_7(const GemmArgs &, hipStream_t, unsigned);
MD_DECL_SMALL(0)
MD_DECL_SMALL(1)

typedef void (*part_fn)(const GemmArgs &, hipStream_t, unsigned);
// [PREC_S, PREC_D, PREC_BF16X3, PREC_H][case]
static const part_fn kParts[4][8] = {
    {launch_part_0_0, launch_part_0_1, launch_part_0_2, launch_part_0_3,
     launch_part_0_4, launch_part_0_5, launch_part_0_6, launch_part_0_7},
    {launch_part_1_0, launch_part_1_1, launch_part_1_2, launch_part_1_3,
     launch_part_1_4, launch_part_1_5, launch_part_1_6, launch_part_1_7},
    {launch_part_2_0, launch_part_2_1, launch_part_2_2, launch_part_2_3,
     launch_part_2_4, launch_part_2_5, launch_part_2_6, launch_part_2_7},
    {launch_part_3_0, launch_part_3_1, launch_part_3_2, launch_part_3_3,
     launch_part_3_4, launch_part_3_5, launch_part_3_6, launch_part_3_7}};
// the small kernel, [PREC_S, PREC_D][case]
static const part_fn kSmall[2][8] = {
    {launch_small_0_0, launch_small_0_1, launch_small_0_2, launch_small_0_3,
     launch_small_0_4, launch_small_0_5, launch_small_0_6, launch_small_0_7},
    {launch_small_1_0, launch_small_1_1, launch_small_1_2, launch_small_1_3,
     launch_small_1_4, launch_small_1_5, launch_small_1_6, launch_small_1_7}};

// C := beta*C (alpha == 0 or k == 0).  beta == 0 writes zeros without reading C.
__global__ __launch_bounds__(256) void md_scale_kernel(GemmArgs g) {
    const int64_t total = g.m * g.n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t % g.m, j = t / g.m;
        const int64_t off = i * g.rsc + j * g.ldc;
        if (g.c_half) {
            // beta is already binary16: a product of two binary16 values is
            // exact in float; a sum of two is rounded to odd in float, then
            // once to binary16 (one rounding)
            _Float16 *c = (_Float16 *)g.C + (g.c_cplx ? 2 * off : off);
            const _Float16 *cin = (const _Float16 *)g.Cin + (g.c_cplx ? 2 * off : off);
            if (g.beta_zero) {
                c[0] = (_Float16)0.0f;
                if (g.c_cplx) c[1] = (_Float16)0.0f;
            } else if (g.c_cplx) {
                const float br = (float)g.beta_re, bi = (float)g.beta_im, cr = (float)cin[0], ci = (float)cin[1];
                c[0] = (_Float16)add_rto(br * cr, -(bi * ci));
                c[1] = (_Float16)add_rto(br * ci, bi * cr);
            } else {
                c[0] = (_Float16)((float)g.beta_re * (float)cin[0]);
            }
        } else if (g.c_cplx) {
            if (g.c_dbl) {
                double *c = (double *)g.C + 2 * off;
                const double *cin = (const double *)g.Cin + 2 * off;
                if (g.beta_zero) { c[0] = 0.0; c[1] = 0.0; }
                else {
                    const double br = g.beta_re, bi = g.beta_im, cr = cin[0], ci = cin[1];
                    c[0] = fma(br, cr, -(bi * ci));
                    c[1] = fma(br, ci, bi * cr);
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


// Sum of the split partial products of C(i, j) in split order, then the
// epilogue of the unsplit kernels (alpha, beta, one rounding to C's type).
template <class T>
__global__ __launch_bounds__(256) void md_split_reduce(GemmArgs g) {
    const int64_t total = g.m * g.n, stride = 2 * total;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t % g.m, j = t / g.m;
        const T *p = (const T *)g.part + 2 * t;
        T re = 0, im = 0;
        for (int s = 0; s < g.splits; ++s) {
            re += p[s * stride];
            im += p[s * stride + 1];
        }
        if (g.c_cplx) update_cplx<T, true, true>(g, i, j, re, im);
        else update_real<T, true, true>(g, i, j, re);
    }
}

static int g_cu_count = 0;
static int cu_count() {
    if (g_cu_count == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        g_cu_count = v;
    }
    return g_cu_count;
}

// k split for the FP32/FP64 kernels when the tiles cannot fill the device:
// fewer tiles than half the CUs, at least 4 k-tiles per split (2: measured
// slower at 256), at most 16.
static int split_count(int prec, int cs, const GemmArgs &a, int64_t tiles) {
    static const bool enabled = [] {
        const char *e = getenv("MDGEMM_SPLITK");  // "0": never split
        return !(e && e[0] == '0');
    }();
    if (!enabled || (prec != PREC_S && prec != PREC_D)) return 1;
    const int cus = cu_count();
    if (tiles * 2 > cus) return 1;
    int bm, bn, bk;
    tile_shape(prec, cs, a.a_vec && a.b_vec, &bm, &bn, &bk);
    const int64_t k_real = a.k * (lower_case(cs).kdbl ? 2 : 1);
    const int64_t nk = (k_real + bk - 1) / bk;
    int64_t s = (cus + tiles - 1) / tiles;
    if (s > nk / 4) s = nk / 4;
    if (s > 16) s = 16;
    return s > 1 ? (int)s : 1;
}

// Split workspaces: one per (device, stream), grown on demand and kept for the
// life of the process (at most about 100 MB each: S x tiles <= CUs + tiles
// workgroup tiles of partial (re, im) pairs).  Work on one stream runs in
// order, so products that share a workspace never overlap on the device, as
// long as each product's two launches (split kernel, reduction) are enqueued
// back to back: the caller holds g_ws_mu from taking the workspace until both
// are enqueued, so two host threads on one stream cannot interleave them.
// Growth frees the old buffer in stream order (after the work already
// enqueued, which includes every earlier user's reduction).
static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, std::pair<void *, size_t>> g_ws;
static void *split_workspace_locked(hipStream_t s, size_t bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    auto &e = g_ws[std::make_pair(dev, s)];
    if (e.first && e.second >= bytes) return e.first;
    void *p = nullptr;
    if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (e.first) (void)hipFreeAsync(e.first, s);
    e.first = p;
    e.second = bytes;
    return p;
}

// Launch the product kernel and, for a split product, the reduction that
// finishes it (a.part must hold a.splits x m x n partial pairs).
static void enqueue_product(int prec, int cs, const GemmArgs &a, hipStream_t s, int64_t tiles) {
    kParts[prec][cs](a, s, (unsigned)(tiles * a.splits));
    if (a.splits > 1) {
        const int64_t total = a.m * a.n;
        int64_t blocks = (total + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        if (prec == PREC_D) hipLaunchKernelGGL(md_split_reduce<double>, dim3((unsigned)blocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL(md_split_reduce<float>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    }
}

int launch_gemm(int prec, int cs, const GemmArgs &a0, void *stream, int64_t *wg, bool may_split) {
    const int64_t n = (int64_t)a0.tiles_m * a0.tiles_n;
    if (wg) *wg = n;
    if (n <= 0) return 0;
    if (prec < PREC_S || prec > PREC_H || cs < 0 || cs > 7) return MD_ERR_UNSUPPORTED;
    if (a0.small) return launch_small(prec, cs, a0, stream);
    hipStream_t s = (hipStream_t)stream;
    GemmArgs a = a0;
    if (a0.packed) {
        // packing takes a workspace: only where the caller allows allocation
        const int rc = may_split ? launch_packed(cs, a0, stream) : MD_ERR_BUDGET;
        if (rc != MD_ERR_BUDGET) return rc;
        // no workspace: the unpacked kernel on its own tiles
        int bm, bn, bk;
        tile_shape(prec, cs, a0.a_vec && a0.b_vec, &bm, &bn, &bk);
        const Lowering L = lower_case(cs);
        const int64_t tmn_a = bm / (L.mdbl ? 2 : 1), tmn_b = bn / (L.ndbl ? 2 : 1);
        a.packed = 0;
        a.tiles_m = (int)((a0.m + tmn_a - 1) / tmn_a);
        a.tiles_n = (int)((a0.n + tmn_b - 1) / tmn_b);
        if (wg) *wg = (int64_t)a.tiles_m * a.tiles_n;
        enqueue_product(prec, cs, a, s, (int64_t)a.tiles_m * a.tiles_n);
        return hipGetLastError() == hipSuccess ? 0 : MD_ERR_HIP;
    }
    a.splits = may_split ? split_count(prec, cs, a0, n) : 1;
    a.part = nullptr;
    if (a.splits > 1) {
        const size_t esz = prec == PREC_D ? sizeof(double) : sizeof(float);
        const size_t bytes = (size_t)a.splits * (size_t)a.m * (size_t)a.n * 2 * esz;
        std::lock_guard<std::mutex> lk(g_ws_mu);
        // the stream's workspace; without it the product runs unsplit
        a.part = split_workspace_locked(s, bytes);
        if (!a.part) a.splits = 1;
        enqueue_product(prec, cs, a, s, n);
    } else {
        enqueue_product(prec, cs, a, s, n);
    }
    return hipGetLastError() == hipSuccess ? 0 : MD_ERR_HIP;
}

// One workgroup per 32 x 32 tile of the real product (md_small.h).
int launch_small(int prec, int cs, const GemmArgs &a, void *stream) {
    const int64_t n = (int64_t)a.tiles_m * a.tiles_n;
    if (n <= 0) return 0;
    if (prec != PREC_S && prec != PREC_D) return MD_ERR_UNSUPPORTED;
    kSmall[prec][cs](a, (hipStream_t)stream, (unsigned)n);
    return hipGetLastError() == hipSuccess ? 0 : MD_ERR_HIP;
}

int launch_scale(const GemmArgs &a, void *stream) {
    const int64_t total = a.m * a.n;
    if (total <= 0) return 0;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(md_scale_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? 0 : MD_ERR_HIP;
}

void tile_shape(int prec, int cs, bool fast, int *bm, int *bn, int *bk) {
    const int kind = tile_kind(prec, cs, fast);
    *bm = (kind == 2 || kind == 4) ? 256 : 128;
    *bn = (kind == 1 || kind == 4) ? 256 : 128;
    *bk = prec == PREC_D ? 16 : 32;  // BF16x3 and half: one 16x16x32 step per tile
}

void kernel_name(int prec, int cs, const GemmArgs &a, char *out, int len) {
    static const char *cases[8] = {"0", "1a", "1b", "1c", "2ab", "2ac", "2bc", "3"};
    static const char *tiles[5] = {"t128x128w4", "t128x256w8", "t256x128w8", "t128x128w8", "t256x256w8"};
    const int kind = tile_kind(prec, cs, a.a_vec && a.b_vec);
    snprintf(out, len, "md_gemm_%s_case%s_%s_%c%c_%s",
             prec == PREC_D ? "f64" : prec == PREC_S ? "f32" : prec == PREC_H ? "f16" : "bf16x3",
             (cs >= 0 && cs < 8) ? cases[cs] : "?",
             a.small ? "small" : a.packed ? "packed" : (a.a_vec && a.b_vec) ? ((a.a_ragged || a.b_ragged) ? "ragged" : "fast") : "generic",
             a.a_dbl ? 'd' : (a.a_half ? 'h' : 's'), a.b_dbl ? 'd' : (a.b_half ? 'h' : 's'),
             a.small ? "t32x32w8" : a.packed ? "t256x256w8" : tiles[kind]);
}

}  // namespace md
