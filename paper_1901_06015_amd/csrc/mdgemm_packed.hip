// mdgemm_packed.hip -- BF16x3 on packed operands (md_pack.h): the packing
// workspace and the three launches (pack A', pack B', multiply).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "md_internal.h"
#include "md_pack.h"

namespace md {

// Packing workspace: one per (device, stream), grown on demand and kept
// until the process ends.  Work on one stream runs in order, so products
// sharing it never overlap on the device, provided each product's three
// launches are enqueued back to back: the lock is held from taking the
// workspace until they are.  Growth frees the old buffer in stream order.
static std::mutex g_pk_mu;
static std::map<std::pair<int, hipStream_t>, std::pair<void *, size_t>> g_pk;

static void *pack_workspace_locked(hipStream_t s, size_t bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    auto &e = g_pk[std::make_pair(dev, s)];
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

template <int CS, bool AD, bool AMNC, bool BD>
static void enqueue_pack_b(const GemmArgs &a, hipStream_t s, char *pa, char *pb, int nkb, unsigned na, unsigned nb) {
    const bool bmnc = a.tb == 1 || a.tb == 2;
    if (bmnc)
        hipLaunchKernelGGL((md_pack_x3_kernel<CS, AD, AMNC, BD, true>), dim3(na + nb), dim3(PK_ROWS), 0, s, a, pa, pb,
                           nkb, na);
    else
        hipLaunchKernelGGL((md_pack_x3_kernel<CS, AD, AMNC, BD, false>), dim3(na + nb), dim3(PK_ROWS), 0, s, a, pa, pb,
                           nkb, na);
}

template <int CS, bool AD, bool AMNC>
static void enqueue_pack_a(const GemmArgs &a, hipStream_t s, char *pa, char *pb, int nkb, unsigned na, unsigned nb) {
    if (a.b_dbl) enqueue_pack_b<CS, AD, AMNC, true>(a, s, pa, pb, nkb, na, nb);
    else enqueue_pack_b<CS, AD, AMNC, false>(a, s, pa, pb, nkb, na, nb);
}

template <int CS>
static void enqueue_packed(const GemmArgs &a, hipStream_t s, char *pa, char *pb, int nkb) {
    const unsigned na = (unsigned)((int64_t)a.tiles_m * nkb), nb = (unsigned)((int64_t)a.tiles_n * nkb);
    const bool amnc = a.ta == 0 || a.ta == 3;
    if (a.a_dbl) {
        if (amnc) enqueue_pack_a<CS, true, true>(a, s, pa, pb, nkb, na, nb);
        else enqueue_pack_a<CS, true, false>(a, s, pa, pb, nkb, na, nb);
    } else {
        if (amnc) enqueue_pack_a<CS, false, true>(a, s, pa, pb, nkb, na, nb);
        else enqueue_pack_a<CS, false, false>(a, s, pa, pb, nkb, na, nb);
    }
    hipLaunchKernelGGL((md_packed_x3_kernel<CS>), dim3((unsigned)((int64_t)a.tiles_m * a.tiles_n)), dim3(PX_NT), 0,
                       s, a, (const char *)pa, (const char *)pb, nkb);
}

// Returns MD_OK, MD_ERR_HIP, or MD_ERR_BUDGET when the workspace could not be
// had (nothing enqueued; the caller runs the unpacked kernel instead).
int launch_packed(int cs, const GemmArgs &a, void *stream) {
    const int64_t kr = a.k * (lower_case(cs).kdbl ? 2 : 1);
    const int64_t nkb64 = (kr + PK_K - 1) / PK_K;
    const size_t blocks = (size_t)(a.tiles_m + a.tiles_n) * (size_t)nkb64;
    if (nkb64 > 0x7fffffff || (int64_t)(a.tiles_m + a.tiles_n) * nkb64 > 0x7fffffff) return MD_ERR_BUDGET;
    const size_t bytes = blocks * 2 * PK_BLOCK;
    if (bytes > PACK_MAX_BYTES) return MD_ERR_BUDGET;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_pk_mu);
    char *ws = (char *)pack_workspace_locked(s, bytes);
    if (!ws) return MD_ERR_BUDGET;
    char *pa = ws, *pb = ws + (size_t)a.tiles_m * (size_t)nkb64 * 2 * PK_BLOCK;
    const int nkb = (int)nkb64;
    switch (cs) {
        case 0: enqueue_packed<0>(a, s, pa, pb, nkb); break;
        case 1: enqueue_packed<1>(a, s, pa, pb, nkb); break;
        case 2: enqueue_packed<2>(a, s, pa, pb, nkb); break;
        case 3: enqueue_packed<3>(a, s, pa, pb, nkb); break;
        case 4: enqueue_packed<4>(a, s, pa, pb, nkb); break;
        case 5: enqueue_packed<5>(a, s, pa, pb, nkb); break;
        case 6: enqueue_packed<6>(a, s, pa, pb, nkb); break;
        case 7: enqueue_packed<7>(a, s, pa, pb, nkb); break;
        default: return MD_ERR_UNSUPPORTED;
    }
    return hipGetLastError() == hipSuccess ? MD_OK : MD_ERR_HIP;
}

}  // namespace md
