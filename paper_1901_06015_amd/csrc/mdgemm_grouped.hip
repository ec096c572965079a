// mdgemm_grouped.hip -- host side of mdgemm_grouped (work table, tile order,
// one persistent launch) and of the tile-shape table the autotuner writes.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "md_grouped.h"

namespace md {
namespace {

// Tile table: for (computation precision, domain case, size bucket of m',
// size bucket of n') the grouped kernel's tile configuration (GCFG_*).
// Buckets: <=64, <=128, <=256, <=512, larger.
constexpr int NBUCKET = MD_TUNE_BUCKETS;
int g_table[3][8][NBUCKET][NBUCKET];
std::mutex g_table_mu;
bool g_table_init = false;

// Built-in rule: per dimension a 64-wide tile up to 256, 128 above.
int default_cfg(int prec, int bm, int bn) {
    if (prec == PREC_BF16X3) return GCFG_64;
    const bool wm = bm > 2, wn = bn > 2;
    return wm ? (wn ? GCFG_128 : GCFG_128x64) : (wn ? GCFG_64x128 : GCFG_64);
}

void fill_defaults(int (&t)[3][8][NBUCKET][NBUCKET]) {
    for (int p = 0; p < 3; ++p)
        for (int c = 0; c < 8; ++c)
            for (int bm = 0; bm < NBUCKET; ++bm)
                for (int bn = 0; bn < NBUCKET; ++bn) t[p][c][bm][bn] = default_cfg(p, bm, bn);
}

void default_table() {
    fill_defaults(g_table);
    g_table_init = true;
}

int bucket_of(int64_t dim) {
    int b = 0;
    for (int64_t lim = 64; b < NBUCKET - 1 && dim > lim; lim *= 2) ++b;
    return b;
}

int choose_cfg(int prec, int cs, int64_t m_real, int64_t n_real) {
    if (prec == PREC_BF16X3) return GCFG_64;  // the only BF16x3 shape of the grouped kernel
    std::lock_guard<std::mutex> lk(g_table_mu);
    if (!g_table_init) default_table();
    return g_table[prec][cs][bucket_of(m_real)][bucket_of(n_real)];
}

int g_num_cu = 0;

// Upload staging of mdgemm_grouped, one per (device, stream): page-locked host
// memory and a device table, grown on demand and kept until the process ends.
// An event marks when the last upload from the host buffer has been read, so
// the next call on the stream waits for it (usually not at all) before
// writing the buffer again; the device table is only rewritten by a later
// upload on the same stream, after the kernel that read it.
struct UploadCache {
    char *host = nullptr;
    char *dev = nullptr;
    size_t cap = 0;
    hipEvent_t read = nullptr;
    bool pending = false;
};
std::mutex g_up_mu;
std::map<std::pair<int, hipStream_t>, UploadCache> g_up;

// The work table of mdgemm_grouped_noalloc: a fixed array that every GPU the
// library runs on holds until the process ends.  In host code the array's
// name only stands for it: the device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is
// passed to copies and kernels.  Every call on one GPU uses the same array,
// which keeps the last call's table.
static __device__ __align__(256) char scratch[MD_GROUPED_NOALLOC_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch[MAX_DEVICES];

// Device address of the current device's scratch, or nullptr.
char *scratch_of_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch[dev] = (char *)p;
    }
    return g_scratch[dev];
}

int num_cu() {
    if (g_num_cu == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        g_num_cu = v;
    }
    return g_num_cu;
}

}  // namespace
}  // namespace md

using namespace md;

namespace md {

int grouped_enqueue(int64_t count, const md_gemm_desc *descs, const void *const *c_in, void *stream,
                    GroupedWs *ws, bool noalloc) {
    if (count < 0) return -1;
    if (count == 0) return MD_OK;
    if (!descs) return -2;
    std::vector<GDesc> gd;
    std::vector<double> work;    // per product in gd: estimated cost of one of its tiles
    std::vector<int64_t> alone;  // products run by the plain kernels instead
    int64_t ntiles64 = 0;
    gd.reserve(count);
    work.reserve(count);
    for (int64_t i = 0; i < count; ++i) {
        const md_gemm_desc &x = descs[i];
        Decision d = decide(x.transa, x.transb, x.m, x.n, x.k, x.alpha, x.A, x.dta, x.lda, x.B, x.dtb, x.ldb,
                            x.beta, x.C, x.dtc, x.ldc, x.comp);
        if (d.status < 0) return -(int)(1000 * i + (-d.status));
        if (d.status != MD_OK) return d.status;
        if (d.quick == 1) continue;
        // the grouped kernel addresses an operand tile with 32-bit offsets:
        // 128 columns of 32 components of 16 bytes must span less than 2 GiB;
        // it also does not scale an operand while staging it (a complex alpha
        // under the literal interpretation with C real), read or write
        // binary16 storage, or compute in half precision
        if ((d.quick == 0 && (x.lda >= ((int64_t)1 << 20) || x.ldb >= ((int64_t)1 << 20) || d.g.a_scale ||
                              d.g.b_scale || d.g.a_half || d.g.b_half || d.prec == PREC_H)) ||
            d.g.c_half) {
            alone.push_back(i);
            continue;
        }
        GDesc e;
        memset(&e, 0, sizeof(e));
        e.g = d.g;
        if (c_in && c_in[i]) e.g.Cin = c_in[i];
        e.prec = d.prec;
        e.cs = d.cs;
        const Lowering L = lower_case(d.cs);
        if (d.quick == 2) {
            e.kind = 1;
            e.cfg = GCFG_64;
            e.tiles_m = (int)((x.m + 63) / 64);
            e.tiles_n = (int)((x.n + 63) / 64);
        } else {
            e.kind = 0;
            const int64_t mr = x.m * (L.mdbl ? 2 : 1), nr = x.n * (L.ndbl ? 2 : 1);
            e.cfg = choose_cfg(d.prec, d.cs, mr, nr);
            const int bm = gcfg_bm(e.cfg), bn = gcfg_bn(e.cfg);
            const int64_t tmn_a = L.mdbl ? bm / 2 : bm, tmn_b = L.ndbl ? bn / 2 : bn;
            e.tiles_m = (int)((x.m + tmn_a - 1) / tmn_a);
            e.tiles_n = (int)((x.n + tmn_b - 1) / tmn_b);
        }
        const int di = (int)gd.size();
        gd.push_back(e);
        // estimated cost of one tile: its real-product flops, weighted by the
        // computation precision's MFMA rate (FP64 is half FP32; BF16x3 ~1/2)
        const double area = e.kind == 1 ? 64.0 * 64.0 : (double)gcfg_bm(e.cfg) * gcfg_bn(e.cfg);
        const double kr = (double)x.k * (L.kdbl ? 2 : 1);
        const double w = e.kind == 1 ? area : area * kr * (d.prec == PREC_D ? 2.0 : (d.prec == PREC_S ? 1.0 : 0.5));
        work.push_back(w);
        ntiles64 += (int64_t)e.tiles_m * e.tiles_n;
        (void)di;
    }
    if (ntiles64 > 0x7fffffffLL) return MD_ERR_UNSUPPORTED;
    auto run_alone = [&]() {
        for (int64_t i : alone) {
            const int rc = gemm_enqueue(descs[i], c_in ? c_in[i] : nullptr, stream, !noalloc);
            if (rc != MD_OK) return rc;
        }
        return (int)MD_OK;
    };
    if (ntiles64 == 0) return run_alone();
    // Largest work first (LPT order) so the tail of the queue is short tiles.
    // All tiles of a product cost the same, so ordering the products (stably)
    // and listing each product's tiles in turn gives the tile order.
    std::vector<int> order(gd.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });

    const size_t ntiles_all = (size_t)ntiles64;
    const size_t hdr_bytes = 256;
    const size_t desc_bytes = gd.size() * sizeof(GDesc);
    const size_t tile_bytes = ntiles_all * sizeof(GTile);
    const size_t total = hdr_bytes + desc_bytes + tile_bytes;
    // the size is checked before any device call
    if (noalloc && total > MD_GROUPED_NOALLOC_BYTES) return MD_ERR_SCRATCH;
    hipStream_t s = (hipStream_t)stream;
    std::vector<char> tmp;
    char *host = nullptr, *dev = nullptr;
    std::unique_lock<std::mutex> up_lock(g_up_mu, std::defer_lock);
    UploadCache *up = nullptr;
    if (noalloc) {
        // the fixed array of this device; the host copy is consumed by the
        // upload before hipMemcpyAsync returns
        dev = scratch_of_current_device();
        if (!dev) return MD_ERR_HIP;
        tmp.resize(total);
        host = tmp.data();
    } else if (ws) {
        // grow the reusable staging: the launch that used it has completed
        if (ws->cap < total) {
            grouped_ws_release(ws);
            const size_t cap = std::max<size_t>(total + total / 2, 1 << 20);
            if (hipHostMalloc((void **)&ws->host, cap, hipHostMallocDefault) != hipSuccess) {
                ws->host = nullptr;
                return MD_ERR_HIP;
            }
            if (hipMalloc((void **)&ws->dev, cap) != hipSuccess) {
                (void)hipHostFree(ws->host);
                ws->host = nullptr;
                ws->dev = nullptr;
                return MD_ERR_HIP;
            }
            ws->cap = cap;
        }
        host = ws->host;
        dev = ws->dev;
    } else {
        int dv = 0;
        if (hipGetDevice(&dv) != hipSuccess) return MD_ERR_HIP;
        // held until the kernel is enqueued: host threads sharing a stream
        // take turns with the staging
        up_lock.lock();
        up = &g_up[std::make_pair(dv, s)];
        if (up->pending) {
            if (hipEventSynchronize(up->read) != hipSuccess) return MD_ERR_HIP;
            up->pending = false;
        }
        if (up->cap < total) {
            if (up->host) (void)hipHostFree(up->host);
            if (up->dev) (void)hipFreeAsync(up->dev, s);
            up->host = nullptr;
            up->dev = nullptr;
            up->cap = 0;
            const size_t cap = std::max<size_t>(total + total / 2, 1 << 20);
            if (hipHostMalloc((void **)&up->host, cap, hipHostMallocDefault) != hipSuccess) {
                up->host = nullptr;
                return MD_ERR_HIP;
            }
            if (hipMallocAsync((void **)&up->dev, cap, s) != hipSuccess) {
                (void)hipHostFree(up->host);
                up->host = nullptr;
                up->dev = nullptr;
                return MD_ERR_HIP;
            }
            up->cap = cap;
        }
        if (!up->read && hipEventCreateWithFlags(&up->read, hipEventDisableTiming) != hipSuccess) {
            up->read = nullptr;
            return MD_ERR_HIP;
        }
        host = up->host;
        dev = up->dev;
    }
    memset(host, 0, hdr_bytes);  // the tile-queue counter starts at zero
    memcpy(host + hdr_bytes, gd.data(), desc_bytes);
    GTile *ht = (GTile *)(host + hdr_bytes + desc_bytes);
    size_t nt = 0;
    for (int di : order)
        for (int tm = 0; tm < gd[di].tiles_m; ++tm)
            for (int tn = 0; tn < gd[di].tiles_n; ++tn) ht[nt++] = GTile{di, tm, tn, 0};
    if (hipMemcpyAsync(dev, host, total, hipMemcpyHostToDevice, s) != hipSuccess) return MD_ERR_HIP;
    if (up) {
        if (hipEventRecord(up->read, s) != hipSuccess) return MD_ERR_HIP;
        up->pending = true;
    }
    const int ntiles = (int)ntiles_all;
    const int grid = std::min(ntiles, num_cu() * GROUPED_OCC);
    launch_grouped_kernel(grid, s, (const GDesc *)(dev + hdr_bytes), (const GTile *)(dev + hdr_bytes + desc_bytes),
                          ntiles, (int *)dev);
    const hipError_t le = hipGetLastError();
    if (up_lock.owns_lock()) up_lock.unlock();
    if (le != hipSuccess) return MD_ERR_HIP;
    return run_alone();
}

void grouped_ws_release(GroupedWs *ws) {
    if (!ws) return;
    if (ws->host) (void)hipHostFree(ws->host);
    if (ws->dev) (void)hipFree(ws->dev);
    ws->host = nullptr;
    ws->dev = nullptr;
    ws->cap = 0;
}

}  // namespace md

extern "C" {

int mdgemm_grouped(int64_t count, const md_gemm_desc *descs, void *stream) {
    return md::grouped_enqueue(count, descs, nullptr, stream, nullptr);
}

int mdgemm_grouped_noalloc(int64_t count, const md_gemm_desc *descs, void *stream) {
    return md::grouped_enqueue(count, descs, nullptr, stream, nullptr, true);
}

// Tile table file: one entry per line, "comp case bucket_m bucket_n config"
// with comp in {s, d, bf16x3}, case in {0, 1a, 1b, 1c, 2ab, 2ac, 2bc, 3},
// buckets 0..4 and config one of the names below; '#' starts a comment.
// Entries not listed keep their default.
static const char *const kCfgNames[GCFG_COUNT] = {"64x64", "128x128", "128x64", "64x128", "64x64k"};

static int prec_of_comp(int comp) {
    return comp == MD_COMP_S ? PREC_S : comp == MD_COMP_D ? PREC_D : comp == MD_COMP_S_BF16X3 ? PREC_BF16X3 : -1;
}

static bool entry_ok(int p, int c, int bm, int bn, int cfg) {
    return p >= 0 && c >= 0 && c < 8 && bm >= 0 && bm < NBUCKET && bn >= 0 && bn < NBUCKET && cfg >= 0 &&
           cfg < GCFG_COUNT && (p != PREC_BF16X3 || cfg == GCFG_64);
}

int mdgemm_tune_load(const char *path) {
    std::lock_guard<std::mutex> lk(g_table_mu);
    if (!path) {
        default_table();
        return MD_OK;
    }
    FILE *f = fopen(path, "r");
    if (!f) return MD_ERR_STATE;
    static const char *cases[8] = {"0", "1a", "1b", "1c", "2ab", "2ac", "2bc", "3"};
    int tmp[3][8][NBUCKET][NBUCKET];
    fill_defaults(tmp);
    char line[256];
    int bad = 0;
    while (fgets(line, sizeof(line), f)) {
        char *h = strchr(line, '#');
        if (h) *h = 0;
        char comp[32], cs[32], cfgname[32];
        int bm, bn;
        if (sscanf(line, "%31s %31s %d %d %31s", comp, cs, &bm, &bn, cfgname) != 5) {
            if (sscanf(line, "%31s", comp) == 1) bad = 1;
            continue;
        }
        const int p = !strcmp(comp, "s") ? PREC_S : !strcmp(comp, "d") ? PREC_D
                    : !strcmp(comp, "bf16x3") ? PREC_BF16X3 : -1;
        int c = -1, cfg = -1;
        for (int i = 0; i < 8; ++i)
            if (!strcmp(cs, cases[i])) c = i;
        for (int i = 0; i < GCFG_COUNT; ++i)
            if (!strcmp(cfgname, kCfgNames[i])) cfg = i;
        if (!entry_ok(p, c, bm, bn, cfg)) {
            bad = 1;
            continue;
        }
        tmp[p][c][bm][bn] = cfg;
    }
    fclose(f);
    if (bad) return MD_ERR_STATE;
    memcpy(g_table, tmp, sizeof(tmp));
    g_table_init = true;
    return MD_OK;
}

int mdgemm_tune_set(int comp, int domain_case, int bucket_m, int bucket_n, int config) {
    std::lock_guard<std::mutex> lk(g_table_mu);
    if (!g_table_init) default_table();
    const int p = prec_of_comp(comp);
    if (!entry_ok(p, domain_case, bucket_m, bucket_n, config)) return MD_ERR_STATE;
    g_table[p][domain_case][bucket_m][bucket_n] = config;
    return MD_OK;
}

int mdgemm_tune_get(int comp, int domain_case, int bucket_m, int bucket_n) {
    std::lock_guard<std::mutex> lk(g_table_mu);
    if (!g_table_init) default_table();
    const int p = prec_of_comp(comp);
    if (!entry_ok(p, domain_case, bucket_m, bucket_n, 0)) return -1;
    return g_table[p][domain_case][bucket_m][bucket_n];
}

}  // extern "C"
