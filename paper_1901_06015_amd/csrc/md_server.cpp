// md_server.cpp -- request loop with continuous batching under an HBM budget
// (include/md_server.h).  One scheduler thread owns all device work: it
// retires finished batches (event queries), admits queued requests while a
// slot and budget are free, and launches each batch on its slot's stream.
// Clients only touch the queues, the operand table and the result records.
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/md_server.h"
#include "md_internal.h"

namespace {

int elem_bytes(int dt) { return dt == MD_H ? 2 : (dt == MD_S || dt == MD_HC) ? 4 : (dt == MD_Z ? 16 : 8); }

// Size class of a device block: 4 KiB minimum, then four classes per power of
// two, so a block wastes less than a quarter of its size.
int64_t size_class(int64_t b) {
    if (b <= 4096) return 4096;
    const int e = 63 - __builtin_clzll((unsigned long long)(b - 1));  // 2^e < b <= 2^(e+1)
    const int64_t step = (int64_t)1 << (e - 2);
    return (b + step - 1) / step * step;
}

// Device allocator of the server: free lists per size class.  A block comes
// back to its list only when no queued or running request can touch it (the
// scheduler returns outputs after their batch's event has completed), so it
// can be handed out again at once.  The cache is trimmed when it holds more
// than `limit` bytes.
class DevicePool {
  public:
    explicit DevicePool(int64_t limit) : limit_(limit) {}

    void *get(int64_t bytes, int64_t *cls) {
        const int64_t c = size_class(bytes);
        *cls = c;
        auto it = free_.find(c);
        if (it != free_.end() && !it->second.empty()) {
            void *p = it->second.back();
            it->second.pop_back();
            cached_ -= c;
            return p;
        }
        void *p = nullptr;
        if (hipMalloc(&p, (size_t)c) != hipSuccess) {
            // release the cache and try once more
            trim(0);
            if (hipMalloc(&p, (size_t)c) != hipSuccess) return nullptr;
        }
        held_ += c;
        mallocs_++;
        return p;
    }

    void put(void *p, int64_t cls) {
        if (!p) return;
        free_[cls].push_back(p);
        cached_ += cls;
        if (cached_ > limit_) trim(limit_ / 2);
    }

    void release_all() { trim(0); }

    int64_t held() const { return held_; }
    int64_t mallocs() const { return mallocs_; }

  private:
    void trim(int64_t keep) {
        // largest classes first
        for (auto it = free_.rbegin(); it != free_.rend() && cached_ > keep; ++it) {
            while (!it->second.empty() && cached_ > keep) {
                (void)hipFree(it->second.back());
                it->second.pop_back();
                cached_ -= it->first;
                held_ -= it->first;
            }
        }
    }

    std::map<int64_t, std::vector<void *>> free_;
    int64_t limit_, cached_ = 0, held_ = 0, mallocs_ = 0;
};

struct Operand {
    void *ptr = nullptr;
    int64_t cls = 0;  // allocator size class of ptr
    int dt = 0;
    int64_t rows = 0, cols = 0;
    int64_t bytes = 0;
    int users = 0;  // queued or running requests (and fetches) that read it
};

struct Req {
    md_request r;
    int64_t id = 0;
    int64_t ws = 0;  // working-set bytes: A + B + input C + output C
    double flops = 0;
    bool big = false;
    md_result res{};
    void *out = nullptr;
    int64_t out_cls = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Req *> batch;
    md::GroupedWs ws;
    bool busy = false;
    bool big = false;
};

}  // namespace

struct md_server {
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Req *> smallq, bigq;
    std::unordered_map<int64_t, Req *> reqs;
    std::unordered_map<int64_t, Operand> ops;
    std::vector<Slot> slots;
    std::thread sched;
    bool stop = false;
    int device = 0;
    int64_t budget = 0, inflight = 0, peak = 0, resident = 0;
    int max_batch = 1, big_lanes = 1, big_running = 0;
    double big_flops = 0;
    int64_t next_id = 1, next_handle = 1;
    md_server_counters st{};
    DevicePool pool;
    std::vector<md_gemm_desc> descs;
    std::vector<const void *> cins;
    std::chrono::steady_clock::time_point t0;

    explicit md_server(int64_t budget_bytes) : pool(budget_bytes) {}

    double now_us() const {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    }
    void run();
    void retire_locked();
    void admit_locked();
    void launch_locked(Slot &sl);
};

void md_server::retire_locked() {
    bool any = false;
    for (auto &sl : slots) {
        if (!sl.busy) continue;
        if (hipEventQuery(sl.done) != hipSuccess) continue;
        any = true;
        const double t = now_us();
        for (Req *q : sl.batch) {
            q->res.done = 1;
            q->res.t_done_us = t;
            inflight -= q->ws;
            for (int64_t h : {q->r.a, q->r.b, q->r.c_in}) {
                auto it = ops.find(h);
                if (it != ops.end()) it->second.users--;
            }
            if (q->res.status == MD_OK && q->r.keep_output && q->out) {
                Operand o;
                o.ptr = q->out;
                o.cls = q->out_cls;
                o.dt = q->r.dtc;
                o.rows = q->r.m;
                o.cols = q->r.n;
                o.bytes = q->r.m * q->r.n * elem_bytes(q->r.dtc);
                const int64_t h = next_handle++;
                ops[h] = o;
                resident += o.bytes;
                q->res.output = h;
            } else {
                pool.put(q->out, q->out_cls);
            }
            q->out = nullptr;
            st.completed++;
        }
        if (sl.big) big_running--;
        sl.batch.clear();
        sl.busy = false;
        sl.big = false;
    }
    if (any) cv_done.notify_all();
}

void md_server::launch_locked(Slot &sl) {
    const double t = now_us();
    descs.clear();
    cins.clear();
    int err = MD_OK;
    for (Req *q : sl.batch) {
        q->res.t_admit_us = t;
        q->res.batch_size = (int)sl.batch.size();
        const int64_t cb = q->r.m * q->r.n * elem_bytes(q->r.dtc);
        q->out = pool.get(cb > 0 ? cb : 1, &q->out_cls);
        if (!q->out) {
            q->res.status = MD_ERR_HIP;
            err = MD_ERR_HIP;
            continue;
        }
        const bool use_c = (q->r.beta.re != 0.0 || q->r.beta.im != 0.0) && q->r.c_in >= 0;
        const Operand &A = ops[q->r.a], &B = ops[q->r.b];
        md_gemm_desc d;
        d.transa = q->r.transa;
        d.transb = q->r.transb;
        d.m = q->r.m;
        d.n = q->r.n;
        d.k = q->r.k;
        d.alpha = q->r.alpha;
        d.A = A.ptr;
        d.dta = (md_dt)A.dt;
        d.lda = A.rows > 0 ? A.rows : 1;
        d.B = B.ptr;
        d.dtb = (md_dt)B.dt;
        d.ldb = B.rows > 0 ? B.rows : 1;
        d.beta = use_c ? q->r.beta : md_scalar{0.0, 0.0};
        d.C = q->out;
        d.dtc = q->r.dtc;
        d.ldc = q->r.m > 0 ? q->r.m : 1;
        d.comp = q->r.comp;
        descs.push_back(d);
        // beta*C is read from the resident input, the result written to the fresh output
        cins.push_back(use_c ? ops[q->r.c_in].ptr : nullptr);
    }
    if (err == MD_OK) {
        int rc;
        if (sl.big) {
            rc = md::gemm_enqueue(descs[0], cins[0], sl.stream);
            st.plain_launches++;
        } else {
            rc = md::grouped_enqueue((int64_t)descs.size(), descs.data(), cins.data(), sl.stream, &sl.ws);
            st.grouped_launches++;
        }
        if (rc != MD_OK)
            for (Req *q : sl.batch) q->res.status = rc;
    }
    (void)hipEventRecord(sl.done, sl.stream);
    sl.busy = true;
    st.batches++;
    int busy = 0;
    for (auto &s2 : slots) busy += s2.busy;
    if (busy > st.max_concurrent_batches) st.max_concurrent_batches = busy;
}

void md_server::admit_locked() {
    for (auto &sl : slots) {
        if (sl.busy) continue;
        if (smallq.empty() && bigq.empty()) break;
        auto take = [&](Req *q) {
            inflight += q->ws;
            if (inflight > peak) peak = inflight;
            sl.batch.push_back(q);
            st.admitted++;
        };
        // the oldest large request first, when a lane is free
        int64_t held_back = INT64_MAX;  // small requests that arrived after this id wait
        if (!bigq.empty() && big_running < big_lanes) {
            Req *q = bigq.front();
            if (inflight + q->ws <= budget) {
                bigq.pop_front();
                take(q);
                sl.big = true;
                big_running++;
                launch_locked(sl);
                continue;
            }
            held_back = q->id;
        }
        while (!smallq.empty() && (int)sl.batch.size() < max_batch) {
            Req *q = smallq.front();
            if (q->id > held_back || inflight + q->ws > budget) break;
            smallq.pop_front();
            take(q);
        }
        if (sl.batch.empty()) break;  // nothing fits: wait for completions
        launch_locked(sl);
    }
}

void md_server::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        retire_locked();
        admit_locked();
        bool busy = false;
        for (auto &sl : slots) busy |= sl.busy;
        if (stop && !busy && smallq.empty() && bigq.empty()) break;
        if (busy) {
            // device work in flight: poll its events at a fine interval
            cv_sched.wait_for(lk, std::chrono::microseconds(20));
        } else {
            cv_sched.wait(lk, [&] { return stop || !smallq.empty() || !bigq.empty(); });
        }
    }
}

extern "C" {

int md_server_create(const md_server_config *cfg, md_server **out) {
    if (!out) return MD_ERR_STATE;
    *out = nullptr;
    if (!cfg || cfg->budget_bytes <= 0 || cfg->slots <= 0 || cfg->max_batch <= 0 || cfg->big_lanes < 1 ||
        cfg->big_lanes > cfg->slots)
        return MD_ERR_STATE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MD_ERR_HIP;
    md_server *s = new md_server(cfg->budget_bytes);
    s->device = dev;
    s->budget = cfg->budget_bytes;
    s->max_batch = cfg->max_batch;
    s->big_flops = cfg->big_flops;
    s->big_lanes = cfg->big_lanes;
    s->t0 = std::chrono::steady_clock::now();
    s->slots.resize(cfg->slots);
    for (auto &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            for (auto &x : s->slots) {
                if (x.stream) (void)hipStreamDestroy(x.stream);
                if (x.done) (void)hipEventDestroy(x.done);
            }
            delete s;
            return MD_ERR_HIP;
        }
    }
    s->st.budget_bytes = cfg->budget_bytes;
    s->sched = std::thread([s] { s->run(); });
    *out = s;
    return MD_OK;
}

int md_server_destroy(md_server *s) {
    if (!s) return MD_ERR_STATE;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_sched.notify_all();
    s->sched.join();
    for (auto &sl : s->slots) (void)hipStreamSynchronize(sl.stream);
    for (auto &kv : s->ops) (void)hipFree(kv.second.ptr);
    for (auto &kv : s->reqs) delete kv.second;
    s->pool.release_all();
    for (auto &sl : s->slots) {
        md::grouped_ws_release(&sl.ws);
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.stream);
    }
    delete s;
    return MD_OK;
}

int md_server_put(md_server *s, const void *host, md_dt dt, int64_t rows, int64_t cols, int64_t *handle) {
    if (!s || !handle || !host || rows < 0 || cols < 0 || dt < MD_S || dt > MD_HC) return MD_ERR_STATE;
    Operand o;
    o.dt = dt;
    o.rows = rows;
    o.cols = cols;
    o.bytes = rows * cols * elem_bytes(dt);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        o.ptr = s->pool.get(o.bytes > 0 ? o.bytes : 1, &o.cls);
    }
    if (!o.ptr) return MD_ERR_HIP;
    if (o.bytes > 0 && hipMemcpy(o.ptr, host, o.bytes, hipMemcpyHostToDevice) != hipSuccess) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->pool.put(o.ptr, o.cls);
        return MD_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    *handle = s->next_handle++;
    s->ops[*handle] = o;
    s->resident += o.bytes;
    return MD_OK;
}

int md_server_drop(md_server *s, int64_t handle) {
    if (!s) return MD_ERR_STATE;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->ops.find(handle);
    if (it == s->ops.end() || it->second.users > 0) return MD_ERR_STATE;
    s->resident -= it->second.bytes;
    s->pool.put(it->second.ptr, it->second.cls);
    s->ops.erase(it);
    return MD_OK;
}

int md_server_fetch(md_server *s, int64_t handle, void *host) {
    if (!s || !host) return MD_ERR_STATE;
    Operand o;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->ops.find(handle);
        if (it == s->ops.end()) return MD_ERR_STATE;
        o = it->second;
        it->second.users++;  // not dropped while the copy runs
    }
    const bool ok = o.bytes == 0 || hipMemcpy(host, o.ptr, o.bytes, hipMemcpyDeviceToHost) == hipSuccess;
    std::lock_guard<std::mutex> lk(s->mu);
    s->ops[handle].users--;
    return ok ? MD_OK : MD_ERR_HIP;
}

int md_server_submit(md_server *s, const md_request *r, int64_t *ticket) {
    if (!s || !r || !ticket) return MD_ERR_STATE;
    std::unique_lock<std::mutex> lk(s->mu);
    s->st.submitted++;
    auto fa = s->ops.find(r->a), fb = s->ops.find(r->b);
    const bool beta0 = r->beta.re == 0.0 && r->beta.im == 0.0;
    auto fc = s->ops.find(r->c_in);
    if (fa == s->ops.end() || fb == s->ops.end() || (!beta0 && fc == s->ops.end())) {
        s->st.refused++;
        return MD_ERR_STATE;
    }
    const Operand &A = fa->second, &B = fb->second;
    // the input C must be m x n of the output's type
    if (!beta0 && (fc->second.dt != r->dtc || fc->second.rows != r->m || fc->second.cols != r->n)) {
        s->st.refused++;
        return -14;
    }
    // validate exactly as mdgemm would (no device work)
    md_plan p;
    const int64_t lda = A.rows > 0 ? A.rows : 1, ldb = B.rows > 0 ? B.rows : 1, ldc = r->m > 0 ? r->m : 1;
    // op 'N'/'R' reads A as m x k (B as k x n), 'T'/'C' as its transpose
    const bool an = r->transa == 'N' || r->transa == 'n' || r->transa == 'R' || r->transa == 'r';
    const bool bn = r->transb == 'N' || r->transb == 'n' || r->transb == 'R' || r->transb == 'r';
    const int64_t arows = an ? r->m : r->k, acols = an ? r->k : r->m;
    const int64_t brows = bn ? r->k : r->n, bcols = bn ? r->n : r->k;
    if (A.rows != arows || A.cols != acols) {
        s->st.refused++;
        return -9;
    }
    if (B.rows != brows || B.cols != bcols) {
        s->st.refused++;
        return -12;
    }
    const int st = mdgemm_plan(r->transa, r->transb, r->m, r->n, r->k, r->alpha, A.ptr, (md_dt)A.dt, lda, B.ptr,
                               (md_dt)B.dt, ldb, beta0 ? md_scalar{0.0, 0.0} : r->beta, (void *)1, r->dtc, ldc,
                               r->comp, &p);
    if (st != MD_OK) {
        s->st.refused++;
        return st;
    }
    Req *q = new Req();
    q->r = *r;
    q->id = s->next_id++;
    q->flops = p.flops;
    q->big = p.flops > s->big_flops;
    const int64_t cb = r->m * r->n * elem_bytes(r->dtc);
    q->ws = A.bytes + B.bytes + cb + (beta0 ? 0 : cb);
    if (q->ws > s->budget) {
        s->st.refused++;
        delete q;
        return MD_ERR_BUDGET;
    }
    q->res.status = MD_OK;
    q->res.done = 0;
    q->res.output = -1;
    q->res.flops = p.flops;
    q->res.t_submit_us = s->now_us();
    for (int64_t h : {r->a, r->b, beta0 ? (int64_t)-1 : r->c_in}) {
        auto it = s->ops.find(h);
        if (it != s->ops.end()) it->second.users++;
    }
    if (beta0) q->r.c_in = -1;
    s->reqs[q->id] = q;
    (q->big ? s->bigq : s->smallq).push_back(q);
    *ticket = q->id;
    lk.unlock();
    s->cv_sched.notify_one();
    return MD_OK;
}

int md_server_poll(md_server *s, int64_t ticket, md_result *out) {
    if (!s || !out) return MD_ERR_STATE;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return MD_ERR_STATE;
    *out = it->second->res;
    return MD_OK;
}

int md_server_wait(md_server *s, int64_t ticket, md_result *out, double timeout_s) {
    if (!s || !out) return MD_ERR_STATE;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return MD_ERR_STATE;
    Req *q = it->second;
    const bool ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return q->res.done != 0; });
    *out = q->res;
    return ok ? MD_OK : MD_ERR_STATE;
}

int md_server_forget(md_server *s, int64_t ticket) {
    if (!s) return MD_ERR_STATE;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || !it->second->res.done) return MD_ERR_STATE;
    delete it->second;
    s->reqs.erase(it);
    return MD_OK;
}

int md_server_stats(md_server *s, md_server_counters *out) {
    if (!s || !out) return MD_ERR_STATE;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->inflight_bytes = s->inflight;
    out->peak_inflight_bytes = s->peak;
    out->resident_bytes = s->resident;
    out->budget_bytes = s->budget;
    out->pool_bytes = s->pool.held();
    out->device_mallocs = s->pool.mallocs();
    return MD_OK;
}

}  // extern "C"
