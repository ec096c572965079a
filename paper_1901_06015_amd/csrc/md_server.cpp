// md_server.cpp -- request loop with continuous batching under an HBM budget
// (include/md_server.h).  One scheduler thread owns all device work: it
// retires finished batches (event queries), admits queued requests in arrival
// order while a slot and budget are free, and launches each batch on its
// slot's stream.  Clients only touch the queue and the result records.
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/md_server.h"
#include "md_internal.h"

namespace {

int elem_bytes(int dt) { return dt == MD_S ? 4 : (dt == MD_Z ? 16 : 8); }

struct Operand {
    void *ptr = nullptr;
    int dt = 0;
    int64_t rows = 0, cols = 0;
    int64_t bytes = 0;
    int users = 0;  // queued or running requests that read it
};

struct Req {
    md_request r;
    int64_t id = 0;
    int64_t ws = 0;  // working-set bytes: A + B + output C
    double flops = 0;
    bool big = false;
    md_result res{};
    void *out = nullptr;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Req *> batch;
    bool busy = false;
};

}  // namespace

struct md_server {
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Req *> pending;
    std::unordered_map<int64_t, Req *> reqs;
    std::unordered_map<int64_t, Operand> ops;
    std::vector<Slot> slots;
    std::thread sched;
    bool stop = false;
    int device = 0;
    int64_t budget = 0, inflight = 0, peak = 0, resident = 0;
    int max_batch = 1;
    double big_flops = 0;
    int64_t next_id = 1, next_handle = 1;
    md_server_counters st{};
    std::chrono::steady_clock::time_point t0;

    double now_us() const {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    }
    void run();
    void retire_locked();
    void admit_locked();
    void launch_locked(Slot &sl);
};

void md_server::retire_locked() {
    for (auto &sl : slots) {
        if (!sl.busy) continue;
        if (hipEventQuery(sl.done) != hipSuccess) continue;
        const double t = now_us();
        for (Req *q : sl.batch) {
            q->res.done = 1;
            q->res.t_done_us = t;
            inflight -= q->ws;
            for (int64_t h : {q->r.a, q->r.b, q->r.c_in}) {
                auto it = ops.find(h);
                if (it != ops.end()) it->second.users--;
            }
            if (q->res.status == MD_OK && q->r.keep_output) {
                Operand o;
                o.ptr = q->out;
                o.dt = q->r.dtc;
                o.rows = q->r.m;
                o.cols = q->r.n;
                o.bytes = q->r.m * q->r.n * elem_bytes(q->r.dtc);
                const int64_t h = next_handle++;
                ops[h] = o;
                resident += o.bytes;
                q->res.output = h;
            } else if (q->out) {
                (void)hipFreeAsync(q->out, sl.stream);
            }
            q->out = nullptr;
            st.completed++;
        }
        sl.batch.clear();
        sl.busy = false;
    }
    cv_done.notify_all();
}

void md_server::launch_locked(Slot &sl) {
    const double t = now_us();
    std::vector<md_gemm_desc> descs;
    int err = MD_OK;
    for (Req *q : sl.batch) {
        q->res.t_admit_us = t;
        q->res.batch_size = (int)sl.batch.size();
        const int64_t cb = q->r.m * q->r.n * elem_bytes(q->r.dtc);
        if (hipMallocAsync(&q->out, cb > 0 ? cb : 1, sl.stream) != hipSuccess) {
            q->out = nullptr;
            q->res.status = MD_ERR_HIP;
            err = MD_ERR_HIP;
            continue;
        }
        const bool use_c = (q->r.beta.re != 0.0 || q->r.beta.im != 0.0) && q->r.c_in >= 0;
        if (use_c) {
            const Operand &c = ops[q->r.c_in];
            if (hipMemcpyAsync(q->out, c.ptr, cb, hipMemcpyDeviceToDevice, sl.stream) != hipSuccess) {
                q->res.status = MD_ERR_HIP;
                err = MD_ERR_HIP;
                continue;
            }
        }
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
    }
    if (err == MD_OK) {
        int rc;
        if (sl.batch.size() == 1 && sl.batch[0]->big) {
            const md_gemm_desc &d = descs[0];
            rc = mdgemm(d.transa, d.transb, d.m, d.n, d.k, d.alpha, d.A, d.dta, d.lda, d.B, d.dtb, d.ldb, d.beta,
                        d.C, d.dtc, d.ldc, d.comp, sl.stream);
            st.plain_launches++;
        } else {
            rc = mdgemm_grouped((int64_t)descs.size(), descs.data(), sl.stream);
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
        if (sl.busy || pending.empty()) continue;
        // take requests in arrival order while they fit the budget; a large
        // request runs alone
        while (!pending.empty() && (int)sl.batch.size() < max_batch) {
            Req *q = pending.front();
            if (inflight + q->ws > budget) break;
            if (q->big && !sl.batch.empty()) break;
            pending.pop_front();
            inflight += q->ws;
            if (inflight > peak) peak = inflight;
            sl.batch.push_back(q);
            st.admitted++;
            if (q->big) break;
        }
        if (sl.batch.empty()) break;  // the head does not fit: wait for completions
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
        if (stop && !busy && pending.empty()) break;
        if (busy) {
            // device work in flight: poll its events at a fine interval
            cv_sched.wait_for(lk, std::chrono::microseconds(20));
        } else {
            cv_sched.wait(lk, [&] { return stop || !pending.empty(); });
        }
    }
}

extern "C" {

int md_server_create(int64_t budget_bytes, int slots, int max_batch, double big_flops, md_server **out) {
    if (!out) return MD_ERR_STATE;
    *out = nullptr;
    if (budget_bytes <= 0 || slots <= 0 || max_batch <= 0) return MD_ERR_STATE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MD_ERR_HIP;
    md_server *s = new md_server();
    s->device = dev;
    s->budget = budget_bytes;
    s->max_batch = max_batch;
    s->big_flops = big_flops;
    s->t0 = std::chrono::steady_clock::now();
    s->slots.resize(slots);
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
    s->st.budget_bytes = budget_bytes;
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
    for (auto &sl : s->slots) {
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.stream);
    }
    delete s;
    return MD_OK;
}

int md_server_put(md_server *s, const void *host, md_dt dt, int64_t rows, int64_t cols, int64_t *handle) {
    if (!s || !handle || !host || rows < 0 || cols < 0 || dt < MD_S || dt > MD_Z) return MD_ERR_STATE;
    Operand o;
    o.dt = dt;
    o.rows = rows;
    o.cols = cols;
    o.bytes = rows * cols * elem_bytes(dt);
    if (hipMalloc(&o.ptr, o.bytes > 0 ? o.bytes : 1) != hipSuccess) return MD_ERR_HIP;
    if (o.bytes > 0 && hipMemcpy(o.ptr, host, o.bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(o.ptr);
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
    void *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->ops.find(handle);
        if (it == s->ops.end() || it->second.users > 0) return MD_ERR_STATE;
        p = it->second.ptr;
        s->resident -= it->second.bytes;
        s->ops.erase(it);
    }
    (void)hipFree(p);
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
    }
    if (o.bytes > 0 && hipMemcpy(host, o.ptr, o.bytes, hipMemcpyDeviceToHost) != hipSuccess) return MD_ERR_HIP;
    return MD_OK;
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
    const int64_t arows = (r->transa == 'N' || r->transa == 'n') ? r->m : r->k;
    const int64_t acols = (r->transa == 'N' || r->transa == 'n') ? r->k : r->m;
    const int64_t brows = (r->transb == 'N' || r->transb == 'n') ? r->k : r->n;
    const int64_t bcols = (r->transb == 'N' || r->transb == 'n') ? r->n : r->k;
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
    q->ws = A.bytes + B.bytes + r->m * r->n * elem_bytes(r->dtc);
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
    s->pending.push_back(q);
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
    return MD_OK;
}

}  // extern "C"
