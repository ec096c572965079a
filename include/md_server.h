/*
 * md_server.h -- a request loop that serves mixed-datatype GEMMs (mdgemm.h)
 * as they arrive, with continuous batching under an HBM budget.
 *
 * This serving layer is an addition of this library; the product each request
 * computes is mdgemm's (Van Zee, Parikh, van de Geijn, Section 1 operation,
 * Figure "mixeddom" cases, Section 7 scalars), written out of place: the
 * output C := beta*C_in + alpha*op(A)*op(B) goes to fresh device memory and
 * the input C_in is only read, so one resident C_in can serve many requests.
 *
 * Model:
 *   - Operands live on the device.  md_server_put uploads a host matrix once
 *     and returns a handle; the matrix stays resident until md_server_drop.
 *   - A request names its A, B (and optional input C) by handle.  It is
 *     validated at submission (invalid requests are refused, the server keeps
 *     serving) and queued.
 *   - Classes: a request with more than `big_flops` algorithmic flops is
 *     "large" and runs alone with the plain kernels (mdgemm); smaller ones are
 *     gathered into grouped launches (mdgemm_grouped), up to `max_batch`
 *     requests each.  A request takes the same path whatever else is in
 *     flight, and its tiles do not depend on the rest of its batch, so its
 *     result is the same alone and in a mix.
 *   - Admission: each class is served in arrival order.  Whenever a stream
 *     slot is free, the oldest large request is admitted first if fewer than
 *     `big_lanes` large requests are running; otherwise the oldest small
 *     requests are gathered into a batch.  A request is admitted only while
 *     the in-flight working set (A, B, input C and output C of every admitted,
 *     unfinished request) stays within the budget; a large request that has a
 *     lane but waits for budget holds back every small request that arrived
 *     after it, so no request waits for budget forever.  A request larger
 *     than the whole budget is refused at submission with MD_ERR_BUDGET.
 *   - Concurrency: each slot is its own stream, so the batches of different
 *     slots overlap on the device while new requests keep being admitted.
 *     Completion is observed through one event per batch.
 *   - Memory: outputs come from the server's own device allocator (size
 *     classes, blocks recycled once the batch that used them has completed),
 *     so admission does no device allocation in steady state.  Each output is
 *     either kept as an operand handle (keep_output = 1; read it with
 *     md_server_fetch) or recycled on completion.  Large requests run on
 *     mdgemm's kernels, so the per-stream split-k and BF16x3 packing
 *     workspaces of mdgemm.h (allocated on first need, grown, kept) apply to
 *     the server's streams too; they are outside budget_bytes.
 *
 * All functions return 0 or a positive MD_ERR_* code (mdgemm.h), or a
 * negative argument position for md_server_submit (mdgemm's numbering).
 * Calls are thread-safe.
 */
#ifndef MD_SERVER_H
#define MD_SERVER_H

#include <stdint.h>

#include "mdgemm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct md_server md_server;

typedef struct {
    int64_t budget_bytes;  /* cap on the in-flight working set (> 0) */
    int slots;             /* concurrent batches = streams (>= 1) */
    int max_batch;         /* requests per grouped launch (>= 1) */
    double big_flops;      /* requests above this run alone on the plain kernels */
    int big_lanes;         /* large requests running at once (1 <= big_lanes <= slots) */
} md_server_config;

typedef struct {
    char transa, transb;
    int64_t m, n, k;
    md_scalar alpha;
    int64_t a, b;       /* operand handles of A and B (layouts as in mdgemm, ld = rows) */
    md_scalar beta;
    int64_t c_in;       /* operand handle of the input C (m x n of type dtc; read when beta != 0); -1: none (beta must be 0) */
    md_dt dtc;          /* storage type of the output C (m x n, ld = m) */
    md_comp comp;
    int keep_output;    /* 1: keep C as an operand handle; 0: recycle it on completion */
} md_request;

typedef struct {
    int status;          /* 0 or an MD_ERR_* code of the launch */
    int done;            /* 1 once the product has completed on the device */
    double t_submit_us;  /* host clock (microseconds since server creation) */
    double t_admit_us;
    double t_done_us;    /* when the scheduler observed completion */
    int64_t output;      /* operand handle of C if kept, else -1 */
    int batch_size;      /* requests in the launch that carried this one */
    double flops;        /* algorithmic flops (Figure "mixeddom") */
} md_result;

typedef struct {
    int64_t submitted, refused, admitted, completed;
    int64_t batches, grouped_launches, plain_launches;
    int64_t inflight_bytes, peak_inflight_bytes, budget_bytes;
    int64_t resident_bytes;   /* operands held by md_server_put / kept outputs */
    int64_t pool_bytes;       /* device memory held by the server's allocator (in use + cached) */
    int64_t device_mallocs;   /* hipMalloc calls made by the allocator */
    int max_concurrent_batches;
} md_server_counters;

/* Start a server on the current HIP device (MD_ERR_STATE for an invalid
 * configuration, MD_ERR_HIP if the device refuses streams or events). */
int md_server_create(const md_server_config *cfg, md_server **out);
/* Waits for every admitted request, then frees all device memory. */
int md_server_destroy(md_server *s);

/* Upload a column-major host matrix (rows x cols, ld = rows) of type dt. */
int md_server_put(md_server *s, const void *host, md_dt dt, int64_t rows, int64_t cols, int64_t *handle);
/* Release an operand (refused with MD_ERR_STATE while a queued or running request uses it). */
int md_server_drop(md_server *s, int64_t handle);
/* Copy an operand to host memory (synchronous). */
int md_server_fetch(md_server *s, int64_t handle, void *host);

/* Queue a request; *ticket identifies it.  Never blocks on the device. */
int md_server_submit(md_server *s, const md_request *req, int64_t *ticket);
/* Current state of a request (out->done says whether it finished). */
int md_server_poll(md_server *s, int64_t ticket, md_result *out);
/* Block until the request finishes or timeout_s passes (MD_ERR_STATE on timeout). */
int md_server_wait(md_server *s, int64_t ticket, md_result *out, double timeout_s);
/* Forget a finished request's record. */
int md_server_forget(md_server *s, int64_t ticket);
int md_server_stats(md_server *s, md_server_counters *out);

#ifdef __cplusplus
}
#endif
#endif
