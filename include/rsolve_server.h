/*
 * rsolve_server.h -- serving loop over many independent solve sequences on one GPU.
 *
 * A server owns a device memory pool (the caller's buffer) from which each admitted sequence's
 * workspace is carved.  Sequences arrive and leave at any time; each keeps its recycle basis W,
 * A W, snapshot ring and Krylov storage on the device between its solves (the state that
 * Algorithm 1 of section 5.2 carries from one time step to the next).  Solves are submitted
 * asynchronously and completed by worker threads:
 *   - sequences within the one-block limits of rsolve.h share one batch worker, which launches
 *     every queued solve of such sequences together (rsolve_solve_batch) and then their recycle
 *     updates (rsolve_update_recycle_batch); requests that arrive while a launch runs join the
 *     next one (continuous batching);
 *   - larger sequences are spread over `large_workers` threads, each with its own HIP stream,
 *     so their kernels overlap on the device; each runs rsolve_solve then rsolve_update_recycle.
 * The solves of one sequence run in submission order.  Every result is the one the sequence
 * would get alone: items never share device memory and the one-block kernel of an item does
 * not depend on its neighbours.
 *
 * Conventions as in rsolve.h: device pointers, caller-owned buffers, int status codes, no
 * aborts.  All calls may come from any host thread; the server serialises them internally.
 */
#ifndef RSOLVE_SERVER_H
#define RSOLVE_SERVER_H

#include <stddef.h>
#include <stdint.h>

#include "rsolve.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsolve_server rsolve_server;

typedef struct {
    void*   pool;            /* device buffer for the sequences' workspaces, 256-byte aligned */
    size_t  pool_bytes;      /* its size: the HBM budget of admission */
    int32_t large_workers;   /* worker threads (one HIP stream each) for large sequences, 1..64 */
    int32_t max_batch;       /* most one-block solves per launch, 1..256 */
    int32_t max_sequences;   /* most sequences admitted at once (slots), >= 1 */
    int32_t small_fp64;      /* 1: a sequence within the one-block limits whose configuration asks
                                for FP32_IR runs in FP64 on the batched path (latency-bound sizes
                                gain nothing from the narrower type); 0: it keeps FP32_IR and runs
                                on a large worker */
} rsolve_server_config;

typedef struct {
    uint64_t tag;            /* the submit call's tag */
    uint64_t seq_id;
    int32_t status;          /* rsolve_solve's status for this request (or the update's, if the
                                solve succeeded and the update failed) */
    int32_t batched;         /* 1 if the solve ran on the batched one-block path */
    rsolve_stats stats;
    double t_latency_ms;     /* submit to completion (host clock) */
    double t_queue_ms;       /* submit to the start of its solve */
} rsolve_completion;

typedef struct {
    size_t pool_used;        /* bytes of the pool held by admitted sequences */
    size_t pool_largest_free;
    int32_t sequences;       /* admitted and not closed */
    int32_t pending;         /* submitted and not yet completed */
    int64_t completed;       /* completions produced so far */
    int64_t batches;         /* batched launches so far */
    int64_t batched_solves;  /* solves that ran in them */
} rsolve_server_info;

/*
 * Start a server on the HIP device current on the calling thread.  Errors: E_INVALID (bad
 * configuration, misaligned pool), E_DEVICE (stream creation).
 */
int rsolve_server_create(const rsolve_server_config* cfg, rsolve_server** out);

/*
 * Admit a sequence (configuration, size and the largest nnz it will see): its workspace,
 * rsolve_workspace_bytes(cfg, n, nnz_max) bytes, is taken from the pool.  E_BUDGET when the
 * pool has no free block that large or every slot is taken (nothing changes; try again after
 * a close), E_INVALID for a bad configuration, E_DEVICE.
 */
int rsolve_server_open(rsolve_server* srv, const rsolve_config* cfg, int64_t n, int64_t nnz_max,
                       uint64_t* seq_id);

/*
 * Queue one time step of a sequence: rsolve_solve(A, b, x0, x, tol) then
 * rsolve_update_recycle(x).  Returns at once.  `ready_event` (a hipEvent_t, nullable) is waited
 * on by the device before the solve reads A, b or x0 (record it after the work that produces
 * them, and do not record it again until this request has completed).  A, b, x0 and x must stay
 * valid until the completion is returned by rsolve_server_poll.  Errors: E_INVALID (unknown or
 * closing sequence, bad arguments); solve errors arrive in the completion.
 */
int rsolve_server_submit(rsolve_server* srv, uint64_t seq_id, const rsolve_csr* A, const double* b,
                         const double* x0, double* x, double tol, void* ready_event, uint64_t tag);

/*
 * Move up to `cap` completions to `out` (host array), *count = how many.  Waits up to
 * `timeout_ms` (0: do not wait) for the first one when none is ready.
 */
int rsolve_server_poll(rsolve_server* srv, rsolve_completion* out, int32_t cap, int32_t* count,
                       int32_t timeout_ms);

/* Release a sequence whose requests have all completed (E_STATE otherwise); its workspace
 * returns to the pool. */
int rsolve_server_close(rsolve_server* srv, uint64_t seq_id);

int rsolve_server_info_get(rsolve_server* srv, rsolve_server_info* info);

/* Finish every queued request, stop the workers, destroy the remaining sequences. */
int rsolve_server_destroy(rsolve_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* RSOLVE_SERVER_H */
