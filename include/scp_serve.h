/*
 * scp_serve.h - continuous-batching server of planning requests on one MI355X (gfx950), on top
 * of the persistent SCP + consensus-ADMM kernel of scp.h (arXiv 2603.10711).
 *
 * A request is a problem description (scp_problem_desc), typically one robust-MPC query: S
 * scenarios of one vehicle forming one consensus group on the first control (Sec. IV-A.4).
 * The server keeps one device pool (caller-allocated arena, as in scp.h) holding the nominal
 * trajectory, ADMM primal/dual/consensus state and per-trajectory records of every resident
 * request.  Scheduling is iteration-level: every scp_server_step() admits queued requests whose
 * footprint fits the HBM budget and the pool, then launches ONE persistent kernel that advances
 * every running request by `scp_per_step` SCP iterations, whatever the request's horizon and
 * model.  A request that arrives while others run joins at the next SCP boundary; finished
 * requests leave at the end of their last step and their results are copied to host memory.
 *
 * Warm start (MPC): a request submitted with a session id >= 0 whose previous request of the
 * same session is finished and still resident (same model, horizon and scenario count) starts
 * from that solution shifted by one node, in place on the device: states, controls and duals
 * move one node earlier (the last node repeated), node-0 duals of the dynamic coupling are
 * cleared, and every scenario's x_init becomes the previous scenario-0 state at node 1.
 * Requests of one session run one after the other, in submission order.
 *
 * All calls are host-thread-compatible per server (one thread at a time) and never throw.
 * Numerical failures are per-trajectory status bits in the returned info records.
 */
#ifndef SCP_SERVE_H
#define SCP_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "scp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    scp_precision prec;       /* arithmetic of every request                               */
    int32_t block;            /* persistent workgroup size for every request: 64, 128, 256  */
    int32_t pack;             /* scp_pack                                                    */
    int64_t max_nodes;        /* node capacity of the pool (sum of S (N+1) over residents)   */
    int32_t max_traj;         /* trajectory capacity                                         */
    int32_t max_wg;           /* workgroup capacity (lane tables of resident requests)       */
    int32_t max_span;         /* consensus groups spanning several workgroups, resident      */
    int32_t max_requests;     /* requests resident at once (running or kept for warm start)  */
    size_t budget_bytes;      /* admission limit: summed footprint of resident requests      */
    scp_params solve;         /* per-request budget (form is ignored: always persistent)     */
    int32_t scp_per_step;     /* SCP iterations per scheduling step; must divide
                                 solve.scp_iters (1 = admission at every SCP boundary)       */
    int32_t max_inflight;     /* scheduling steps enqueued ahead of the device, >= 1         */
    double timeout_ms;        /* > 0: a request still queued, or still running, this long after
                                 its submission ends without a result (SCP_REQ_TIMEOUT) at the
                                 next scheduling step and frees its place; 0: no limit        */
} scp_server_config;

typedef struct scp_server scp_server;

typedef enum {
    SCP_REQ_UNKNOWN = 0,      /* no such id, or already collected                         */
    SCP_REQ_QUEUED = 1,       /* waiting for admission                                    */
    SCP_REQ_RUNNING = 2,      /* resident, SCP iterations in progress                     */
    SCP_REQ_DONE = 3,         /* finished; results ready for scp_server_collect            */
    SCP_REQ_CANCELLED = 4,    /* ended by scp_server_cancel, no result                     */
    SCP_REQ_TIMEOUT = 5       /* ended by the configured timeout, no result                */
} scp_req_state;

typedef struct {
    int64_t submitted, completed, rejected;   /* counts since create                    */
    int32_t queued, running, resident;        /* current                                */
    int64_t steps;                            /* kernel launches                        */
    int64_t evictions;                        /* warm states dropped for lack of room   */
    int64_t warm_starts;                      /* requests started from a session state  */
    size_t resident_bytes;                    /* summed footprint of resident requests  */
    size_t peak_resident_bytes;
    int64_t cancelled, timed_out;             /* requests ended without a result        */
    double latency_ms_p50, latency_ms_p99;    /* over every completed request: submission
                                                 to the host observing its completion
                                                 (nearest-rank quantiles; 0 if none)    */
    double solves_per_s;                      /* completed requests per second from the
                                                 first submission to the last completion */
    double latency_ms_p999;                   /* as latency_ms_p50, the 99.9 % quantile  */
} scp_server_stats;

/* Arena bytes the configuration needs (0 if invalid).  Pure host computation. */
size_t scp_server_device_bytes(const scp_server_config* cfg);

/* Create a server on the caller's arena (>= scp_server_device_bytes, 256-byte aligned) and
 * hip stream (every launch and copy goes there).  Allocates pinned host staging buffers
 * (hipHostMalloc); never calls hipMalloc.  Errors: SCP_ERR_ARG, SCP_ERR_HIP, SCP_ERR_NOMEM. */
scp_status scp_server_create(const scp_server_config* cfg, void* arena_dev, size_t arena_bytes, void* hip_stream,
                             scp_server** out);

/* Waits for the server's device work, then releases host resources; never frees the arena. */
void scp_server_destroy(scp_server* s);

/* Footprint in bytes of a request in this server's pool (what admission charges against
 * budget_bytes); 0 if the request is invalid or can never fit. */
size_t scp_server_request_bytes(const scp_server* s, const scp_problem_desc* req);

/* Queue a request (its description is copied).  session >= 0 names an MPC session for warm
 * starts, -1 none.  Errors: SCP_ERR_ARG (invalid, or larger than the pool or the budget, or
 * a trajectory of the 6-DOF quadrotor model, which the persistent kernel does not run). */
scp_status scp_server_submit(scp_server* s, const scp_problem_desc* req, int32_t session, int64_t* id);

/* Submission flags. */
enum {
    /* Closed-loop MPC (Sec. IV-A.4, the controller applies the shared first control to the
     * plant): a warm start keeps the request's own x_init (the measured state) instead of the
     * previous scenario-0 state at node 1; the shifted trajectory and duals still seed the solve.
     * No effect on a cold start. */
    SCP_SUBMIT_MEASURED = 1
};

/* scp_server_submit with flags (SCP_SUBMIT_*); scp_server_submit is flags = 0.  Unknown flag
 * bits: SCP_ERR_ARG. */
scp_status scp_server_submit_ex(scp_server* s, const scp_problem_desc* req, int32_t session, uint32_t flags,
                                int64_t* id);

/* One scheduling step: collect finished device work, admit what fits, and launch one step of
 * the running requests if fewer than max_inflight steps are pending.  Blocks only when
 * max_inflight steps are pending and `wait` is nonzero.  *pending (optional) = requests
 * queued or running after the call. */
scp_status scp_server_step(scp_server* s, int32_t wait, int32_t* pending);

/* State of a request; for SCP_REQ_DONE also its latency (submission to the host observing its
 * completion, in ms) and its host results: info (n_traj * SCP_INFO_FIELDS doubles), x (rows
 * of SCP_MAX_NX, N+1 per trajectory) and u (rows of SCP_MAX_NU, N per trajectory), as doubles;
 * any pointer may be NULL.  For SCP_REQ_CANCELLED and SCP_REQ_TIMEOUT the latency is the time
 * to its end and there are no results.  `release` = 1 drops the record afterwards (the warm
 * state stays resident for the session); the id is then SCP_REQ_UNKNOWN. */
scp_status scp_server_collect(scp_server* s, int64_t id, int32_t release, int32_t* state, double* latency_ms,
                              double* info, double* x, double* u);

/* Cancel a queued or running request: a queued one ends at once, a running one at the next
 * scheduling step (its place in the pool is freed; with a session, the session's warm state goes
 * with it), one whose results are already being copied when they arrive (they are discarded).
 * Its state becomes SCP_REQ_CANCELLED.  Errors: SCP_ERR_STATE (unknown id, or already ended). */
scp_status scp_server_cancel(scp_server* s, int64_t id);

/* Ids of requests that ended (done, cancelled, timed out) since the last call, oldest first, at
 * most cap of them (the rest stay for the next call); *n = number written.  Lets a client
 * collect only the requests that changed instead of polling every pending id. */
scp_status scp_server_take_done(scp_server* s, int64_t* ids, int32_t cap, int32_t* n);

scp_status scp_server_get_stats(const scp_server* s, scp_server_stats* out);

/* Last error message of the server ("" if none); for s == NULL, the last create error. */
const char* scp_server_last_error(const scp_server* s);

#ifdef __cplusplus
}
#endif
#endif /* SCP_SERVE_H */
